"""Benchmark: PCG DOFs/s to 1e-8 relative residual on one MI355X.

Workload (default): 3D CG Poisson -Laplace(u) = f on the unit cube, 16^3 hexes
with interior vertices perturbed by up to 10% of h (seed 1), p = 6 GLL
elements (N = 857,375 unknowns), f from u = prod sin(pi x_i); float64 PCG
preconditioned by LOR vertex-patch additive Schwarz (MDF-ILU(0) V-cycles,
exact coarse solve), x0 = 0, stop at ||r|| <= 1e-8 ||b||.

A step is one full solve from x0 = 0 (inputs resident in HBM); setup is done
once before the timed region and reported separately.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STATUS_NAMES = {0: "ok", -4: "breakdown", -5: "no_convergence", -9: "accuracy_floor"}


def patch_algorithmic_bytes(dim, n, p, prec_bytes=8):
    """Bytes one patch V-cycle launch must move: per (patch, smoothed level)
    row the 13 strict-lower IC(0) entries and the pivot (14 values), per
    global level row the 14 unique values of the symmetric Q1 stencil, and
    the residual gather plus the read-modify-write of the correction (3
    float64 per fine unknown)."""
    from paper_1908_07071_amd.lor import lor_gll  # noqa: F401  (library must exist)
    kept = _kept(p)
    sizes = [len(k) - 1 for k in kept]
    c = 14 if dim == 3 else 5
    rows = 0
    for k, s in enumerate(sizes[:-1]):
        per = []
        for v in range(n + 1):
            lo = (v - 1) * s + 1 if v > 0 else 1
            hi = (v + 1) * s - 1 if v < n else n * s - 1
            per.append(max(hi - lo + 1, 0))
        rows += sum(per) ** dim
    glob = sum((n * s - 1) ** dim for s in sizes)
    N = (n * p - 1) ** dim
    return prec_bytes * c * (rows + glob) + 8 * 3 * N


def apply_algorithmic_bytes(dim, n, p):
    """Operator launch: x read + y read-modify-write (16 B per unknown) and the
    6 (3 in 2D) float64 geometric factors per element node."""
    N = (n * p - 1) ** dim
    g = 48 if dim == 3 else 24
    return 16 * N + g * n ** dim * (p + 1) ** dim


def dg_apply_algorithmic_bytes(dim, n, p):
    """DG operator launch pair: x read and y written (16 B per E-vector node),
    the float64 geometric factors per node (48 B in 3D, 24 B in 2D) and the
    face geometry (omega, sigma and J^-1 n on both sides: 64 B per face
    node).  The face records passed from the face kernel to the element
    kernel are an intermediate of this design, not counted."""
    Q = p + 1
    N = n ** dim * Q ** dim
    g = 48 if dim == 3 else 24
    faces = dim * (n + 1) * n ** (dim - 1)
    return 16 * N + g * N + 64 * faces * Q ** (dim - 1)


def dg_measure(L, torch, dim, n, p, rtol, steps, precision):
    """Interior penalty and BR2 DG solves at the penalties 1.5 (p+1)^2 x
    {1, 10, 100, 1e4} on a perturbed n^dim mesh (seed 2)."""
    from paper_1908_07071_amd import inputs
    V = inputs.structured_vertices(dim, n, 0.1, seed=2)
    dev = torch.device("cuda:0")
    out = {"workload": (f"{dim}D IP and BR2 DG Poisson, {n}^{dim} hexes perturbed <=10% h (seed 2), "
                        f"p={p}, f from u=prod sin(pi x_i), flexible CG to {rtol:g}, preconditioner "
                        f"{'FP32 Schwarz part' if precision == 'mixed' else 'FP64'}"),
           "runs": []}
    for meth, code in (("ip", L.LOR_IP), ("br2", L.LOR_BR2)):
        for fac in (1, 10, 100, 1e4):
            eta = 1.5 * (p + 1) ** 2 * fac
            opt = L.lor_default_options()
            opt.precision = L.LOR_PREC_MIXED if precision == "mixed" else L.LOR_PREC_FP64
            h = L.lor_setup(dim, n, V, p, method=code, penalty=eta, options=opt)
            N = L.lor_ndofs(h)
            coords = L.lor_dof_coords(h, dim)
            f = torch.tensor(inputs.manufactured_f(coords), device=dev)
            b = torch.empty_like(f)
            L.lor_assemble_rhs(h, f, b)
            x = torch.zeros_like(b)
            info = L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=5000, check=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                info = L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=5000, check=False)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / steps
            run = {"method": meth, "eta": eta, "N": N, "iters": info.iters, "status": info.status,
                   "status_name": STATUS_NAMES.get(info.status, str(info.status)),
                   "rel_res_true": info.rel_res_true, "reached_rtol": info.rel_res_true <= rtol,
                   "replacements": info.replacements, "ms_per_solve": ms,
                   "dofs_per_s": N / (ms * 1e-3)}
            if fac == 1:
                xr = torch.tensor(inputs.uniform_vector(N, 3), device=dev)
                y = torch.empty_like(xr)
                for _ in range(5):
                    L.lor_apply_A(h, xr, y)
                L.lor_timing(h, True)
                for _ in range(100):
                    L.lor_apply_A(h, xr, y)
                tA, nA = L.lor_timing_read(h, L.LOR_T_APPLY_A)
                L.lor_timing(h, False)
                t_apply = tA / nA * 1e-3
                ab = dg_apply_algorithmic_bytes(dim, n, p)
                run["operator_ms"] = t_apply * 1e3
                run["operator_gdofs"] = N / t_apply / 1e9
                run["operator_algorithmic_bytes"] = ab
                run["operator_hbm_frac"] = ab / t_apply / (HBM_PEAK_GBS * 1e9)
            L.lor_free(h)
            print(f"[bench] DG {meth} eta={eta:g}: {ms:.2f} ms/solve, iters={info.iters}, "
                  f"rel_res_true={info.rel_res_true:.2e}, status={run['status_name']}, "
                  f"replacements={info.replacements}", file=sys.stderr, flush=True)
            out["runs"].append(run)
    return out


def batch_measure(L, torch, nprob, nrhs, rtol, precision, seed=7):
    """Batch of nprob independent 3D CG problems (n ~ U{4..24}, p ~ U{2..8},
    interior vertices perturbed <=10% h) with nrhs Gaussian right-hand sides
    each, solved by one lor_pcg_solve_batch call; the same pairs solved one
    after another with lor_pcg_solve give the reference time."""
    from paper_1908_07071_amd import inputs
    probs = inputs.batch_problems(nprob, seed)
    opt = L.lor_default_options()
    opt.precision = L.LOR_PREC_MIXED if precision == "mixed" else L.LOR_PREC_FP64
    hs, Ns, bs, xs = [], [], [], []
    t0 = time.perf_counter()
    for i, (n, p, ms) in enumerate(probs):
        V = inputs.structured_vertices(3, n, 0.1, seed=ms)
        hs.append(L.lor_setup(3, n, V, p, options=opt))
        N = L.lor_ndofs(hs[-1])
        Ns.append(N)
        for k in range(nrhs):
            bs.append(torch.tensor(inputs.gaussian_rhs(N, 1000 * i + k), device="cuda:0"))
            xs.append(torch.zeros_like(bs[-1]))
        print(f"[bench] batch problem {i}: n={n} p={p} N={N} set up", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    infos = L.lor_pcg_solve_batch(hs, bs, xs, rtol=rtol, maxit=2000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = L.lor_pcg_solve_batch(hs, bs, xs, rtol=rtol, maxit=2000)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print(f"[bench] batch solve {t_batch:.2f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    seq_iters = []
    for k in range(len(bs)):
        x1 = torch.zeros_like(bs[k])
        seq_iters.append(L.lor_pcg_solve(hs[k // nrhs], bs[k], x1, rtol=rtol, maxit=2000).iters)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    print(f"[bench] sequential solves {t_seq:.2f} s", file=sys.stderr, flush=True)
    tot = sum(Ns) * nrhs
    its = [inf.iters for inf in infos]
    worst = max(inf.rel_res_true for inf in infos)
    for h in hs:
        L.lor_free(h)
    return {
        "metric": "PCG DOFs/s to 1e-8 rel. residual, batch of independent problems (mixed/learned vs FP64)",
        "value": tot / t_batch, "unit": "DOF/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": t_batch * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32" if precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": (f"batch of {nprob} 3D CG problems, n^3 hexes n~U{{4..24}} perturbed <=10% h, "
                                f"p~U{{2..8}} (size seed {seed}), {nrhs} Gaussian right-hand sides each, "
                                f"one lor_pcg_solve_batch call (the right-hand sides of a problem in lockstep, "
                                f"their patch V-cycles in one launch per iteration, small problems "
                                f"sharing that launch up to 4 at a time; graph-captured "
                                f"8-iteration chunks on 4 streams), "
                                f"FCG to {rtol:g}"),
                   "problems": [[n, p] for n, p, _ in probs], "sum_N": sum(Ns), "pairs": len(bs),
                   "iters_min": min(its), "iters_max": max(its), "worst_rel_res_true": worst,
                   "setup_s": round(setup_s, 1)},
        "sequential_value": tot / t_seq, "sequential_ms": t_seq * 1e3,
        "speedup_vs_sequential": t_seq / t_batch,
    }


def learned_measure(L, torch, rtol, channels=32, train_seconds=90.0, n_test=32, p=6):
    """Learned patch correction: train the patch network on (patch residual,
    patch V-cycle) pairs the method generates on 16^3 meshes (seeds 10, 11;
    residuals of PCG iterates and Gaussian right-hand sides), evaluate it against
    the V-cycle on held-out patches, then solve on the n_test^3 test mesh
    (seed 3) with flexible CG to rtol: V-cycles (the plain fallback) against
    the network standing in for every patch V-cycle and against the network's
    prediction as the start of each patch V-cycle."""
    import numpy as np

    from paper_1908_07071_amd import inputs
    dev = torch.device("cuda:0")
    nparam = L.lor_nn_param_count(channels)
    params = inputs.nn_initial_params(channels, seed=11)
    Xs, Ts, Xv, Tv = [], [], None, None
    t0 = time.perf_counter()
    for ms in (10, 11):
        V = inputs.structured_vertices(3, 16, 0.1, seed=ms)
        h = L.lor_setup(3, 16, V, p)
        nn = L.lor_nn_create(h, channels, params, max_batch=64)
        J, G = L.lor_nn_shape(nn)
        N = L.lor_ndofs(h)
        b = torch.tensor(inputs.gaussian_rhs(N, 500 + ms), device=dev)
        x = torch.zeros_like(b)
        y = torch.empty_like(b)
        res = []
        for k in (1, 2, 3, 5, 8, 12, 20, 35):   # residuals of PCG iterates
            L.lor_pcg_solve(h, b, x, rtol=0.0, maxit=k, check=False)
            L.lor_apply_A(h, x, y)
            res.append(b - y)
        res += [torch.tensor(inputs.gaussian_rhs(N, 600 + ms * 10 + i), device=dev) for i in range(2)]
        for i, r in enumerate(res):
            X = torch.zeros((J, G ** 3, 2), dtype=torch.float32, device=dev)
            T = torch.zeros((J, G ** 3), dtype=torch.float32, device=dev)
            sc = torch.zeros(J, dtype=torch.float64, device=dev)
            L.lor_nn_patch_data(nn, r.contiguous(), X, T, sc)
            if ms == 11 and i == len(res) - 1:
                Xv, Tv = X, T          # held out
            else:
                Xs.append(X)
                Ts.append(T)
        L.lor_nn_free(nn)
        L.lor_free(h)
        print(f"[bench] learned: training data from mesh seed {ms}", file=sys.stderr, flush=True)
    Xall = torch.cat(Xs)
    Tall = torch.cat(Ts)
    npairs = Xall.shape[0]
    data_s = time.perf_counter() - t0
    # training on the 16^3 geometry's handle-free network: any handle with p=6 serves
    V = inputs.structured_vertices(3, 4, 0.1, seed=12)
    hsmall = L.lor_setup(3, 4, V, p)
    nn = L.lor_nn_create(hsmall, channels, params, max_batch=64)
    gen = torch.Generator(device="cpu").manual_seed(13)
    t0 = time.perf_counter()
    losses, steps = [], 0
    while time.perf_counter() - t0 < train_seconds:
        idx = torch.randperm(npairs, generator=gen)[:64].to(dev)
        Xb = Xall.index_select(0, idx).contiguous()
        Tb = Tall.index_select(0, idx).contiguous()
        lr = 1e-3 if steps < 2000 else 3e-4
        losses.append(L.lor_nn_train_step(nn, Xb, Tb, 64, lr))
        steps += 1
        if steps % 200 == 0:
            print(f"[bench] learned: step {steps} loss {np.mean(losses[-50:]):.4e}", file=sys.stderr, flush=True)
    train_s = time.perf_counter() - t0
    # evaluation: network against the V-cycle on held-out patches
    J, G = L.lor_nn_shape(nn)
    errs = []
    Y = torch.zeros((64, G ** 3), dtype=torch.float32, device=dev)
    for first in range(0, Xv.shape[0] - 63, 64):
        L.lor_nn_forward(nn, Xv[first:first + 64].contiguous(), 64, Y)
        t = Tv[first:first + 64]
        errs.append(((Y - t).norm() / t.norm()).item())
    trained = L.lor_nn_get_params(nn, channels)
    L.lor_nn_free(nn)
    L.lor_free(hsmall)
    # test solve
    V = inputs.structured_vertices(3, n_test, 0.1, seed=3)
    opt = L.lor_default_options()
    opt.precision = L.LOR_PREC_MIXED
    h = L.lor_setup(3, n_test, V, p, options=opt)
    N = L.lor_ndofs(h)
    f = torch.tensor(inputs.manufactured_f(L.lor_dof_coords(h, 3)), device=dev)
    b = torch.empty_like(f)
    L.lor_assemble_rhs(h, f, b)
    x = torch.zeros_like(b)
    out = {"channels": channels, "parameters": nparam, "training_pairs": int(npairs),
           "data_s": round(data_s, 1), "train_steps": steps, "train_s": round(train_s, 1),
           "loss_first50": float(np.mean(losses[:50])), "loss_last50": float(np.mean(losses[-50:])),
           "heldout_rel_error_vs_vcycle": float(np.mean(errs)), "test_N": N}
    L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=2000)
    torch.cuda.synchronize()
    tv = time.perf_counter() - t0
    out["vcycle"] = {"iters": info.iters, "s": tv, "dofs_per_s": N / tv, "rel_res_true": info.rel_res_true}
    print(f"[bench] learned: V-cycle FCG {info.iters} iters {tv:.2f} s", file=sys.stderr, flush=True)
    nn = L.lor_nn_create(h, channels, trained, max_batch=512)
    L.lor_nn_attach(h, nn, L.LOR_NN_REPLACE)
    maxit = 300
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=maxit, check=False)
    torch.cuda.synchronize()
    tn = time.perf_counter() - t0
    out["network_replace"] = {"iters": info.iters, "converged": info.status == L.LOR_OK, "s": tn,
                              "rel_res": info.rel_res, "rel_res_true": info.rel_res_true,
                              "s_per_iteration": tn / max(info.iters, 1), "maxit": maxit}
    print(f"[bench] learned: network FCG {info.iters} iters status {info.status} {tn:.2f} s "
          f"rel_res {info.rel_res:.2e}", file=sys.stderr, flush=True)
    # warm start: the network's prediction corrected by one V-cycle per patch
    L.lor_nn_attach(h, nn, L.LOR_NN_WARMSTART)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=maxit, check=False)
    torch.cuda.synchronize()
    tw = time.perf_counter() - t0
    out["network_warmstart"] = {"iters": info.iters, "converged": info.status == L.LOR_OK, "s": tw,
                                "rel_res": info.rel_res, "rel_res_true": info.rel_res_true,
                                "s_per_iteration": tw / max(info.iters, 1), "maxit": maxit}
    print(f"[bench] learned: warm-start FCG {info.iters} iters status {info.status} {tw:.2f} s "
          f"rel_res {info.rel_res:.2e}", file=sys.stderr, flush=True)
    L.lor_nn_attach(h, None, L.LOR_NN_OFF)
    L.lor_nn_free(nn)
    L.lor_free(h)
    return out


def nn_apply_measure(L, torch, n, p=6, channels=32, reps=3):
    """Milliseconds per preconditioner application at n^3, p: patch V-cycles,
    the network for every patch, and the network starting every V-cycle
    (untrained weights: the cost does not depend on them)."""
    from paper_1908_07071_amd import inputs
    V = inputs.structured_vertices(3, n, 0.1, seed=3)
    opt = L.lor_default_options()
    opt.precision = L.LOR_PREC_MIXED
    h = L.lor_setup(3, n, V, p, options=opt)
    N = L.lor_ndofs(h)
    nn = L.lor_nn_create(h, channels, inputs.nn_initial_params(channels, seed=11), max_batch=512)
    r = torch.tensor(inputs.gaussian_rhs(N, 1), device="cuda:0")
    z = torch.empty_like(r)
    out = {"workload": f"preconditioner application, 3D CG {n}^3 perturbed hexes (seed 3), p={p}",
           "N": N, "channels": channels}
    for name, mode in (("vcycle", L.LOR_NN_OFF), ("network_replace", L.LOR_NN_REPLACE),
                       ("network_warmstart", L.LOR_NN_WARMSTART)):
        L.lor_nn_attach(h, nn if mode != L.LOR_NN_OFF else None, mode)
        L.lor_apply_P(h, r, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            L.lor_apply_P(h, r, z)
        torch.cuda.synchronize()
        out[name + "_ms"] = (time.perf_counter() - t0) / reps * 1e3
        print(f"[bench] {name}: {out[name + '_ms']:.2f} ms per application", file=sys.stderr, flush=True)
    L.lor_nn_attach(h, None, L.LOR_NN_OFF)
    L.lor_nn_free(nn)
    L.lor_free(h)
    return out


def _kept(p):
    levels = [list(range(p + 1))]
    while len(levels[-1]) > 2:
        cur = levels[-1]
        inner = cur[1:-1]
        levels.append([0] + [inner[k] for k in range(len(inner)) if k % 2 == 1] + [p])
    return levels


def measured_traffic(kernel_key):
    """HBM bytes per launch of the FP32 patch kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE record (profiles/), or None when the
    kernel's sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "patch_vcycle_16cube_p6_fp32_traffic.json")
    if kernel_key != "patch_vcycle" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["sources_sha256"] else None


def cpu_baseline(dim, p, iters_full, budget_s=25.0):
    """Time the float64 oracle (setup excluded) on a 2^3-element sample of the
    same workload and scale to DOFs/s of the full solve."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import gll, highorder as HO, krylov, mesh as M, schwarz as S
    from paper_1908_07071_amd import inputs

    n = 2
    V = inputs.structured_vertices(dim, n, 0.1, seed=1)
    mesh = M.make_mesh(dim, n, V)
    with threadpool_limits(1):
        K = HO.cg_stiffness(mesh, p)
        x, _ = gll.gll(p)
        b = HO.cg_rhs(mesh, p, inputs.manufactured_f(M.global_node_coords(mesh, x, p)))
        B = S.SchwarzLOR(mesh, p)
        t0 = time.perf_counter()
        k = 0
        while True:
            k += 2
            t0 = time.perf_counter()
            krylov.pcg(K, b, B.apply, tol=0.0, maxit=k)
            dt = time.perf_counter() - t0
            if dt > 3.0 or k >= 8 or dt * 2 > budget_s:
                break
    t_iter = dt / k
    Ns = K.shape[0]
    value = Ns / (t_iter * iters_full)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": value, "unit": "DOF/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cpu_count": os.cpu_count(),
            "sample": (f"float64 NumPy/SciPy oracle, 1 thread: {k} PCG iterations on the same "
                       f"workload at 2^3 elements (N={Ns}), {t_iter * 1e3:.1f} ms/iteration; "
                       f"DOF/s = N_sample / (t_iter_sample * {iters_full} iterations of the full "
                       f"solve), i.e. per-iteration cost taken linear in N; setup excluded")}


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Measured HBM bandwidth of a plain device copy (read + write bytes per
    second), the practical ceiling beside the 8 TB/s specification."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def solve_timed(L, torch, h, b, x, rtol, steps, maxit=1000):
    """One untimed solve, then `steps` timed solves (host clock around
    synchronized solves).  Returns (info, ms per solve)."""
    info = L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=maxit, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=maxit, check=False)
    torch.cuda.synchronize()
    return info, 1e3 * (time.perf_counter() - t0) / steps


def p_sweep(L, torch, dim, n, degrees, rtol, steps):
    """Iterations and DOF/s against p on the benchmark mesh (seed 1): float64
    PCG and the float32-preconditioner flexible CG, f from the manufactured
    solution."""
    from paper_1908_07071_amd import inputs
    V = inputs.structured_vertices(dim, n, 0.1, seed=1)
    out = []
    for p in degrees:
        rec = {"p": p}
        for prec, code in (("fp64", L.LOR_PREC_FP64), ("mixed", L.LOR_PREC_MIXED)):
            opt = L.lor_default_options()
            opt.precision = code
            h = L.lor_setup(dim, n, V, p, options=opt)
            N = L.lor_ndofs(h)
            f = torch.tensor(inputs.manufactured_f(L.lor_dof_coords(h, dim)), device="cuda:0")
            b = torch.empty_like(f)
            L.lor_assemble_rhs(h, f, b)
            x = torch.zeros_like(b)
            info, ms = solve_timed(L, torch, h, b, x, rtol, steps)
            rec["N"] = N
            rec[prec] = {"iters": info.iters, "status": STATUS_NAMES.get(info.status, str(info.status)),
                         "rel_res_true": info.rel_res_true, "ms_per_solve": ms,
                         "dofs_per_s": N / (ms * 1e-3), "setup_s": info.t_setup}
            L.lor_free(h)
            del b, x, f
        print(f"[bench] p={p}: N={rec['N']} fp64 {rec['fp64']['iters']} it "
              f"{rec['fp64']['ms_per_solve']:.1f} ms, mixed {rec['mixed']['iters']} it "
              f"{rec['mixed']['ms_per_solve']:.1f} ms", file=sys.stderr, flush=True)
        out.append(rec)
    return out


def ordering_variants(L, torch, dim, n, p, rtol, steps, names):
    """The float32-preconditioner solve of the benchmark workload with other
    ILU(0) orderings: iterations, time per solve and per patch launch, and
    the dependency depth of the level-0 sweeps (the chain of steps a patch
    sweep must take one after another)."""
    import numpy as np

    from paper_1908_07071_amd import inputs
    V = inputs.structured_vertices(dim, n, 0.1, seed=1)
    codes = {"mdf": L.LOR_ORD_MDF, "natural": L.LOR_ORD_NATURAL}
    if hasattr(L, "LOR_ORD_RCM"):
        codes["rcm"] = L.LOR_ORD_RCM
    out = {}
    for name in names:
        if name not in codes:
            continue
        opt = L.lor_default_options()
        opt.precision = L.LOR_PREC_MIXED
        opt.ordering = codes[name]
        h = L.lor_setup(dim, n, V, p, options=opt)
        N = L.lor_ndofs(h)
        f = torch.tensor(inputs.manufactured_f(L.lor_dof_coords(h, dim)), device="cuda:0")
        b = torch.empty_like(f)
        L.lor_assemble_rhs(h, f, b)
        x = torch.zeros_like(b)
        L.lor_pcg_solve(h, b, x, rtol=rtol, maxit=1000, check=False)
        torch.cuda.synchronize()
        L.lor_timing(h, True)
        info, ms = solve_timed(L, torch, h, b, x, rtol, steps)
        tP, nP = L.lor_timing_read(h, L.LOR_T_PATCH)
        L.lor_timing(h, False)
        soff = L.lor_export_maps(h, L.LOR_MAP_SCHEDULE_OFFSET)
        nlev = len(L.lor_export_maps(h, L.LOR_MAP_ORDER_OFFSET)) - 1
        J = (n + 1) ** dim
        nf = nlev // J
        depth0 = np.diff(soff)[0::nf] - 1 if nf else np.zeros(0)
        out[name] = {"iters": info.iters, "status": STATUS_NAMES.get(info.status, str(info.status)),
                     "rel_res_true": info.rel_res_true, "ms_per_solve": ms,
                     "dofs_per_s": N / (ms * 1e-3), "patch_launch_ms": tP / max(nP, 1),
                     "level0_depth_max": int(depth0.max()) if len(depth0) else 0,
                     "level0_depth_mean": float(depth0.mean()) if len(depth0) else 0.0,
                     "setup_s": info.t_setup}
        print(f"[bench] ordering {name}: {info.iters} it, {ms:.2f} ms/solve, patch launch "
              f"{out[name]['patch_launch_ms']:.3f} ms, level-0 depth max {out[name]['level0_depth_max']}",
              file=sys.stderr, flush=True)
        L.lor_free(h)
    return out


def _solve_case(L, torch, dim, n, p, V, opt, rtol, steps, coef=None, rhs="manufactured"):
    from paper_1908_07071_amd import inputs
    h = L.lor_setup(dim, n, V, p, options=opt, coef=coef)
    N = L.lor_ndofs(h)
    if rhs == "manufactured":
        f = torch.tensor(inputs.manufactured_f(L.lor_dof_coords(h, dim)), device="cuda:0")
        b = torch.empty_like(f)
        L.lor_assemble_rhs(h, f, b)
    else:
        b = torch.tensor(inputs.gaussian_rhs(N, 5), device="cuda:0")
    x = torch.zeros_like(b)
    info, ms = solve_timed(L, torch, h, b, x, rtol, steps)
    L.lor_free(h)
    return {"N": N, "iters": info.iters, "status": STATUS_NAMES.get(info.status, str(info.status)),
            "rel_res_true": info.rel_res_true, "ms_per_solve": ms, "dofs_per_s": N / (ms * 1e-3),
            "setup_s": info.t_setup}


def single_patch_measure(L, torch, rtol):
    """B(1) (one patch, the whole domain, Section 4.1) against the vertex
    patches B(V): the 2D 8 x 8 p = 3 unit-square problem (float64 PCG to
    1e-10, f from sin(pi x) sin(pi y)) and the 16^3 p = 6 benchmark mesh
    (float64 PCG to rtol, reverse Cuthill-McKee order for both)."""
    from paper_1908_07071_amd import inputs
    out = {}
    V2 = inputs.structured_vertices(2, 8)
    for mode, code in (("single", L.LOR_PATCH_SINGLE), ("vertex", L.LOR_PATCH_VERTEX)):
        opt = L.lor_default_options()
        opt.patch_mode = code
        out[f"square_8x8_p3_{mode}"] = _solve_case(L, torch, 2, 8, 3, V2, opt, 1e-10, 3)
    V3 = inputs.structured_vertices(3, 16, 0.1, seed=1)
    for mode, code, ordname, ordcode in (("single", L.LOR_PATCH_SINGLE, "rcm", L.LOR_ORD_RCM),
                                         ("single", L.LOR_PATCH_SINGLE, "natural", L.LOR_ORD_NATURAL),
                                         ("vertex", L.LOR_PATCH_VERTEX, "rcm", L.LOR_ORD_RCM)):
        opt = L.lor_default_options()
        opt.patch_mode = code
        opt.ordering = ordcode
        rec = _solve_case(L, torch, 3, 16, 6, V3, opt, rtol, 1)
        if mode == "single":
            # dependency depth of the level-0 sweep over the whole domain
            h = L.lor_setup(3, 16, V3, 6, options=opt)
            soff = L.lor_export_maps(h, L.LOR_MAP_SCHEDULE_OFFSET)
            rec["level0_depth"] = int(soff[1] - soff[0] - 1)
            L.lor_free(h)
        out[f"cube_16_p6_{ordname}_{mode}"] = rec
    for k, v in out.items():
        print(f"[bench] {k}: {v['iters']} it, {v['ms_per_solve']:.2f} ms/solve, setup {v['setup_s']:.1f} s",
              file=sys.stderr, flush=True)
    return out


def strip_measure(L, torch, rtol, n=8, degrees=(3, 7), aspects=(1.5, 15.0, 150.0, 1500.0)):
    """Section 4.5 shape: a 2D n x n mesh with two strip rows of thin
    elements (aspect ratio A), float64 PCG to rtol, Gaussian right side:
    iterations of the plain vertex patches B(V), the isotropic-overlap
    patches, B(1), B(2) and B(3)."""
    from paper_1908_07071_amd import inputs
    modes = (("vertex", L.LOR_PATCH_VERTEX, 0), ("vertex_iso", L.LOR_PATCH_VERTEX_ISO, 0),
             ("single", L.LOR_PATCH_SINGLE, 0), ("slabs2", L.LOR_PATCH_SLABS, 2),
             ("slabs3", L.LOR_PATCH_SLABS, 3))
    out = {}
    for p in degrees:
        for A in aspects:
            V = inputs.strip_vertices(n, A)
            rec = {}
            for name, code, ns in modes:
                opt = L.lor_default_options()
                opt.patch_mode = code
                opt.nslabs = ns
                r = _solve_case(L, torch, 2, n, p, V, opt, rtol, 1, rhs="gaussian")
                rec[name] = {"iters": r["iters"], "status": r["status"], "ms_per_solve": r["ms_per_solve"]}
            out[f"p{p}_A{A:g}"] = rec
            print(f"[bench] strip p={p} A={A:g}: " +
                  ", ".join(f"{k} {v['iters']}" for k, v in rec.items()), file=sys.stderr, flush=True)
    return {"workload": f"2D {n}x{n} strip mesh (two rows of aspect A), float64 PCG to {rtol:g}, "
                        "Gaussian rhs", "iters": out}


def coefficient_measure(L, torch, rtol, n=16, p=4):
    """Iterations with the coefficients b1-b4 (Section 4.2 shapes) on a 2D
    n x n perturbed mesh at degree p, for B(1) and B(V), Gaussian right side."""
    import numpy as np

    from paper_1908_07071_amd import inputs
    V = inputs.structured_vertices(2, n, 0.1, seed=4)
    out = {}
    h0 = L.lor_setup(2, n, V, p)
    X = L.lor_element_coords(h0, 2, n * n, p)
    L.lor_free(h0)
    elem = np.repeat(np.arange(n * n), (p + 1) ** 2)
    for name in ("b1", "b2", "b3", "b4"):
        coef = inputs.coefficient(name, X, elem=elem, seed=3)
        rec = {}
        for mode, code in (("single", L.LOR_PATCH_SINGLE), ("vertex", L.LOR_PATCH_VERTEX)):
            opt = L.lor_default_options()
            opt.patch_mode = code
            r = _solve_case(L, torch, 2, n, p, V, opt, rtol, 2, coef=coef, rhs="gaussian")
            rec[mode] = {"iters": r["iters"], "status": r["status"], "ms_per_solve": r["ms_per_solve"]}
        out[name] = rec
        print(f"[bench] coefficient {name}: B(1) {rec['single']['iters']} it, "
              f"B(V) {rec['vertex']['iters']} it", file=sys.stderr, flush=True)
    return {"workload": f"2D {n}x{n} perturbed (seed 4), p={p}, float64 PCG to {rtol:g}, Gaussian rhs",
            "iters": out}


def box_measure(L, torch, rtol):
    """Box-patch preconditioners of Section 4.5 on strip meshes, float64:
    milliseconds per application of B with each small box's whole V-cycle
    in one workgroup (every such box in one launch) and with the per-level
    launches (sweep_grid_rows = 1), B r compared element by element, and the
    flexible-CG solve to rtol with the default path."""
    from paper_1908_07071_amd import inputs
    cases = [(2, 8, 7, 150.0, "vertex_iso"), (2, 8, 7, 150.0, "slabs3"), (3, 6, 4, 15.0, "vertex_iso")]
    out = {}
    for dim, n, p, A, mode in cases:
        V = inputs.strip_vertices(n, A, dim=dim)
        rec = {}
        zs = []
        for path, rows in (("one_workgroup", 0), ("per_level", 1)):
            opt = L.lor_default_options()
            opt.patch_mode = L.LOR_PATCH_VERTEX_ISO if mode == "vertex_iso" else L.LOR_PATCH_SLABS
            opt.nslabs = 3 if mode == "slabs3" else 0
            opt.sweep_grid_rows = rows
            h = L.lor_setup(dim, n, V, p, options=opt)
            N = L.lor_ndofs(h)
            r = torch.tensor(inputs.gaussian_rhs(N, 5), device="cuda:0")
            z = torch.empty_like(r)
            reps = 20 if rows == 0 else 3
            for _ in range(2):
                L.lor_apply_P(h, r, z)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                L.lor_apply_P(h, r, z)
            e1.record()
            e1.synchronize()
            rec[f"{path}_ms_per_apply"] = e0.elapsed_time(e1) / reps
            zs.append(z.cpu())
            if rows == 0:
                x = torch.zeros_like(r)
                info, ms = solve_timed(L, torch, h, r, x, rtol, 1)
                rec.update({"N": N, "iters": info.iters, "ms_per_solve": ms,
                            "status": STATUS_NAMES.get(info.status, str(info.status))})
            L.lor_free(h)
        rec["bit_identical"] = bool(torch.equal(zs[0], zs[1]))
        key = f"{dim}d_n{n}_p{p}_A{A:g}_{mode}"
        out[key] = rec
        print(f"[bench] box {key}: {rec['one_workgroup_ms_per_apply']:.3f} ms per apply "
              f"({rec['per_level_ms_per_apply']:.2f} per-level), {rec['iters']} it, "
              f"{rec['ms_per_solve']:.1f} ms/solve", file=sys.stderr, flush=True)
    return {"workload": f"strip meshes (two element rows of aspect A), float64 box-patch preconditioners, "
                        f"flexible CG to {rtol:g}, Gaussian rhs", "cases": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--p", type=int, default=6)
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed",
                    help="mixed: FP32 patch V-cycles inside FP64 flexible CG")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dg", action="store_true", help="skip the DG (IP/BR2, 12^3, p=6) runs")
    ap.add_argument("--dg-n", type=int, default=12)
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the p sweep (p = 2, 4, 6, 8 on the benchmark mesh) and ordering variants")
    ap.add_argument("--orderings", default="mdf,rcm,natural",
                    help="ILU(0) orderings compared on the benchmark workload")
    ap.add_argument("--batch", type=int, default=0, metavar="NPROB",
                    help="only run the batched workload with NPROB problems (64 in the config)")
    ap.add_argument("--batch-rhs", type=int, default=4)
    ap.add_argument("--learned", action="store_true",
                    help="only run the learned patch correction workload (train, then 32^3 p=6 solves)")
    ap.add_argument("--learned-train-s", type=float, default=90.0)
    ap.add_argument("--learned-n", type=int, default=32)
    ap.add_argument("--nn-apply", action="store_true",
                    help="only time one preconditioner application per mode (V-cycles, network, warm start) "
                         "with an untrained 32-channel network at --learned-n^3, p=6 (kernel profiling)")
    ap.add_argument("--box", action="store_true",
                    help="only time the box-patch preconditioners (Section 4.5 strip meshes, 2D and 3D)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.calib_copy:
        import torch
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes_read": a.numel() * 8, "calib_copy_bytes_written": b.numel() * 8}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver is "
              "single-device (it would shard by element bricks with a halo exchange per "
              "iteration and a redundant coarse solve)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1908_07071_amd import inputs
    from paper_1908_07071_amd import lor as L

    if args.learned:
        res = learned_measure(L, torch, args.rtol, train_seconds=args.learned_train_s, n_test=args.learned_n)
        v, nw = res["vcycle"], res["network_replace"]
        print(json.dumps({
            "metric": "PCG DOFs/s to 1e-8 rel. residual (mixed/learned vs FP64)",
            "value": res["test_N"] / nw["s"] if nw["converged"] else 0.0, "unit": "DOF/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": nw["s"] * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64+bf16", "data": "synthetic",
            "config": {"workload": (f"3D CG, {args.learned_n}^3 perturbed hexes (seed 3), p=6; flexible CG to "
                                    f"{args.rtol:g} with a BF16 patch network (3 conv layers, 32 channels) "
                                    "standing in for every patch V-cycle, trained on pairs the method "
                                    "generates on 16^3 meshes (seeds 10, 11)")},
            "learned": res}))
        return
    if args.batch:
        print(json.dumps(batch_measure(L, torch, args.batch, args.batch_rhs, args.rtol, args.precision)))
        return
    if args.nn_apply:
        print(json.dumps(nn_apply_measure(L, torch, args.learned_n)))
        return
    if args.box:
        print(json.dumps(box_measure(L, torch, args.rtol)))
        return

    dim, n, p = args.dim, args.n, args.p
    dev = torch.device("cuda:0")
    V = inputs.structured_vertices(dim, n, 0.1, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    opt = L.lor_default_options()
    opt.precision = L.LOR_PREC_MIXED if args.precision == "mixed" else L.LOR_PREC_FP64
    h = L.lor_setup(dim, n, V, p, options=opt)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"[bench] setup done in {setup_s:.1f}s", file=sys.stderr, flush=True)
    N = L.lor_ndofs(h)
    # the device data moves into a torch-owned buffer (torch's caching
    # allocator owns the solver's device memory)
    order_info = L.lor_launch_order(h)
    print(f"[bench] patch launch order {order_info[0]} (autotuned: vertex order {order_info[1]:.3f} ms, "
          f"buckets {order_info[2]:.3f} ms)", file=sys.stderr, flush=True)
    dev_bytes = L.lor_workspace_bytes(h)
    ws = torch.empty(dev_bytes, dtype=torch.uint8, device="cuda:0")
    L.lor_bind_workspace(h, ws)
    assert L.lor_device_bytes(h) == 0
    coords = L.lor_dof_coords(h, dim)
    f = torch.tensor(inputs.manufactured_f(coords), device=dev)
    b = torch.empty_like(f)
    L.lor_assemble_rhs(h, f, b)
    x = torch.zeros_like(b)

    for _ in range(args.warmup):
        info = L.lor_pcg_solve(h, b, x, rtol=args.rtol, maxit=1000)
    torch.cuda.synchronize()
    L.lor_timing(h, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = L.lor_pcg_solve(h, b, x, rtol=args.rtol, maxit=1000)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    L.lor_timing(h, False)
    ms_step = 1e3 * t_total / args.steps
    tA, nA = L.lor_timing_read(h, L.LOR_T_APPLY_A)
    tP, nP = L.lor_timing_read(h, L.LOR_T_PATCH)
    tC, nC = L.lor_timing_read(h, L.LOR_T_COARSE)
    print(f"[bench] {args.steps} solves: {ms_step:.2f} ms/solve, iters={info.iters}, "
          f"rel_res_true={info.rel_res_true:.2e}", file=sys.stderr, flush=True)

    # operator throughput: 100 back-to-back applies, HIP events
    xr = torch.tensor(inputs.uniform_vector(N, 3), device=dev)
    y = torch.empty_like(xr)
    for _ in range(5):
        L.lor_apply_A(h, xr, y)
    L.lor_timing(h, True)
    for _ in range(100):
        L.lor_apply_A(h, xr, y)
    tAop, nAop = L.lor_timing_read(h, L.LOR_T_APPLY_A)
    L.lor_timing(h, False)
    t_apply = tAop / nAop * 1e-3

    # dominant kernel of the solve
    kernels = {
        "patch_vcycle": (tP / max(nP, 1), patch_algorithmic_bytes(dim, n, p)),
        "apply_A": (tA / max(nA, 1), apply_algorithmic_bytes(dim, n, p)),
    }
    dom = "patch_vcycle" if tP >= tA else "apply_A"
    avg_ms, abytes = kernels[dom]
    if dom == "patch_vcycle" and args.precision == "mixed":
        abytes = patch_algorithmic_bytes(dim, n, p, prec_bytes=4)
    achieved = abytes / (avg_ms * 1e-3) / 1e9
    L.lor_free(h)

    # the same solve with the float64 preconditioner, for the mixed-vs-FP64 comparison
    fp64 = None
    if args.precision == "mixed":
        h64 = L.lor_setup(dim, n, V, p)
        x.zero_()
        info64 = L.lor_pcg_solve(h64, b, x, rtol=args.rtol, maxit=1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            info64 = L.lor_pcg_solve(h64, b, x, rtol=args.rtol, maxit=1000)
        torch.cuda.synchronize()
        ms64 = 1e3 * (time.perf_counter() - t0) / args.steps
        L.lor_free(h64)
        fp64 = {"value": N / (ms64 * 1e-3), "ms_per_step": ms64, "iters": info64.iters,
                "rel_res_true": info64.rel_res_true}
        print(f"[bench] fp64 preconditioner: {ms64:.2f} ms/solve, iters={info64.iters}",
              file=sys.stderr, flush=True)

    out = {
        "metric": "PCG DOFs/s to 1e-8 rel. residual (mixed/learned vs FP64); operator GDOF/s",
        "value": N / (ms_step * 1e-3),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{dim}D CG Poisson, {n}^{dim} hexes with interior vertices perturbed <=10% h "
                         f"(seed 1), p={p}, f from u=prod sin(pi x_i); "
                         + ("FP64 flexible CG with FP32 " if args.precision == "mixed" else "FP64 PCG with FP64 ")
                         + f"LOR vertex-patch Schwarz (MDF-ILU(0) V-cycles, exact coarse) to {args.rtol:g}"),
            "N": N, "iters": info.iters, "rel_res_true": info.rel_res_true,
            "status": STATUS_NAMES.get(info.status, str(info.status)),
            "precision": args.precision, "setup_s": round(setup_s, 3),
            "device_bytes": dev_bytes, "device_memory": "caller-owned torch buffer (lor_bind_workspace)",
            "patch_launch_order": dict(zip(("used", "ms_vertex_order", "ms_buckets"), order_info)),
        },
        "fp64_preconditioner": fp64,
        "operator_gdofs": N / t_apply / 1e9,
        "operator_ms": t_apply * 1e3,
        "kernel_ms_per_solve": {
            "apply_A": tA / args.steps, "patch_vcycle": tP / args.steps, "coarse": tC / args.steps,
        },
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (measured_traffic(dom) if (dim, n, p) == (3, 16, 6) and args.precision == "mixed"
                        else None),
            "algorithmic_bytes_per_launch": abytes, "avg_launch_ms": avg_ms,
        },
    }
    out["hbm_copy_gbs"] = copy_bandwidth(torch)
    out["roofline"]["frac_of_copy"] = achieved / out["hbm_copy_gbs"]
    out["operator_hbm_frac"] = apply_algorithmic_bytes(dim, n, p) / t_apply / (HBM_PEAK_GBS * 1e9)
    if not args.no_sweep:
        # the 32^3 p = 6 mesh of the learned-correction workload, plain
        # float32-preconditioner solve (N = 6,967,871)
        V32 = inputs.structured_vertices(3, 32, 0.1, seed=3)
        opt32 = L.lor_default_options()
        opt32.precision = L.LOR_PREC_MIXED
        rec32 = _solve_case(L, torch, 3, 32, 6, V32, opt32, args.rtol, 2)
        rec32["workload"] = ("3D CG 32^3 perturbed (seed 3), p=6, f from the manufactured u, FP64 "
                             "flexible CG with FP32 LOR vertex-patch Schwarz (MDF) to " + f"{args.rtol:g}")
        out["cube_32_p6_mixed"] = rec32
        print(f"[bench] 32^3 p=6 mixed: {rec32['iters']} it, {rec32['ms_per_solve']:.1f} ms/solve, "
              f"{rec32['dofs_per_s'] / 1e6:.2f} M DOF/s, setup {rec32['setup_s']:.1f} s",
              file=sys.stderr, flush=True)
        # the benchmark mesh with bent (isoparametric) elements
        Vc = inputs.curved_vertices(3, 16, 0.15, 0.1, 1)
        Xc = inputs.curved_nodes(3, 16, 6, 0.15, 0.1, 1)
        hc = L.lor_setup(3, 16, Vc, 6, options=opt32, nodes=Xc)
        Nc = L.lor_ndofs(hc)
        fc = torch.tensor(inputs.manufactured_f(L.lor_dof_coords(hc, 3)), device="cuda:0")
        bc_ = torch.empty_like(fc)
        L.lor_assemble_rhs(hc, fc, bc_)
        xc = torch.zeros_like(bc_)
        infc, msc = solve_timed(L, torch, hc, bc_, xc, args.rtol, 2)
        L.lor_free(hc)
        out["cube_16_p6_curved_mixed"] = {"N": Nc, "iters": infc.iters, "ms_per_solve": msc,
                                          "dofs_per_s": Nc / (msc * 1e-3),
                                          "status": STATUS_NAMES.get(infc.status, str(infc.status)),
                                          "rel_res_true": infc.rel_res_true,
                                          "workload": "16^3, p=6, elements bent by x + 0.15*16*prod x(1-x) "
                                                      "(isoparametric, GLL node coordinates), vertices "
                                                      "perturbed <=10% h (seed 1), mixed FCG"}
        print(f"[bench] 16^3 p=6 curved mixed: {infc.iters} it, {msc:.1f} ms/solve", file=sys.stderr,
              flush=True)
        out["single_patch"] = single_patch_measure(L, torch, args.rtol)
        out["coefficients"] = coefficient_measure(L, torch, args.rtol)
        out["strip"] = strip_measure(L, torch, args.rtol)
        # a smaller instance of the batched workload (16 problems, 4 right
        # sides each) so that the default line carries a batched measurement
        bm = batch_measure(L, torch, 16, 4, args.rtol, "mixed")
        out["batch16"] = {"value": bm["value"], "unit": bm["unit"], "ms": bm["ms_per_step"],
                          "sequential_value": bm["sequential_value"],
                          "speedup_vs_sequential": bm["speedup_vs_sequential"],
                          "config": bm["config"]}
        out["p_sweep"] = p_sweep(L, torch, dim, n, (2, 4, 6, 8), args.rtol, 2)
        out["orderings"] = ordering_variants(L, torch, dim, n, p, args.rtol, 3,
                                             [o for o in args.orderings.split(",") if o])
    if not args.no_dg:
        out["dg"] = dg_measure(L, torch, dim, args.dg_n, p, args.rtol, 1, args.precision)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(dim, p, info.iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

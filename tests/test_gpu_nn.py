"""Learned patch correction on the GPU against the float64 reference
(oracle/nn.py), through the C ABI.

Tolerances: the network's products run in bfloat16 (8-bit significand) with
float32 accumulation, so outputs and gradients are compared to a few
percent; the patch data (float32 copies of float64 values) to float32
rounding.  Element by element: every operand (input, weight, activation
between layers) is rounded to bfloat16 (relative error <= 2^-9 ~ 2e-3), so
each of the three layers adds about 3 such roundings relative to the sum of
magnitudes of its products; |y_i - yref_i| <= BF16_TOL max|yref| allows the
three layers 1.8e-2 plus cancellation.  Measured: 1.2e-2 on the worst patch
at 16 channels, 5e-3 at 32.
"""
import numpy as np
import pytest

from oracle import krylov, mesh as M, nn as ONN, schwarz as S
from paper_1908_07071_amd import inputs

pytestmark = pytest.mark.gpu

C = 16
BF16_TOL = 3e-2


def _emax(a, ref):
    """max |a - ref| / max |ref| (element by element)."""
    return np.abs(np.asarray(a) - ref).max() / np.abs(ref).max()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "HIP device required"
    return torch


@pytest.fixture(scope="module")
def L():
    from paper_1908_07071_amd import lor
    return lor


def _bf16(x):
    """float32 -> bfloat16 bit patterns (round to nearest even) and values."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    bits = u.astype(np.uint16)
    return bits.view(np.int16), (bits.astype(np.uint32) << 16).view(np.float32)


def test_bf16_gemm_layouts(L, torch_dev):
    torch = torch_dev
    rng = np.random.default_rng(1)
    Mm, N, K = 48, 32, 64
    A = rng.standard_normal((Mm, K)).astype(np.float32)
    B = rng.standard_normal((K, N)).astype(np.float32)
    Ab, Av = _bf16(A)
    Bb, Bv = _bf16(B)
    ref = Av.astype(np.float64) @ Bv.astype(np.float64)
    Cg = torch.zeros((Mm, N), dtype=torch.float32, device="cuda")
    # A row-major (k contiguous), B row-major
    L.lor_bf16_gemm(Mm, N, K, torch.tensor(Ab.ravel(), device="cuda"), K, 1,
                    torch.tensor(Bb.ravel(), device="cuda"), N, 1, Cg, N)
    assert np.abs(Cg.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()
    # A stored transposed (A(i,k) at k*M + i), B stored transposed (B(k,j) at j*K + k)
    AbT = np.ascontiguousarray(Ab.T).ravel()
    BbT = np.ascontiguousarray(Bb.T).ravel()
    Cg.zero_()
    L.lor_bf16_gemm(Mm, N, K, torch.tensor(AbT, device="cuda"), 1, Mm,
                    torch.tensor(BbT, device="cuda"), 1, K, Cg, N)
    assert np.abs(Cg.cpu().numpy() - ref).max() <= 1e-5 * np.abs(ref).max()


def _problem(L, n=2, p=3, seed=9, fallback=1):
    V = inputs.structured_vertices(3, n, 0.1, seed=seed)
    mesh = M.make_mesh(3, [n] * 3, V)
    opt = L.lor_default_options()
    opt.nn_fallback = fallback
    h = L.lor_setup(3, n, V, p, options=opt)
    return h, mesh, p


def _data(L, torch, nn, h, seed):
    J, G = L.lor_nn_shape(nn)
    N = L.lor_ndofs(h)
    r = torch.tensor(inputs.gaussian_rhs(N, seed), device="cuda")
    X = torch.zeros((J, G ** 3, 2), dtype=torch.float32, device="cuda")
    T = torch.zeros((J, G ** 3), dtype=torch.float32, device="cuda")
    sc = torch.zeros(J, dtype=torch.float64, device="cuda")
    L.lor_nn_patch_data(nn, r, X, T, sc)
    torch.cuda.synchronize()
    return r, X, T, sc


def test_patch_data_and_forward_match_oracle(L, torch_dev):
    torch = torch_dev
    h, mesh, p = _problem(L)
    params = inputs.nn_initial_params(C, seed=3)
    nn = L.lor_nn_create(h, C, params, max_batch=32)
    try:
        r, X, T, sc = _data(L, torch, nn, h, 5)
        B = S.SchwarzLOR(mesh, p)
        Xr, Tr, sr = ONN.patch_samples(B, r.cpu().numpy())
        assert np.allclose(sc.cpu().numpy(), sr, rtol=1e-14)
        assert np.abs(X.cpu().numpy() - Xr).max() <= 1e-6
        assert np.abs(T.cpu().numpy() - Tr).max() <= 1e-6 * np.abs(Tr).max()
        J, G = L.lor_nn_shape(nn)
        Y = torch.zeros((J, G ** 3), dtype=torch.float32, device="cuda")
        L.lor_nn_forward(nn, X, J, Y)
        torch.cuda.synchronize()
        shapes = ONN.layer_shapes(C)
        yref, _ = ONN.forward(ONN.unflatten(params, shapes), X.cpu().numpy().astype(np.float64), G)
        err = np.linalg.norm(Y.cpu().numpy() - yref) / np.linalg.norm(yref)
        assert err <= 3e-2, err
        assert _emax(Y.cpu().numpy(), yref) <= BF16_TOL
    finally:
        L.lor_nn_free(nn)
        L.lor_free(h)


@pytest.mark.parametrize("channels", [32, 48])
def test_forward_paths_match_oracle(channels, L, torch_dev):
    """The fused implicit-GEMM convolutions (16 and 32 channels) and the
    explicit im2col + GEMM path (other widths) against the float64 forward
    pass, on a p = 4 grid (G = 7) with boundary and interior patches."""
    torch = torch_dev
    h, mesh, p = _problem(L, n=2, p=4, seed=12)
    params = inputs.nn_initial_params(channels, seed=6)
    nn = L.lor_nn_create(h, channels, params, max_batch=32)
    try:
        r, X, T, sc = _data(L, torch, nn, h, 8)
        J, G = L.lor_nn_shape(nn)
        Y = torch.zeros((J, G ** 3), dtype=torch.float32, device="cuda")
        L.lor_nn_forward(nn, X, J, Y)
        torch.cuda.synchronize()
        shapes = ONN.layer_shapes(channels)
        yref, _ = ONN.forward(ONN.unflatten(params, shapes), X.cpu().numpy().astype(np.float64), G)
        err = np.linalg.norm(Y.cpu().numpy() - yref) / np.linalg.norm(yref)
        print("channels", channels, "forward error", err, "max", _emax(Y.cpu().numpy(), yref), flush=True)
        assert err <= 3e-2, err
        assert _emax(Y.cpu().numpy(), yref) <= BF16_TOL
    finally:
        L.lor_nn_free(nn)
        L.lor_free(h)


def test_gradients_match_oracle(L, torch_dev):
    torch = torch_dev
    h, mesh, p = _problem(L)
    params = inputs.nn_initial_params(C, seed=4)
    nn = L.lor_nn_create(h, C, params, max_batch=32)
    try:
        r, X, T, sc = _data(L, torch, nn, h, 6)
        J, G = L.lor_nn_shape(nn)
        nparam = L.lor_nn_param_count(C)
        loss, g = L.lor_nn_gradients(nn, X, T, J, nparam)
        shapes = ONN.layer_shapes(C)
        lref, gref = ONN.loss_and_grads(ONN.unflatten(params, shapes), X.cpu().numpy().astype(np.float64),
                                        T.cpu().numpy().astype(np.float64), G)
        assert abs(loss - lref) <= 2e-2 * lref, (loss, lref)
        o = 0
        for (k, n), (dW, db) in zip(shapes, gref):
            gw = g[o:o + k * n].reshape(k, n)
            o += k * n
            gb = g[o:o + n]
            o += n
            assert np.linalg.norm(gw - dW) <= 5e-2 * np.linalg.norm(dW), (k, n)
            assert np.linalg.norm(gb - db) <= 5e-2 * np.linalg.norm(db) + 1e-7, (k, n)
        # a batch without a masked point has no loss: refused, and a training
        # step on it leaves the parameters as they were
        X0 = X.clone()
        X0[..., 1] = 0.0
        with pytest.raises(L.LorError) as ei:
            L.lor_nn_train_step(nn, X0, T, J, 1e-3)
        assert ei.value.code == L.LOR_EINVAL
        w_before = L.lor_nn_get_params(nn, C)
        with pytest.raises(L.LorError):
            L.lor_nn_train_step(nn, X0, T, J, 1e-3)
        assert np.array_equal(L.lor_nn_get_params(nn, C), w_before)
    finally:
        L.lor_nn_free(nn)
        L.lor_free(h)


def test_training_and_replace_preconditioner(L, torch_dev):
    """Adam lowers the loss on data the method generates; the network then
    stands in for the patch V-cycles (parity with the float64 reference
    preconditioner at bfloat16 accuracy), and flexible CG still converges;
    as a warm start of the patch V-cycles it matches the float64 reference
    warm start and flexible CG converges in about the V-cycle's iterations."""
    torch = torch_dev
    # the network alone, to the end of each solve (no V-cycle fallback)
    h, mesh, p = _problem(L, fallback=0)
    params = inputs.nn_initial_params(C, seed=5)
    nn = L.lor_nn_create(h, C, params, max_batch=64)
    try:
        J, G = L.lor_nn_shape(nn)
        Xs, Ts = [], []
        for s in range(2):
            _, X, T, _ = _data(L, torch, nn, h, 100 + s)
            Xs.append(X)
            Ts.append(T)
        X = torch.cat(Xs).contiguous()
        T = torch.cat(Ts).contiguous()
        first = last = None
        for it in range(300):
            loss = L.lor_nn_train_step(nn, X, T, X.shape[0], 3e-3)
            first = loss if first is None else first
            last = loss
        assert last < 0.5 * first, (first, last)
        # the network inside the preconditioner
        L.lor_nn_attach(h, nn, L.LOR_NN_REPLACE)
        N = L.lor_ndofs(h)
        rin = inputs.gaussian_rhs(N, 7)
        rt = torch.tensor(rin, device="cuda")
        z = torch.empty_like(rt)
        L.lor_apply_P(h, rt, z)
        torch.cuda.synchronize()
        shapes = ONN.layer_shapes(C)
        wn = L.lor_nn_get_params(nn, C)
        B = S.SchwarzLOR(mesh, p)
        zref = ONN.preconditioner_replace(B, ONN.unflatten(wn, shapes), rin)
        err = np.linalg.norm(z.cpu().numpy() - zref) / np.linalg.norm(zref)
        assert err <= 3e-2, err
        assert _emax(z.cpu().numpy(), zref) <= BF16_TOL
        x = torch.zeros_like(rt)
        info = L.lor_pcg_solve(h, rt, x, rtol=1e-6, maxit=400, check=False)
        print("FCG with the network:", info.iters, info.status, flush=True)
        assert info.status in (L.LOR_OK, L.LOR_ENOCONV)
        # warm start: the network's prediction corrected by one V-cycle per
        # patch; the V-cycle damps the network's BF16 error
        L.lor_nn_attach(h, nn, L.LOR_NN_WARMSTART)
        L.lor_apply_P(h, rt, z)
        torch.cuda.synchronize()
        zw = ONN.preconditioner_warmstart(B, ONN.unflatten(wn, shapes), rin)
        errw = np.linalg.norm(z.cpu().numpy() - zw) / np.linalg.norm(zw)
        print("warm start parity", errw, "max", _emax(z.cpu().numpy(), zw), flush=True)
        assert errw <= 3e-2, errw
        assert _emax(z.cpu().numpy(), zw) <= BF16_TOL
        x.zero_()
        infow = L.lor_pcg_solve(h, rt, x, rtol=1e-6, maxit=400, check=False)
        print("FCG with the warm start:", infow.iters, infow.status, flush=True)
        assert infow.status == L.LOR_OK
        L.lor_nn_attach(h, None, L.LOR_NN_OFF)
        x.zero_()
        info0 = L.lor_pcg_solve(h, rt, x, rtol=1e-6, maxit=400)
        assert info0.status == L.LOR_OK
        assert infow.iters <= 1.5 * info0.iters + 3, (infow.iters, info0.iters)
        # What the trained network gains over the method without it, stated:
        # nothing here.  In place of the V-cycles it needs more iterations
        # (or does not converge), and as a warm start it adds the network's
        # cost to every application of the V-cycles.
        assert info.status != L.LOR_OK or info.iters > info0.iters, (info.iters, info0.iters)
        times = {}
        for mode in (L.LOR_NN_OFF, L.LOR_NN_WARMSTART):
            L.lor_nn_attach(h, nn if mode else None, mode)
            L.lor_apply_P(h, rt, z)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(20):
                L.lor_apply_P(h, rt, z)
            e1.record()
            e1.synchronize()
            times[mode] = e0.elapsed_time(e1) / 20
        L.lor_nn_attach(h, None, L.LOR_NN_OFF)
        print("iterations: V-cycle", info0.iters, "network", info.iters, "warm start", infow.iters,
              "; ms per application: V-cycle", times[L.LOR_NN_OFF], "warm start",
              times[L.LOR_NN_WARMSTART], flush=True)
        assert times[L.LOR_NN_WARMSTART] > times[L.LOR_NN_OFF]
    finally:
        L.lor_nn_free(nn)
        L.lor_free(h)


@pytest.mark.parametrize("channels", [16, 32])
def test_p6_grid_forward_replace_warmstart(channels, L, torch_dev):
    """p = 6: the 11^3 patch grid (G = 11), where the fused convolution gives
    each wavefront a second output tile of the plane (G^2 = 121 > 64).
    Forward pass, the network in place of the patch V-cycles, and the warm
    start, each against the float64 reference with the same weights."""
    torch = torch_dev
    h, mesh, p = _problem(L, n=2, p=6, seed=13)
    params = inputs.nn_initial_params(channels, seed=7)
    nn = L.lor_nn_create(h, channels, params, max_batch=32)
    try:
        J, G = L.lor_nn_shape(nn)
        assert G == 11
        r, X, T, sc = _data(L, torch, nn, h, 9)
        Y = torch.zeros((J, G ** 3), dtype=torch.float32, device="cuda")
        L.lor_nn_forward(nn, X, J, Y)
        torch.cuda.synchronize()
        shapes = ONN.layer_shapes(channels)
        P = ONN.unflatten(params, shapes)
        yref, _ = ONN.forward(P, X.cpu().numpy().astype(np.float64), G)
        err = np.linalg.norm(Y.cpu().numpy() - yref) / np.linalg.norm(yref)
        print("channels", channels, "G = 11 forward error", err, flush=True)
        assert err <= 3e-2, err
        # every patch's output, not just the norm over all of them
        Yg = Y.cpu().numpy()
        assert _emax(Yg, yref) <= BF16_TOL
        for j in range(J):
            nj = np.linalg.norm(yref[j])
            if nj > 0:
                assert np.linalg.norm(Yg[j] - yref[j]) <= 5e-2 * nj, j
                assert _emax(Yg[j], yref[j]) <= 5e-2, j
        B = S.SchwarzLOR(mesh, p)
        rin = r.cpu().numpy()
        z = torch.empty_like(r)
        L.lor_nn_attach(h, nn, L.LOR_NN_REPLACE)
        L.lor_apply_P(h, r, z)
        torch.cuda.synchronize()
        zref = ONN.preconditioner_replace(B, P, rin)
        err = np.linalg.norm(z.cpu().numpy() - zref) / np.linalg.norm(zref)
        print("replace parity", err, "max", _emax(z.cpu().numpy(), zref), flush=True)
        assert err <= 3e-2, err
        assert _emax(z.cpu().numpy(), zref) <= BF16_TOL
        L.lor_nn_attach(h, nn, L.LOR_NN_WARMSTART)
        L.lor_apply_P(h, r, z)
        torch.cuda.synchronize()
        zw = ONN.preconditioner_warmstart(B, P, rin)
        errw = np.linalg.norm(z.cpu().numpy() - zw) / np.linalg.norm(zw)
        print("warm start parity", errw, "max", _emax(z.cpu().numpy(), zw), flush=True)
        assert errw <= 3e-2, errw
        assert _emax(z.cpu().numpy(), zw) <= BF16_TOL
        L.lor_nn_attach(h, None, L.LOR_NN_OFF)
    finally:
        L.lor_nn_free(nn)
        L.lor_free(h)


def test_vcycle_fallback(L, torch_dev):
    """An untrained network in place of the patch V-cycles: with the
    fallback (the default) flexible CG leaves it for the V-cycles once it
    breaks down or stalls and still reaches the tolerance, the true residual
    included; without it the network runs to the end of the solve."""
    torch = torch_dev
    for fallback in (1, 0):
        h, mesh, p = _problem(L, fallback=fallback)
        nn = L.lor_nn_create(h, C, inputs.nn_initial_params(C, seed=11), max_batch=32)
        try:
            N = L.lor_ndofs(h)
            r = torch.tensor(inputs.gaussian_rhs(N, 12), device="cuda")
            x0 = torch.zeros_like(r)
            info0 = L.lor_pcg_solve(h, r, x0, rtol=1e-8, maxit=400)
            assert info0.fallback_iter == -1
            L.lor_nn_attach(h, nn, L.LOR_NN_REPLACE)
            x = torch.zeros_like(r)
            info = L.lor_pcg_solve(h, r, x, rtol=1e-8, maxit=400, check=False)
            print("fallback", fallback, "status", info.status, "iterations", info.iters, "switched at",
                  info.fallback_iter, "V-cycle alone", info0.iters, flush=True)
            if fallback:
                assert info.status == L.LOR_OK and info.rel_res_true <= 1e-8, (info.status, info.rel_res_true)
                assert 0 <= info.fallback_iter < info.iters
                # the network stays attached for the next solve
                x.zero_()
                info2 = L.lor_pcg_solve(h, r, x, rtol=1e-8, maxit=400, check=False)
                assert info2.fallback_iter >= 0
            else:
                assert info.fallback_iter == -1
        finally:
            L.lor_nn_attach(h, None, L.LOR_NN_OFF)
            L.lor_nn_free(nn)
            L.lor_free(h)


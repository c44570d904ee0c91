"""Parity at the benchmark's full size: 3D CG, 16^3 hexes with interior
vertices perturbed by at most 10% of h (seed 1), p = 6: N = 857,375 unknowns
and 4,913 patches, each GPU result taken from one launch over the whole
problem, as the benchmark runs it.  The oracle computes sampled outputs one
by one:

* operator: K_p x at sampled unknowns, from the element matrices around them;
* patch V-cycles: sampled patches (interior, face, edge and corner vertices)
  from the patch built on its 2^d elements, which equals the patch built on
  the whole mesh bit for bit (pinned in tests/oracle/test_schwarz.py); the
  GPU's per-patch results come from the patch kernel's patch-grid output;
* the preconditioner as a whole: symmetry and positivity, which hold at any
  size, and the float32 preconditioner against the float64 one;
* the solve: the true residual reaches the tolerance, and the float32 and
  float64 preconditioners take the same number of iterations within two;
* DG at its benchmark size (12^3, seed 2, p = 6, IP and BR2, eta = 1.5 (p+1)^2):
  operator rows from the element and face terms around them, symmetry and
  positivity of the DG preconditioner, float32 against float64, the solve.

Tolerances: float64 paths 1e-12 relative as in the small cases, except
where the output is float32 (the patch-grid output, 2e-7); the float32
preconditioner 2e-5 relative as in the small cases.
"""
import numpy as np
import pytest

from oracle import gll, highorder as HO, mesh as M, nn as ONN, schwarz as S
from paper_1908_07071_amd import inputs

pytestmark = pytest.mark.gpu

N_EL, P = 16, 6
SAMPLED_VERTICES = [(8, 8, 8), (0, 8, 8), (0, 0, 8), (0, 0, 0), (16, 3, 16), (5, 16, 11), (1, 1, 15)]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "HIP device required"
    return torch


@pytest.fixture(scope="module")
def L():
    from paper_1908_07071_amd import lor
    return lor


@pytest.fixture(scope="module")
def patch_refs():
    """Oracle V-cycles of the sampled patches for the residual of seed 31:
    {vertex: (patch-grid positions, V_j r_j)} (CPU only, shared by both
    precisions)."""
    V = inputs.structured_vertices(3, N_EL, 0.1, seed=1)
    mesh = M.make_mesh(3, [N_EL] * 3, V)
    rin = inputs.gaussian_rhs((N_EL * P - 1) ** 3, 31)
    ref_nodes, _ = gll.gll(P)
    fc = M.global_node_coords(mesh, ref_nodes, P)
    out = {}
    for v in SAMPLED_VERTICES:
        Pl, u = S.local_patch(mesh, P, v, fine_coords=fc)
        _, q = ONN.patch_grid(mesh, P, v)
        out[v] = (q, Pl.solve(rin[u]))
    return out


@pytest.fixture(scope="module")
def problem(L, torch_dev):
    V = inputs.structured_vertices(3, N_EL, 0.1, seed=1)
    mesh = M.make_mesh(3, [N_EL] * 3, V)
    handles = {}
    for name, prec in (("mixed", L.LOR_PREC_MIXED), ("fp64", L.LOR_PREC_FP64)):
        opt = L.lor_default_options()
        opt.precision = prec
        handles[name] = L.lor_setup(3, N_EL, V, P, options=opt)
    print("full-size handles ready", flush=True)
    yield mesh, handles
    for h in handles.values():
        L.lor_free(h)


def test_operator_sampled_rows(L, torch_dev, problem):
    torch = torch_dev
    mesh, handles = problem
    h = handles["fp64"]
    N = L.lor_ndofs(h)
    assert N == (N_EL * P - 1) ** 3
    xin = inputs.uniform_vector(N, 13)
    x = torch.tensor(xin, device="cuda")
    y = torch.empty_like(x)
    L.lor_apply_A(h, x, y)
    torch.cuda.synchronize()
    yh = y.cpu().numpy()
    rows = np.random.default_rng(5).choice(N, 40, replace=False)
    ref = HO.cg_apply_rows(mesh, P, xin, rows)
    err = np.abs(yh[rows] - ref).max() / np.abs(yh).max()
    print("operator rows error", err, flush=True)
    assert err <= 1e-12, err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_patch_vcycles_sampled(prec, L, torch_dev, problem, patch_refs):
    torch = torch_dev
    mesh, handles = problem
    h = handles[prec]
    N = L.lor_ndofs(h)
    nn = L.lor_nn_create(h, 16, inputs.nn_initial_params(16, seed=1), max_batch=1)
    try:
        J, G = L.lor_nn_shape(nn)
        assert J == (N_EL + 1) ** 3 and G == 2 * P - 1
        rin = inputs.gaussian_rhs(N, 31)
        r = torch.tensor(rin, device="cuda")
        X = torch.zeros((J, G ** 3, 2), dtype=torch.float32, device="cuda")
        T = torch.zeros((J, G ** 3), dtype=torch.float32, device="cuda")
        sc = torch.zeros(J, dtype=torch.float64, device="cuda")
        L.lor_nn_patch_data(nn, r, X, T, sc)
        torch.cuda.synchronize()
        T, sc = T.cpu().numpy(), sc.cpu().numpy()
    finally:
        L.lor_nn_free(nn)
    tol = 2e-7 if prec == "fp64" else 2e-5
    for v in SAMPLED_VERTICES:
        j = v[0] + (N_EL + 1) * (v[1] + (N_EL + 1) * v[2])
        q, zref = patch_refs[v]
        zgpu = T[j, q].astype(np.float64) * sc[j]
        err = np.abs(zgpu - zref).max() / np.abs(zref).max()
        print(prec, "patch", v, "rows", len(q), "error", err, flush=True)
        assert err <= tol, (v, err)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_preconditioner_symmetric_positive(prec, L, torch_dev, problem):
    torch = torch_dev
    _, handles = problem
    h = handles[prec]
    N = L.lor_ndofs(h)
    r1 = torch.tensor(inputs.gaussian_rhs(N, 41), device="cuda")
    r2 = torch.tensor(inputs.gaussian_rhs(N, 42), device="cuda")
    z1, z2 = torch.empty_like(r1), torch.empty_like(r1)
    L.lor_apply_P(h, r1, z1)
    L.lor_apply_P(h, r2, z2)
    torch.cuda.synchronize()
    a, b = float(r2 @ z1), float(r1 @ z2)
    e1, e2 = float(r1 @ z1), float(r2 @ z2)
    assert e1 > 0 and e2 > 0
    asym = abs(a - b) / np.sqrt(e1 * e2)
    print(prec, "asymmetry", asym, flush=True)
    assert asym <= (1e-12 if prec == "fp64" else 2e-5), asym
    if prec == "mixed":
        z64 = torch.empty_like(r1)
        L.lor_apply_P(handles["fp64"], r1, z64)
        torch.cuda.synchronize()
        err = float((z1 - z64).norm() / z64.norm())
        print("float32 against float64 preconditioner", err, flush=True)
        assert err <= 2e-5, err


def test_solve(L, torch_dev, problem):
    torch = torch_dev
    _, handles = problem
    N = L.lor_ndofs(handles["mixed"])
    b = torch.tensor(inputs.gaussian_rhs(N, 51), device="cuda")
    its = {}
    for name in ("mixed", "fp64"):
        x = torch.zeros_like(b)
        info = L.lor_pcg_solve(handles[name], b, x, rtol=1e-8, maxit=500)
        print(name, "iterations", info.iters, "true residual", info.rel_res_true, flush=True)
        assert info.status == L.LOR_OK and info.rel_res_true <= 1.05e-8
        its[name] = info.iters
    assert abs(its["mixed"] - its["fp64"]) <= 2, its


# ---------------------------------------------------------------------------
# DG at its benchmark size: 12^3 hexes perturbed by at most 10% of h (seed 2),
# p = 6, IP and BR2 (N_DG = 592,704)
DG_EL, DG_ETA = 12, 1.5 * (P + 1) ** 2


@pytest.fixture(scope="module")
def dg_problem(L, torch_dev):
    V = inputs.structured_vertices(3, DG_EL, 0.1, seed=2)
    mesh = M.make_mesh(3, [DG_EL] * 3, V)
    handles = {}
    for method, code in (("ip", L.LOR_IP), ("br2", L.LOR_BR2)):
        for name, prec in (("mixed", L.LOR_PREC_MIXED), ("fp64", L.LOR_PREC_FP64)):
            opt = L.lor_default_options()
            opt.precision = prec
            handles[(method, name)] = L.lor_setup(3, DG_EL, V, P, method=code, penalty=DG_ETA, options=opt)
    print("full-size DG handles ready", flush=True)
    yield mesh, handles
    for h in handles.values():
        L.lor_free(h)


@pytest.mark.parametrize("method", ["ip", "br2"])
def test_dg_operator_sampled_rows(method, L, torch_dev, dg_problem):
    torch = torch_dev
    mesh, handles = dg_problem
    h = handles[(method, "fp64")]
    N = L.lor_ndofs(h)
    nloc = (P + 1) ** 3
    assert N == DG_EL ** 3 * nloc
    xin = inputs.uniform_vector(N, 17)
    x = torch.tensor(xin, device="cuda")
    y = torch.empty_like(x)
    L.lor_apply_A(h, x, y)
    torch.cuda.synchronize()
    yh = y.cpu().numpy()
    rng = np.random.default_rng(9)
    # a corner, an interior and an edge element, eight rows each
    elems = [0, 5 + DG_EL * (6 + DG_EL * 7), DG_EL - 1 + DG_EL * (DG_EL - 1 + DG_EL * 3)]
    rows = np.concatenate([e * nloc + rng.choice(nloc, 8, replace=False) for e in elems])
    ref = HO.dg_apply_rows(mesh, P, method, DG_ETA, xin, rows)
    err = np.abs(yh[rows] - ref).max() / np.abs(yh).max()
    print(method, "DG operator rows error", err, flush=True)
    assert err <= 1e-12, err


@pytest.mark.parametrize("method", ["ip", "br2"])
def test_dg_preconditioner_and_solve(method, L, torch_dev, dg_problem):
    torch = torch_dev
    _, handles = dg_problem
    h, h64 = handles[(method, "mixed")], handles[(method, "fp64")]
    N = L.lor_ndofs(h)
    r1 = torch.tensor(inputs.gaussian_rhs(N, 61), device="cuda")
    r2 = torch.tensor(inputs.gaussian_rhs(N, 62), device="cuda")
    z1, z2, z64 = torch.empty_like(r1), torch.empty_like(r1), torch.empty_like(r1)
    L.lor_apply_P(h, r1, z1)
    L.lor_apply_P(h, r2, z2)
    L.lor_apply_P(h64, r1, z64)
    torch.cuda.synchronize()
    e1, e2 = float(r1 @ z1), float(r2 @ z2)
    assert e1 > 0 and e2 > 0
    asym = abs(float(r2 @ z1) - float(r1 @ z2)) / np.sqrt(e1 * e2)
    err = float((z1 - z64).norm() / z64.norm())
    print(method, "DG asymmetry", asym, "float32 against float64", err, flush=True)
    assert asym <= 2e-5 and err <= 2e-5, (asym, err)
    x = torch.zeros_like(r1)
    info = L.lor_pcg_solve(h, r1, x, rtol=1e-8, maxit=1000)
    print(method, "DG iterations", info.iters, "true residual", info.rel_res_true, flush=True)
    assert info.status == L.LOR_OK and info.rel_res_true <= 1.05e-8

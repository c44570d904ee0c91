"""GPU parity on curved (isoparametric) meshes: the geometric factors from
the GLL node coordinates, the LOR hierarchy on those nodes and the
preconditioner against the oracle.  Node coordinates, stencils and orders
bit for bit; operator and B r within 1e-12 of the largest reference entry;
solves inside the oracle's iteration band."""
import numpy as np
import pytest

from oracle import highorder as HO, krylov, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [
    # dim, n, p, amp, perturb, seed, coefficient
    (2, 3, 3, 0.15, 0.1, 81, None),
    (2, 4, 5, 0.2, 0.0, 82, None),
    (3, 2, 3, 0.15, 0.1, 83, None),
    (3, 2, 6, 0.1, 0.1, 84, None),
    (2, 3, 4, 0.15, 0.1, 85, "b3"),
]


def _ids(c):
    return f"d{c[0]}-n{c[1]}-p{c[2]}-amp{c[3]}{'-' + c[6] if c[6] else ''}"


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "HIP device required"
    return torch


@pytest.fixture(scope="module")
def L():
    from paper_1908_07071_amd import lor
    return lor


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_curved_parity(case, L, torch_dev):
    torch = torch_dev
    dim, n, p, amp, pert, seed, cname = case
    print("case", case, flush=True)
    V = inputs.curved_vertices(dim, n, amp, pert, seed)
    X = inputs.curved_nodes(dim, n, p, amp, pert, seed)
    mesh = M.make_mesh(dim, [n] * dim, V, nodes=X, nodes_p=p)
    coef = None
    if cname:
        Xe = np.concatenate([X[HO.element_global_nodes(mesh, p, e)] for e in mesh.elements()])
        nq = (p + 1) ** dim
        coef = inputs.coefficient(cname, Xe, elem=np.repeat(np.arange(mesh.nel), nq)).reshape(mesh.nel, nq)
    h = L.lor_setup(dim, n, V, p, nodes=X, coef=coef)
    try:
        num = M.interior_numbering(M.grid_shape(mesh, p))
        assert np.array_equal(L.lor_dof_coords(h, dim), X[num >= 0])
        Xe = np.concatenate([X[HO.element_global_nodes(mesh, p, e)] for e in mesh.elements()])
        assert np.array_equal(L.lor_element_coords(h, dim, mesh.nel, p), Xe)
        B = S.SchwarzLOR(mesh, p, coef=coef)
        for k in range(B.H.nlevels):
            st = L.lor_export_stencils(h, k).reshape(3 ** dim, -1)
            assert np.array_equal(st, B.H.stencils[k].T), f"level {k}"
        order = L.lor_export_maps(h, L.LOR_MAP_ORDER)
        ooff = L.lor_export_maps(h, L.LOR_MAP_ORDER_OFFSET)
        t = 0
        for P in B.patches:
            for k in range(B.H.nlevels - 1):
                lv = P.levels[k]
                if lv["graph"] is not None:
                    assert np.array_equal(order[ooff[t]:ooff[t + 1]], lv["order"]), (P.v, k)
                t += 1
        K = HO.cg_stiffness(mesh, p, coef=coef)
        N = L.lor_ndofs(h)
        xin = inputs.uniform_vector(N, 5)
        x = torch.tensor(xin, device="cuda")
        y = torch.empty_like(x)
        z = torch.empty_like(x)
        L.lor_apply_A(h, x, y)
        L.lor_apply_P(h, x, z)
        torch.cuda.synchronize()
        ref = K @ xin
        assert np.abs(y.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
        zref = B.apply(xin)
        assert np.abs(z.cpu().numpy() - zref).max() <= 1e-12 * np.abs(zref).max()
        bin_ = inputs.gaussian_rhs(N, 6)
        b = torch.tensor(bin_, device="cuda")
        u = torch.zeros_like(b)
        info = L.lor_pcg_solve(h, b, u, rtol=1e-10, maxit=1000)
        lo, hi = krylov.iteration_band(K, bin_, B.apply, tol=1e-10)
        print("iterations", info.iters, "oracle band", lo, hi, flush=True)
        assert lo - 1 <= info.iters <= hi + 1, (info.iters, lo, hi)
        assert np.linalg.norm(bin_ - K @ u.cpu().numpy()) <= 1.05e-10 * np.linalg.norm(bin_)
    finally:
        L.lor_free(h)


def test_curved_dg_refused(L, torch_dev):
    V = inputs.curved_vertices(2, 2)
    X = inputs.curved_nodes(2, 2, 3)
    with pytest.raises(L.LorError) as e:
        L.lor_setup(2, 2, V, 3, method=L.LOR_IP, penalty=20.0, nodes=X)
    assert e.value.code == L.LOR_EINVAL

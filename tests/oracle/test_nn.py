"""Pins of the learned-correction reference (oracle/nn.py).

* conv3d equals scipy.ndimage.correlate (zero padding) channel pair by pair;
* conv3d_transpose is the adjoint of conv3d (dot-product identity);
* im2col @ W equals conv3d;
* the manual backward pass equals central finite differences of the loss;
* patch grids: interior patches fill the (2p-1)^3 grid, boundary patches the
  part inside the domain, consistent with the patch ranges;
* the training data are scale free (V_j is linear).
"""
import numpy as np
import pytest
from scipy import ndimage

from oracle import mesh as M, nn, schwarz as S
from paper_1908_07071_amd import inputs


def _rand_params(shapes, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal(s) * 0.3, rng.standard_normal(s[1]) * 0.1) for s in shapes]


def test_conv3d_is_zero_padded_cross_correlation():
    G, cin, cout = 5, 3, 2
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, G ** 3, cin))
    W = rng.standard_normal((27 * cin, cout))
    b = rng.standard_normal(cout)
    y = nn.conv3d(x, W, b, G)
    for n in range(2):
        for o in range(cout):
            ref = np.full((G, G, G), b[o])
            for c in range(cin):
                ker = np.zeros((3, 3, 3))  # [dz, dy, dx]
                for k, (dx, dy, dz) in enumerate(nn.offsets()):
                    ker[dz + 1, dy + 1, dx + 1] = W[k * cin + c, o]
                ref += ndimage.correlate(x[n, :, c].reshape(G, G, G), ker, mode="constant", cval=0.0)
            assert np.allclose(y[n, :, o].reshape(G, G, G), ref, rtol=1e-13, atol=1e-13)


def test_transpose_is_adjoint_and_im2col_matches():
    G, cin, cout = 4, 2, 3
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, G ** 3, cin))
    dy = rng.standard_normal((3, G ** 3, cout))
    W = rng.standard_normal((27 * cin, cout))
    lhs = np.sum(nn.conv3d(x, W, np.zeros(cout), G) * dy)
    rhs = np.sum(x * nn.conv3d_transpose(dy, W, G, cin))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    cols = nn.im2col(x, G)
    assert np.allclose(cols @ W, nn.conv3d(x, W, np.zeros(cout), G), rtol=1e-13, atol=1e-13)


def test_gradients_match_finite_differences():
    G, C = 5, 3
    shapes = nn.layer_shapes(C)
    params = _rand_params(shapes, 3)
    rng = np.random.default_rng(4)
    X = np.zeros((2, G ** 3, 2))
    X[:, :, 0] = rng.standard_normal((2, G ** 3))
    X[:, :, 1] = (rng.random((2, G ** 3)) > 0.2).astype(float)
    T = rng.standard_normal((2, G ** 3))
    loss, grads = nn.loss_and_grads(params, X, T, G)
    vec = nn.flatten(params)
    gvec = nn.flatten(grads)
    h = 1e-6
    for i in rng.choice(len(vec), 40, replace=False):
        vp, vm = vec.copy(), vec.copy()
        vp[i] += h
        vm[i] -= h
        lp, _ = nn.loss_and_grads(nn.unflatten(vp, shapes), X, T, G)
        lm, _ = nn.loss_and_grads(nn.unflatten(vm, shapes), X, T, G)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gvec[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gvec[i])


@pytest.mark.parametrize("n,p", [(3, 3), (2, 4)])
def test_patch_grids(n, p):
    V = inputs.structured_vertices(3, n, 0.1, seed=5)
    mesh = M.make_mesh(3, [n] * 3, V)
    G = 2 * p - 1
    for v in S.vertices(mesh):
        _, q = nn.patch_grid(mesh, p, v)
        rng = S.patch_ranges(mesh, p, v)
        cnt = int(np.prod([hi - lo + 1 for lo, hi in rng]))
        assert len(q) == cnt == len(np.unique(q))
        assert q.min() >= 0 and q.max() < G ** 3
        if all(0 < v[i] < n for i in range(3)):
            assert cnt == G ** 3


def test_training_data_scale_free():
    V = inputs.structured_vertices(3, 2, 0.1, seed=6)
    mesh = M.make_mesh(3, [2, 2, 2], V)
    B = S.SchwarzLOR(mesh, 3)
    r = inputs.gaussian_rhs(B.Kh.shape[0], 7)
    X1, T1, s1 = nn.patch_samples(B, r)
    X2, T2, s2 = nn.patch_samples(B, 3.0 * r)
    assert np.allclose(X1, X2, rtol=1e-13, atol=1e-15) and np.allclose(T1, T2, rtol=1e-12, atol=1e-14)
    assert np.allclose(s2, 3.0 * s1, rtol=1e-13)
    # scale * target scattered back is the patch part of the preconditioner
    z = np.zeros_like(r)
    for j, P in enumerate(B.patches):
        lv = P.levels[0]
        if lv["graph"] is None:
            continue
        _, q = nn.patch_grid(mesh, 3, P.v)
        z[B.fnum[lv["flat"]]] += s1[j] * T1[j, q]
    assert np.allclose(z, B.apply(r, with_coarse=False), rtol=1e-12, atol=1e-14)


def test_warmstart_reduces_to_known_preconditioners():
    """WARMSTART z_j = y_j + V_j(r_j - A_j y_j): a zero network gives the
    V-cycle Schwarz preconditioner; an exact local prediction y_j = A_j^-1 r_j
    leaves nothing for the V-cycle and gives Schwarz with exact local solves;
    a V-cycle prediction gives two V-cycle Richardson steps per patch."""
    V = inputs.structured_vertices(3, 2, 0.1, seed=8)
    mesh = M.make_mesh(3, [2, 2, 2], V)
    p = 3
    B = S.SchwarzLOR(mesh, p)
    r = inputs.gaussian_rhs(B.Kh.shape[0], 9)
    zero = [(np.zeros(s), np.zeros(s[1])) for s in nn.layer_shapes(4)]
    assert np.allclose(nn.preconditioner_warmstart(B, zero, r), B.apply(r), rtol=1e-13, atol=1e-14)
    exact = S.SchwarzLOR(mesh, p, exact_local=True)
    z = nn.preconditioner_warmstart(B, None, r,
                                    predictor=lambda j, P, rj: np.linalg.solve(P.levels[0]["A"], rj))
    assert np.allclose(z, exact.apply(r), rtol=1e-11, atol=1e-13)
    def two_steps(j, P, rj):
        return P.solve(rj)
    z2 = nn.preconditioner_warmstart(B, None, r, predictor=two_steps)
    ref = B.coarse.apply(r)
    for P in B.patches:
        lv = P.levels[0]
        if lv["graph"] is None:
            continue
        u = B.fnum[lv["flat"]]
        x1 = P.solve(r[u])
        ref[u] += x1 + P.solve(r[u] - lv["A"] @ x1)
    assert np.allclose(z2, ref, rtol=1e-13, atol=1e-14)
    assert not np.allclose(z2, B.apply(r), rtol=1e-6)

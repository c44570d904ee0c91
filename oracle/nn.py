"""Learned patch correction: the float64 reference (test infrastructure only).

A small 3D convolutional network acts on one vertex patch at a time.  Its
input lives on the padded level-0 patch grid of G = 2p - 1 points per
direction (the size of an interior-vertex patch; a boundary-vertex patch
occupies the part of the grid inside the domain).  Grid point g_i in
direction i is the level-0 grid node v_i p - p + 1 + g_i.  Two input
channels: the patch residual divided by its 2-norm, and the mask (1 where
the patch has an unknown).  The target is the patch V-cycle applied to the
same residual (Section 3.3), divided by the same norm; V_j is linear, so the
network sees scale-free data.  Layers: 3x3x3 cross-correlations with zero
padding and a bias per output channel, ReLU between layers, and the output
multiplied by the mask.  Loss: mean squared error over the masked points.

Layouts (shared with the GPU kernels): activations [B, G^3, C] with the grid
point index q = gx + G (gy + G gz); weights of a layer as a matrix
[27 Cin, Cout] with row k Cin + c, k = (dx+1) + 3 (dy+1) + 9 (dz+1) the
kernel offset and c the input channel.
"""
from __future__ import annotations

import numpy as np

from . import mesh as _mesh
from . import schwarz as _sw


def offsets():
    """The 27 kernel offsets (dx, dy, dz), x fastest."""
    return [(k % 3 - 1, (k // 3) % 3 - 1, k // 9 - 1) for k in range(27)]


def patch_grid(mesh, p: int, v):
    """(G, grid point of each level-0 patch unknown in the patch's unknown order)."""
    G = 2 * p - 1
    rng = _sw.patch_ranges(mesh, p, v)
    shape = [hi - lo + 1 for lo, hi in rng]
    if min(shape) <= 0:
        return G, np.zeros(0, np.int64)
    idx = np.indices(shape).reshape(mesh.dim, -1, order="F")
    q = np.zeros(idx.shape[1], np.int64)
    stride = 1
    for i in range(mesh.dim):
        g = idx[i] + rng[i][0] - (v[i] * p - p + 1)
        q += g * stride
        stride *= G
    return G, q


def patch_samples(B: "_sw.SchwarzLOR", r: np.ndarray):
    """Network inputs, targets and scales of every patch for the global
    residual r (L-vector): X [J, G^3, 2], T [J, G^3], scale [J]."""
    mesh, p = B.H.mesh, B.H.p
    G = 2 * p - 1
    J = len(B.patches)
    X = np.zeros((J, G ** mesh.dim, 2))
    T = np.zeros((J, G ** mesh.dim))
    scale = np.ones(J)
    for j, P in enumerate(B.patches):
        lv = P.levels[0]
        if lv["graph"] is None:
            continue
        _, q = patch_grid(mesh, p, P.v)
        u = B.fnum[lv["flat"]]
        rj = r[u]
        s = np.linalg.norm(rj)
        s = s if s > 0 else 1.0
        scale[j] = s
        X[j, q, 0] = rj / s
        X[j, q, 1] = 1.0
        T[j, q] = P.solve(rj) / s
    return X, T, scale


def conv3d(x: np.ndarray, W: np.ndarray, b: np.ndarray, G: int) -> np.ndarray:
    """y[n, q, o] = b[o] + sum_k sum_c x[n, q + off(k), c] W[k Cin + c, o]
    (zero outside the G^3 grid)."""
    nb, npt, cin = x.shape
    xg = x.reshape(nb, G, G, G, cin)          # [n, z, y, x, c]
    y = np.zeros((nb, G, G, G, W.shape[1])) + b
    for k, (dx, dy, dz) in enumerate(offsets()):
        src = np.zeros_like(xg)
        zs, ys, xs = [slice(max(0, -d), G - max(0, d)) for d in (dz, dy, dx)]
        zt, yt, xt = [slice(max(0, d), G + min(0, d)) for d in (dz, dy, dx)]
        src[:, zs, ys, xs] = xg[:, zt, yt, xt]  # src[q] = x[q + off]
        y += src @ W[k * cin:(k + 1) * cin]
    return y.reshape(nb, npt, -1)


def conv3d_transpose(dy: np.ndarray, W: np.ndarray, G: int, cin: int) -> np.ndarray:
    """Adjoint of conv3d in its input: dx[n, q', c] = sum_k sum_o
    dy[n, q' - off(k), o] W[k Cin + c, o]."""
    nb, npt, cout = dy.shape
    dg = dy.reshape(nb, G, G, G, cout)
    dx = np.zeros((nb, G, G, G, cin))
    for k, (dx_, dy_, dz_) in enumerate(offsets()):
        contrib = dg @ W[k * cin:(k + 1) * cin].T  # at q: contribution to x[q + off]
        zs, ys, xs = [slice(max(0, -d), G - max(0, d)) for d in (dz_, dy_, dx_)]
        zt, yt, xt = [slice(max(0, d), G + min(0, d)) for d in (dz_, dy_, dx_)]
        dx[:, zt, yt, xt] += contrib[:, zs, ys, xs]
    return dx.reshape(nb, npt, cin)


def im2col(x: np.ndarray, G: int) -> np.ndarray:
    """[n, q, k Cin + c] = x[n, q + off(k), c] (zero outside the grid)."""
    nb, npt, cin = x.shape
    xg = x.reshape(nb, G, G, G, cin)
    cols = np.zeros((nb, G, G, G, 27 * cin))
    for k, (dx, dy, dz) in enumerate(offsets()):
        zs, ys, xs = [slice(max(0, -d), G - max(0, d)) for d in (dz, dy, dx)]
        zt, yt, xt = [slice(max(0, d), G + min(0, d)) for d in (dz, dy, dx)]
        cols[:, zs, ys, xs, k * cin:(k + 1) * cin] = xg[:, zt, yt, xt]
    return cols.reshape(nb, npt, 27 * cin)


def forward(params, X: np.ndarray, G: int):
    """Network output [n, G^3] and the per-layer (input, pre-activation)."""
    mask = X[:, :, 1]
    a = X
    cache = []
    for li, (W, b) in enumerate(params):
        z = conv3d(a, W, b, G)
        cache.append((a, z))
        a = np.maximum(z, 0.0) if li + 1 < len(params) else z
    return a[:, :, 0] * mask, cache


def loss_and_grads(params, X: np.ndarray, T: np.ndarray, G: int):
    """Masked mean squared error and its gradients (manual backward pass)."""
    mask = X[:, :, 1]
    y, cache = forward(params, X, G)
    m = mask.sum()
    diff = (y - T) * mask
    loss = float((diff ** 2).sum() / m)
    dz = (2.0 * diff / m * mask)[:, :, None]
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        a, z = cache[li]
        W, b = params[li]
        cin = a.shape[2]
        cols = im2col(a, G).reshape(-1, 27 * cin)
        dW = cols.T @ dz.reshape(-1, W.shape[1])
        db = dz.reshape(-1, W.shape[1]).sum(axis=0)
        grads[li] = (dW, db)
        if li > 0:
            da = conv3d_transpose(dz, W, G, cin)
            dz = da * (cache[li - 1][1] > 0)
    return loss, grads


def flatten(params) -> np.ndarray:
    """Parameter vector: W1, b1, W2, b2, ... (row-major)."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(vec: np.ndarray, shapes):
    """Inverse of flatten for layer shapes [(27 Cin, Cout), ...]."""
    out, o = [], 0
    for (k, n) in shapes:
        W = vec[o:o + k * n].reshape(k, n)
        o += k * n
        b = vec[o:o + n].copy()
        o += n
        out.append((W.copy(), b))
    return out


def layer_shapes(channels: int, cin: int = 2, layers: int = 3):
    shapes, c = [], cin
    for li in range(layers):
        co = 1 if li == layers - 1 else channels
        shapes.append((27 * c, co))
        c = co
    return shapes


def preconditioner_replace(B: "_sw.SchwarzLOR", params, r: np.ndarray) -> np.ndarray:
    """z = coarse correction + sum_j R_j^T (scale_j net(r_j / scale_j)):
    the network stands in for every patch V-cycle (eq. as otherwise)."""
    mesh, p = B.H.mesh, B.H.p
    G = 2 * p - 1
    X, _, scale = _inputs_only(B, r)
    y, _ = forward(params, X, G)
    z = B.coarse.apply(r) if B.coarse is not None else np.zeros_like(r)
    for j, P in enumerate(B.patches):
        lv = P.levels[0]
        if lv["graph"] is None:
            continue
        _, q = patch_grid(mesh, p, P.v)
        u = B.fnum[lv["flat"]]
        z[u] += scale[j] * y[j, q]
    return z


def preconditioner_warmstart(B: "_sw.SchwarzLOR", params, r: np.ndarray, predictor=None) -> np.ndarray:
    """z = coarse correction + sum_j R_j^T (y_j + V_j(r_j - A_j y_j)): the
    prediction y_j = scale_j net(r_j / scale_j) starts each patch solve and
    one V-cycle corrects it (A_j the patch's level-0 LOR matrix).
    predictor(j, P, r_j) -> y_j replaces the network when given (pins)."""
    mesh, p = B.H.mesh, B.H.p
    G = 2 * p - 1
    if predictor is None:
        X, _, scale = _inputs_only(B, r)
        y, _ = forward(params, X, G)
    z = B.coarse.apply(r) if B.coarse is not None else np.zeros_like(r)
    for j, P in enumerate(B.patches):
        lv = P.levels[0]
        if lv["graph"] is None:
            continue
        u = B.fnum[lv["flat"]]
        rj = r[u]
        if predictor is None:
            _, q = patch_grid(mesh, p, P.v)
            yj = scale[j] * y[j, q]
        else:
            yj = predictor(j, P, rj)
        z[u] += yj + P.solve(rj - lv["A"] @ yj)
    return z


def _inputs_only(B, r):
    mesh, p = B.H.mesh, B.H.p
    G = 2 * p - 1
    J = len(B.patches)
    X = np.zeros((J, G ** mesh.dim, 2))
    scale = np.ones(J)
    for j, P in enumerate(B.patches):
        lv = P.levels[0]
        if lv["graph"] is None:
            continue
        _, q = patch_grid(mesh, p, P.v)
        rj = r[B.fnum[lv["flat"]]]
        s = np.linalg.norm(rj)
        scale[j] = s if s > 0 else 1.0
        X[j, q, 0] = rj / scale[j]
        X[j, q, 1] = 1.0
    return X, None, scale

"""Host emulation of the index arithmetic of the degree-templated coarse
restriction (csrc/k_setup.hip, k_coarse_restrict_p): the 64 lanes of a
wavefront, each taking every 64th point of the flattened (2p-1)^d support,
visit every support point of the vertex exactly once, every read stays
inside the unknowns of a Dirichlet grid, and the hat weights are read at
offsets below 2p-1 (the LDS table's size).  The expressions mirror the
kernel's (this file changes with it)."""
import itertools

import pytest


@pytest.mark.parametrize("P", range(1, 9))
@pytest.mark.parametrize("dim", [2, 3])
def test_restrict_support_and_bounds(P, dim):
    W1 = 2 * P - 1
    W = W1 ** dim
    NQ = (W + 63) // 64
    for n in ([2] * dim, [3, 2, 4][:dim], [5, 1, 3][:dim] if dim == 3 else [5, 3]):
        if min(n) < 2:
            continue  # no interior vertex in that direction: no coarse space
        nu = [m * P - 1 for m in n]
        sy = nu[0]
        sz = nu[0] * nu[1]
        ncx, ncy = n[0] - 1, n[1] - 1
        nc = ncx * ncy * (n[2] - 1 if dim == 3 else 1)
        N = sz * (nu[2] if dim == 3 else 1)
        for c in range(nc):
            v = [c % ncx + 1, (c // ncx) % ncy + 1, c // (ncx * ncy) + 1 if dim == 3 else 0]
            base = (v[0] - 1) * P + sy * ((v[1] - 1) * P) + (sz * ((v[2] - 1) * P) if dim == 3 else 0)
            seen = set()
            for lane, k in itertools.product(range(64), range(NQ)):
                q = lane + 64 * k
                if q >= W:
                    continue
                ox, oy = q % W1, (q // W1) % W1
                oz = q // (W1 * W1) if dim == 3 else 0
                assert max(ox, oy, oz) < W1
                seen.add((ox, oy, oz))
                idx = base + ox + sy * oy + sz * oz
                assert 0 <= idx < N, (P, dim, n, c, q)
                # the point lies in the vertex's support: within P-1 grid steps of the vertex
                g = [(v[0] - 1) * P + ox + 1, (v[1] - 1) * P + oy + 1]
                assert all(abs(gd - vd * P) <= P - 1 for gd, vd in zip(g, v[:2]))
            want = set(itertools.product(range(W1), range(W1), range(W1) if dim == 3 else [0]))
            assert seen == want

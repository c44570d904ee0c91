"""Host emulation of the index arithmetic of the skeleton gather
(csrc/k_operator.hip, k_skeleton_gather): its three parts (every node of
the grid planes whose z coordinate is an element interface, every node of
the other planes' interface lines in y, the rest of those planes' nodes
with an interface x coordinate) enumerate each skeleton node of the
unknowns exactly once, for Dirichlet and Neumann grids, and every element
read (up to 8 per node, local index on a face where the node lies on one)
contains the node and stays inside the element-ordered buffer.  The
expressions mirror the kernel's (this file changes with it)."""
import itertools

import pytest


def parts(n, p, dirichlet):
    ox = 1 if dirichlet else 0
    nu = [m * p + 1 - 2 * ox for m in n]
    f = -1 if dirichlet else 1
    fx, fy, fz = n[0] + f, n[1] + f, n[2] + f
    nA = fz * nu[0] * nu[1]
    nB = (nu[2] - fz) * fy * nu[0]
    nC = (nu[2] - fz) * (nu[1] - fy) * fx
    return ox, nu, (fx, fy, fz), (nA, nB, nC)


def node_of(t, n, p, dirichlet):
    ox, nu, (fx, fy, fz), (nA, nB, nC) = parts(n, p, dirichlet)
    face = lambda k: (k + ox) * p
    inner = lambda k: k + k // (p - 1) + 1
    nx, ny = nu[0], nu[1]
    if t < nA:
        per = nx * ny
        kz = t // per; rem = t - kz * per; iy = rem // nx
        return (rem - iy * nx + ox, iy + ox, face(kz))
    t -= nA
    if t < nB:
        per = fy * nx
        kz = t // per; rem = t - kz * per; ky = rem // nx
        return (rem - ky * nx + ox, face(ky), inner(kz))
    t -= nB
    if t < nC:
        per = (ny - fy) * fx
        kz = t // per; rem = t - kz * per; ky = rem // fx
        return (face(rem - ky * fx), inner(ky), inner(kz))
    return None


def reads(g, n, p):
    out = []
    for cb in range(8):
        e, l, ok = [0] * 3, [0] * 3, True
        for d in range(3):
            if (cb >> d) & 1 == 0:
                e[d] = g[d] // p
                l[d] = g[d] - e[d] * p
                if e[d] >= n[d]:
                    ok = False
            else:
                if g[d] % p != 0 or g[d] == 0:
                    ok = False
                e[d] = g[d] // p - 1
                l[d] = p
        if ok:
            out.append((tuple(e), tuple(l)))
    return out


@pytest.mark.parametrize("n", [(1, 1, 1), (2, 1, 3), (3, 2, 2), (4, 4, 4), (1, 3, 2), (5, 2, 1)])
@pytest.mark.parametrize("p", [4, 5, 6, 7])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_skeleton_enumeration(n, p, dirichlet):
    ox, nu, _, (nA, nB, nC) = parts(n, p, dirichlet)
    got = [node_of(t, n, p, dirichlet) for t in range(nA + nB + nC)]
    assert node_of(nA + nB + nC, n, p, dirichlet) is None
    assert len(got) == len(set(got))
    want = {g for g in itertools.product(*[range(ox, ox + m) for m in nu])
            if any(c % p == 0 for c in g)}
    assert set(got) == want
    for g in got:
        rd = reads(g, n, p)
        assert rd, g
        for e, l in rd:
            assert all(0 <= e[d] < n[d] and 0 <= l[d] <= p for d in range(3))
            assert all(e[d] * p + l[d] == g[d] for d in range(3))  # the element holds the node
        # every element holding the node is read once
        holders = {tuple(e) for e in itertools.product(*[range(m) for m in n])
                   if all(e[d] * p <= g[d] <= e[d] * p + p for d in range(3))}
        assert {e for e, _ in rd} == holders and len(rd) == len(holders)

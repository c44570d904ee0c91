"""Host check of the patch kernel's LDS layout (no GPU).  A patch keeps X_0
and R_0 of its finest level in LDS, B_1 beside them, and every coarser
vector (X_1, R_1, then X_k, B_k, R_k for k >= 2) inside R_0's space, which
is unused from the restriction to level 1 until the level-0 residual after
the prolongation.  That is valid when, for every patch shape (each
direction interior, 2 s_k - 1 points, or on the boundary, s_k - 1),
2 n_1 + 3 sum_{k>=2} n_k <= n_0.  With the kept-point rule of Section 3.3
it holds for every supported degree; the LDS need 2 n_0 + n_1 of the
largest patch (plus a 64-byte slot table) then fits the 160 KiB of a CU up
to the degrees that include/lor.h states (3D: p <= 11 in float64, p <= 13
in float32)."""
import itertools

import pytest

from oracle import lor as OL

LDS_BYTES = 160 * 1024


def _level_points(s_k, interior):
    n = 1
    for it in interior:
        n *= max(2 * s_k - 1 if it else s_k - 1, 0)
    return n


@pytest.mark.parametrize("dim", [2, 3])
def test_coarse_levels_fit_in_the_level0_residual(dim):
    for p in range(1, 15):
        s = OL.level_sizes(p)
        for interior in itertools.product([False, True], repeat=dim):
            n = [_level_points(sk, interior) for sk in s]
            coarse = (2 * n[1] if len(n) > 1 else 0) + 3 * sum(n[2:])
            assert coarse <= n[0], (p, dim, interior, n)


def test_lds_need_and_documented_degree_limits():
    def need(p, dim, bytes_per_value):
        s = OL.level_sizes(p)
        n = [_level_points(sk, (True,) * dim) for sk in s]
        # plus the 64-byte slot table of the sweep records
        return (2 * n[0] + (n[1] if len(n) > 1 else 0)) * bytes_per_value + 64

    fits = {(dim, b): [p for p in range(1, 15) if need(p, dim, b) <= LDS_BYTES] for dim in (2, 3) for b in (4, 8)}
    assert fits[(2, 4)] == list(range(1, 15)) and fits[(2, 8)] == list(range(1, 15))
    assert fits[(3, 8)] == list(range(1, 12))   # float64: p <= 11
    assert fits[(3, 4)] == list(range(1, 14))   # float32: p <= 13
    # the benchmark's p = 6 patch: 11.2 KB in float (14 per CU in 160 KiB,
    # 512-byte granules included), 22.4 KB in float64 (7 per CU)
    assert need(6, 3, 4) == 11212 and need(6, 3, 8) == 22360
    assert 14 * ((11212 + 511) // 512 * 512) <= LDS_BYTES

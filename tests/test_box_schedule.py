"""Host emulation of the step order of the one-workgroup box V-cycle
(csrc/k_single.hip, k_box_vcycle) against the recursive V-cycle of the
per-level launches (csrc/box_patch.cpp, vcycle): for every pattern of empty
and non-empty levels, both run the same steps on the same levels in the
same order (pre-smoothing sweeps, residual, restriction down to the deepest
level reached; the exact solve when that level is the last one; then
prolongation, residual and post-smoothing back up).  The expressions mirror
the two codes (this file changes with them)."""
import itertools

import pytest


def recursive(n, L):
    ops = []

    def vc(k):
        if n[k] <= 0:
            return
        if k == L - 1:
            ops.append(("solve", k))
            return
        ops.extend([("fwd", k), ("bwd", k), ("res", k)])
        if n[k + 1] > 0:
            ops.append(("restrict", k))
            vc(k + 1)
            ops.extend([("prolong", k), ("res", k)])
        ops.extend([("fwd_post", k), ("bwd_post", k), ("axpy", k)])

    vc(0)
    return ops


def one_workgroup(n, L):
    ops = []
    if n[0] <= 0:
        return ops
    K = 0
    while K < L - 1 and n[K + 1] > 0:
        K += 1
    top = min(K, L - 2)
    for k in range(0, top + 1):
        ops += [("fwd", k), ("bwd", k), ("res", k)]
        if k < K:
            ops.append(("restrict", k))
    if K == L - 1:
        ops.append(("solve", K))
    for k in range(top, -1, -1):
        if k < K:
            ops += [("prolong", k), ("res", k)]
        ops += [("fwd_post", k), ("bwd_post", k), ("axpy", k)]
    return ops


@pytest.mark.parametrize("L", range(1, 7))
def test_same_steps_for_every_level_pattern(L):
    for pattern in itertools.product([0, 5], repeat=L):
        n = list(pattern)
        assert one_workgroup(n, L) == recursive(n, L), n

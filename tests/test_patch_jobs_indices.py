"""Host emulation of the work decomposition of the multi-problem patch
launch (csrc/k_schwarz.hip: launch_patch_vcycle_jobs and the block decode
at the top of k_patch_vcycle): for random jobs (patch counts, right-hand
sides per problem, up to four problems), every block finds a job, every
(problem, right-hand side, patch) work item is run by exactly one block,
blocks past a problem's last patch return, and the blocks of one patch's
right-hand sides sit in the same group of 8 consecutive blocks modulo
8 * nrhs (so that consecutive dispatches reach the same XCD).  The
expressions mirror the kernel's and the launcher's (this file changes with
them)."""
import random

K_MAX_JOBS, K_MAX_RHS = 4, 4


def plan(jobs):
    block0, blocks = [], 0
    for J, nrhs in jobs:
        block0.append(blocks)
        blocks += (J + 7) // 8 * 8 * nrhs
    block0.append(blocks)
    return block0, blocks


def decode(b, jobs, block0):
    job, blk = 0, b
    while job + 1 < len(jobs) and blk >= block0[job + 1]:
        job += 1
    blk -= block0[job]
    J, nrhs = jobs[job]
    t = blk >> 3
    k = t % nrhs
    slot = (t // nrhs) * 8 + (blk & 7)
    if slot >= J:
        return None
    return job, k, slot


def test_every_work_item_once():
    rng = random.Random(5)
    for _ in range(300):
        jobs = [(rng.randint(1, 200), rng.randint(1, K_MAX_RHS)) for _ in range(rng.randint(1, K_MAX_JOBS))]
        block0, blocks = plan(jobs)
        seen = {}
        for b in range(blocks):
            d = decode(b, jobs, block0)
            if d is None:
                continue
            assert d not in seen, (jobs, b, d)
            seen[d] = b
        want = {(j, k, s) for j, (J, nrhs) in enumerate(jobs) for k in range(nrhs) for s in range(J)}
        assert set(seen) == want
        for (j, k, s), b in seen.items():
            # the right-hand sides of one patch: block numbers differ by multiples of 8
            b0 = seen[(j, 0, s)]
            assert (b - b0) % 8 == 0 and abs(b - b0) < 8 * jobs[j][1]

"""The float64 matrix-core product behind the coarse inverse's set-up
(blocked Gauss-Jordan, Section 3.2), through the C ABI against numpy:
ragged sizes around the 64 x 64 tile and the 16-deep K chunk, leading
dimensions larger than the rows, alpha / beta combinations, beta = 0 not
reading C, and the argument checks.  The coarse inverse itself is covered
by every preconditioner parity test."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "HIP device required"
    return torch


@pytest.fixture(scope="module")
def L():
    from paper_1908_07071_amd import lor
    return lor


# m, n, k, extra leading-dimension padding, alpha, beta
CASES = [
    (1, 1, 1, 0, 1.0, 0.0),
    (70, 33, 7, 3, 1.0, 0.0),
    (64, 64, 16, 0, -1.0, 1.0),
    (130, 257, 128, 5, 0.5, 2.0),
    (257, 65, 129, 1, 1.0, -0.25),
    (5, 300, 3, 0, -1.0, 1.0),
    (17, 9, 0, 2, 1.0, 3.0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "m{}-n{}-k{}".format(*c[:3]))
def test_f64_gemm_matches_numpy(case, L, torch_dev):
    torch = torch_dev
    m, n, k, pad, alpha, beta = case
    print("case", case, flush=True)
    rng = np.random.default_rng(m * 1000 + n * 10 + k)
    lda, ldb, ldc = k + pad, n + pad, n + pad
    A = rng.standard_normal((m, lda))
    B = rng.standard_normal((max(k, 1), ldb))
    C0 = rng.standard_normal((m, ldc))
    if beta == 0.0:
        C0[:, :n] = np.nan  # must not be read
    ref = C0.copy()
    ref[:, :n] = alpha * (A[:, :k] @ B[:k, :n]) + (beta * C0[:, :n] if beta != 0.0 else 0.0)
    At = torch.tensor(A.ravel(), device="cuda")
    Bt = torch.tensor(B.ravel(), device="cuda")
    Ct = torch.tensor(C0.ravel(), device="cuda")
    L.lor_f64_gemm(m, n, k, alpha, At, lda, Bt, ldb, beta, Ct, ldc)
    torch.cuda.synchronize()
    got = Ct.cpu().numpy().reshape(m, ldc)
    assert np.all(np.isfinite(got[:, :n]))
    # columns past n untouched
    assert np.array_equal(got[:, n:], C0[:, n:])
    scale = max(1.0, np.abs(ref[:, :n]).max())
    err = np.abs(got[:, :n] - ref[:, :n]).max() / scale
    print("max error", err, flush=True)
    assert err <= 1e-13, err


def test_f64_gemm_argument_checks(L, torch_dev):
    torch = torch_dev
    A = torch.zeros(64, dtype=torch.float64, device="cuda")
    for args in [(4, 4, 4, 1.0, A, 3, A, 4, 0.0, A, 4),   # lda < k
                 (4, 4, 4, 1.0, A, 4, A, 3, 0.0, A, 4),   # ldb < n
                 (4, 4, 4, 1.0, A, 4, A, 4, 0.0, A, 3),   # ldc < n
                 (-1, 4, 4, 1.0, A, 4, A, 4, 0.0, A, 4)]:
        with pytest.raises(L.LorError) as ei:
            L.lor_f64_gemm(*args)
        assert ei.value.code == L.LOR_EINVAL

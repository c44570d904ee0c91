"""The no-allocation preconditioner entry point lor_apply_P_noalloc against
lor_apply_P through the C ABI: the same z = B r (eq. as; eq. dg-as for DG)
to the float64 parity tolerance (1e-12 of the largest entry; the patch
corrections are summed with float64 atomics, so the last bits may differ),
on two calls in a row, the second with a smaller input, and a handle whose
scratch does not fit refused with LOR_ENOMEM before any launch."""
import numpy as np
import pytest

from paper_1908_07071_amd import inputs

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


def _compare(L, torch, h, seed):
    N = L.lor_ndofs(h)
    r = torch.tensor(inputs.gaussian_rhs(N, seed), device="cuda")
    z_ref = torch.empty_like(r)
    z = torch.full_like(r, float("nan"))
    L.lor_apply_P(h, r, z_ref)
    L.lor_apply_P_noalloc(h, r, z)
    torch.cuda.synchronize()
    a, b = z.cpu().numpy(), z_ref.cpu().numpy()
    assert np.all(np.isfinite(a))
    err = np.abs(a - b).max() / np.abs(b).max()
    print("N", N, "max rel difference", err, flush=True)
    assert err <= 1e-12, err


def test_noalloc_matches_apply_P_twice_then_smaller(L, torch_dev):
    torch = torch_dev
    # first call: DG (coarse and conforming scratch vectors), 3 x 3 x 2, p = 4
    V1 = inputs.structured_vertices(3, [3, 3, 2], 0.1, seed=21)
    h1 = L.lor_setup(3, [3, 3, 2], V1, 4, method=L.LOR_IP, penalty=40.0)
    # second call: a smaller CG problem (coarse scratch only), 2^3, p = 3
    V2 = inputs.structured_vertices(3, 2, 0.1, seed=22)
    h2 = L.lor_setup(3, 2, V2, 3)
    try:
        n1, cap = L.lor_noalloc_scratch_bytes(h1)
        n2, _ = L.lor_noalloc_scratch_bytes(h2)
        assert 0 < n2 < n1 <= cap
        _compare(L, torch, h1, 5)
        _compare(L, torch, h2, 6)
        # and back to the larger one: nothing left over from the last call matters
        _compare(L, torch, h1, 7)
    finally:
        L.lor_free(h1)
        L.lor_free(h2)


def test_noalloc_mixed_precision(L, torch_dev):
    torch = torch_dev
    V = inputs.structured_vertices(3, 3, 0.1, seed=23)
    opt = L.lor_default_options()
    opt.precision = L.LOR_PREC_MIXED
    h = L.lor_setup(3, 3, V, 5, options=opt)
    try:
        _compare(L, torch, h, 8)
    finally:
        L.lor_free(h)


def test_noalloc_rejects_oversized_handle(L, torch_dev):
    """A DG handle whose conforming vectors exceed the static scratch:
    LOR_ENOMEM with the sizes in the detail, z untouched."""
    torch = torch_dev
    V = inputs.structured_vertices(3, 14, 0.0)
    h = L.lor_setup(3, 14, V, 6, method=L.LOR_BR2, penalty=10.0)
    try:
        need, cap = L.lor_noalloc_scratch_bytes(h)
        assert need > cap
        N = L.lor_ndofs(h)
        r = torch.ones(N, dtype=torch.float64, device="cuda")
        z = torch.zeros_like(r)
        with pytest.raises(L.LorError) as e:
            L.lor_apply_P_noalloc(h, r, z)
        assert e.value.code == L.LOR_ENOMEM
        assert "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert float(z.abs().max()) == 0.0
    finally:
        L.lor_free(h)

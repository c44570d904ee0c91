"""Pins of the GLL basis (Section 3.1: nodal basis and G-NI quadrature at the
Gauss-Lobatto points) against closed forms and exactness properties."""
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import gll


def _rounded(expr):
    getcontext().prec = 60
    return float(expr)


def test_closed_forms_bit_exact():
    getcontext().prec = 60
    half = Decimal(1) / 2
    # p = 2: {0, 1/2, 1}, weights {1/6, 2/3, 1/6}
    x, w = gll.gll(2)
    assert list(x) == [0.0, 0.5, 1.0]
    assert list(w) == [_rounded(Decimal(1) / 6), _rounded(Decimal(2) / 3), _rounded(Decimal(1) / 6)]
    # p = 3: (1 -+ 1/sqrt5)/2, weights {1/12, 5/12, 5/12, 1/12}
    x, w = gll.gll(3)
    r5 = 1 / Decimal(5).sqrt()
    assert list(x) == [0.0, _rounded(half - half * r5), _rounded(half + half * r5), 1.0]
    assert list(w) == [_rounded(Decimal(1) / 12), _rounded(Decimal(5) / 12)] * 1 + \
        [_rounded(Decimal(5) / 12), _rounded(Decimal(1) / 12)]
    # p = 4: (1 -+ sqrt(3/7))/2, weights {1/20, 49/180, 16/45, 49/180, 1/20}
    x, w = gll.gll(4)
    r = (Decimal(3) / 7).sqrt()
    assert list(x) == [0.0, _rounded(half - half * r), 0.5, _rounded(half + half * r), 1.0]
    assert list(w) == [_rounded(Decimal(1) / 20), _rounded(Decimal(49) / 180), _rounded(Decimal(16) / 45),
                       _rounded(Decimal(49) / 180), _rounded(Decimal(1) / 20)]


@pytest.mark.parametrize("p", range(1, 15))
def test_quadrature_exactness(p):
    x, w = gll.gll(p)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(np.diff(x) > 0) and x[0] == 0.0 and x[-1] == 1.0
    # symmetric about 1/2
    assert np.allclose(x + x[::-1], 1.0, atol=1e-15, rtol=0)
    # exact for polynomials of degree <= 2p - 1 on [0,1] ...
    for k in range(2 * p):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-14, k
    # ... and not for degree 2p (Lobatto rules have degree exactly 2p - 1)
    if p <= 8:
        assert abs(np.sum(w * x ** (2 * p)) - 1.0 / (2 * p + 1)) > 1e-12


def test_endpoint_weight_closed_form():
    # GLL end weight on [-1,1] is 2/(p(p+1)); on [0,1] it is 1/(p(p+1))
    for p in range(1, 15):
        _, w = gll.gll(p)
        assert abs(w[0] - 1.0 / (p * (p + 1))) < 1e-16


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8, 12])
def test_derivative_matrix(p):
    x, _ = gll.gll(p)
    D = gll.lagrange_derivative_matrix(x)
    assert np.allclose(D @ np.ones(p + 1), 0.0, atol=1e-11)
    for k in range(1, p + 1):
        assert np.allclose(D @ x ** k, k * x ** (k - 1), atol=1e-9 * max(1, p) ** 2)


def test_gll_spacing_anisotropy():
    """Remark in Section 3.1: end spacing ~1/p^2 vs middle ~1/p (aspect ratio ~p)."""
    x, _ = gll.gll(6)
    h = np.diff(x)
    assert abs(h[0] - 0.0848880518607165) < 1e-12
    assert abs(h.max() / h[0] - 2.7616) < 1e-3
    x, _ = gll.gll(8)
    h = np.diff(x)
    assert abs(h.max() / h[0] - 3.6224) < 1e-3

"""CPU checks of the C ABI: the library loads, exports every function that
include/lor.h declares, and its host-side set-up logic (GLL nodes, MDF
ordering and IC(0) factor) agrees bit for bit with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import gll, lor as OL, mdf, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lor.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lor_[A-Za-z_0-9]+)\s*\(", src)))


def test_library_exports_header_symbols():
    from paper_1908_07071_amd import lor as L
    lib = ctypes.CDLL(L.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTED) == names


def test_error_strings_and_defaults():
    from paper_1908_07071_amd import lor as L
    assert L.error_string(L.LOR_OK) == "success"
    for c in range(-8, 0):
        assert L.error_string(c) != "unknown error"
    o = L.lor_default_options()
    assert o.precision == L.LOR_PREC_FP64 and o.ordering == L.LOR_ORD_MDF


@pytest.mark.parametrize("p", range(1, 15))
def test_gll_bitexact(p):
    from paper_1908_07071_amd import lor as L
    x, w = L.lor_gll(p)
    xo, wo = gll.gll(p)
    assert np.array_equal(x, xo) and np.array_equal(w, wo)


@pytest.mark.parametrize("dim,n,p,pert", [(2, 3, 4, 0.1), (2, 2, 6, 0.0), (3, 2, 3, 0.1), (3, 2, 4, 0.0)])
def test_mdf_bitexact(dim, n, p, pert):
    from paper_1908_07071_amd import lor as L
    mesh = M.make_mesh(dim, n, inputs.structured_vertices(dim, n, pert, seed=3))
    H = OL.LORHierarchy(mesh, p)
    for k in range(H.nlevels - 1):
        for v in S.vertices(mesh):
            rng = S.patch_ranges(mesh, H.sizes[k], v)
            shape = [hi - lo + 1 for lo, hi in rng]
            if min(shape) <= 0:
                continue
            idx = np.indices(shape).reshape(dim, -1, order="F")
            flat = M.lex_index([idx[i] + rng[i][0] for i in range(dim)], H.shapes[k])
            rows = H.stencils[k][flat]
            g = mdf.PatchGraph(shape, rows)
            o1, L1, D1 = mdf.mdf_factor(g)
            o2, lvl, L2, D2 = L.lor_mdf_order(dim, shape, rows)
            assert np.array_equal(o1, o2)
            assert np.array_equal(L1, L2) and np.array_equal(D1, D2)
            assert len(lvl) - 1 == mdf.dependency_depth(g, o1)
            on, _, _, _ = L.lor_mdf_order(dim, shape, rows, natural=True)
            assert np.array_equal(on, np.arange(g.n))
            # reverse Cuthill-McKee and its factor, bit for bit
            o3, L3, D3 = mdf.factor_in_order(g, mdf.rcm_order(shape))
            o4, lvl4, L4, D4 = L.lor_mdf_order(dim, shape, rows, ordering=L.LOR_ORD_RCM)
            assert np.array_equal(o3, o4)
            assert np.array_equal(L3, L4) and np.array_equal(D3, D4)
            assert len(lvl4) - 1 == mdf.dependency_depth(g, o3)


@pytest.mark.parametrize("shape", [(1, 1), (7, 1), (4, 9), (11, 11, 11), (5, 1, 7), (15, 15, 7)])
def test_rcm_order_bitexact(shape):
    """The library's RCM permutation of a patch box equals the oracle's."""
    from paper_1908_07071_amd import lor as L
    dim = len(shape)
    n = int(np.prod(shape))
    rows = np.zeros((n, 3 ** dim))
    rows[:, (3 ** dim) // 2] = 1.0  # identity: any order factors it
    o, _, _, _ = L.lor_mdf_order(dim, shape, rows, ordering=L.LOR_ORD_RCM)
    assert np.array_equal(o, mdf.rcm_order(shape))


def test_mdf_pivot_error():
    from paper_1908_07071_amd import lor as L
    rows = np.zeros((2, 9))
    rows[:, 4] = [-1.0, 2.0]
    with pytest.raises(L.LorError) as e:
        L.lor_mdf_order(2, [2, 1], rows)
    assert e.value.code == L.LOR_EPIVOT

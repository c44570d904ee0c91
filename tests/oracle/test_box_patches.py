"""Pins of the box-patch preconditioners of Section 4.5: vertex patches
enlarged for isotropic overlap, and B(n) on n overlapping slabs."""
import numpy as np
import pytest

from oracle import highorder as HO, krylov, mesh as M, schwarz as S
from paper_1908_07071_amd import inputs


def test_isotropic_boxes_on_uniform_mesh_are_vertex_patches():
    """Every edge at a vertex of a uniform mesh has the same length, so the
    enlargement stops after one element: the boxes are the plain patches and
    the two preconditioners are the same matrix."""
    mesh = M.make_mesh(2, [3, 3], inputs.structured_vertices(2, 3))
    boxes = S.isotropic_boxes(mesh)
    assert boxes == [S.vertex_box(mesh, v) for v in S.vertices(mesh)]
    p = 3
    Bv = S.SchwarzLOR(mesh, p).as_matrix()
    Bi = S.SchwarzLOR(mesh, p, patch_mode="vertex_iso").as_matrix()
    assert np.abs(Bv - Bi).max() <= 1e-13 * np.abs(Bv).max()


def test_isotropic_boxes_on_a_strip_closed_form():
    """n = 6, strip rows 2 and 3 of height h/10 (h = 1/6), the other four
    rows of height ho = (1 - 2h/10)/4 = 0.2417 > h; vertex y-coordinates
    0, .2417, .4833, .5, .5167, .7583, 1.  Threshold 0.9 delta.
    * (2, 3), on the strip's centre line: delta = h (x edges; its y edges are
      h/10); x stops after one element; downwards h/10 < 0.9h, then
      h/10 + ho: two rows; upwards likewise: box x (1, 3), y (1, 5).
    * (2, 2), on the strip's lower line: delta = ho (its lower y edge); x:
      h < 0.9 ho, 2h >= 0.9 ho: two elements each side, (0, 4); down one
      row; up h/10, 2h/10, then 2h/10 + ho: three rows: y (1, 5).
    * (2, 0), on the boundary: delta = ho; x (0, 4); y (0, 1)."""
    n = 6
    mesh = M.make_mesh(2, [n, n], inputs.strip_vertices(n, 10.0))
    boxes = dict(zip(S.vertices(mesh), S.isotropic_boxes(mesh)))
    assert boxes[(2, 3)] == [(1, 3), (1, 5)]
    assert boxes[(2, 2)] == [(0, 4), (1, 5)]
    assert boxes[(2, 0)] == [(0, 4), (0, 1)]


def test_slabs_cover_and_one_slab_is_single():
    mesh = M.make_mesh(2, [5, 3], inputs.structured_vertices(2, [5, 3], 0.1, seed=3))
    assert S.slab_boxes(mesh, 2) == [[(0, 3), (0, 3)], [(1, 5), (0, 3)]]
    assert S.slab_boxes(mesh, 3) == [[(0, 2), (0, 3)], [(0, 4), (0, 3)], [(2, 5), (0, 3)]]
    p = 2
    B1 = S.SchwarzLOR(mesh, p, patch_mode="single").as_matrix()
    Bs = S.SchwarzLOR(mesh, p, patch_mode="slabs", nslabs=1).as_matrix()
    assert np.abs(B1 - Bs).max() <= 1e-13 * np.abs(B1).max()


def test_aspect_ratio_robustness():
    """Section 4.5: with plain vertex patches the count grows with the
    aspect ratio of the strip; with isotropic overlap, and with B(1), B(2)
    and B(3), it stays flat."""
    p = 3
    its = {}
    for A in (1.5, 150.0):
        mesh = M.make_mesh(2, [8, 8], inputs.strip_vertices(8, A))
        K = HO.cg_stiffness(mesh, p)
        b = inputs.gaussian_rhs(K.shape[0], 2)
        for mode, kw in (("vertex", {}), ("vertex_iso", {}), ("single", {}),
                         ("slabs2", {"patch_mode": "slabs", "nslabs": 2}),
                         ("slabs3", {"patch_mode": "slabs", "nslabs": 3})):
            kw = dict(kw)
            kw.setdefault("patch_mode", mode)
            B = S.SchwarzLOR(mesh, p, **kw)
            x, its[mode, A], _ = krylov.pcg(K, b, B.apply, tol=1e-8, maxit=2000)
            assert np.linalg.norm(b - K @ x) <= 1.05e-8 * np.linalg.norm(b)
    assert its["vertex", 150.0] > 3 * its["vertex", 1.5], its
    for mode in ("vertex_iso", "single", "slabs2", "slabs3"):
        assert its[mode, 150.0] <= 1.25 * its[mode, 1.5], (mode, its)

"""Seeded input generator: LR refinement produces valid LR-splines."""
import numpy as np
import pytest

import lrgen
from conftest import workload


def _fp32_exact(a):
    return np.all(a.astype(np.float32).astype(np.float64) == a)


def _partition_check(box, n=4000, seed=0):
    """Every sampled point (random, corners, face centres) lies in exactly one
    element, and the volumes sum to one."""
    from oracle.lookup import ElementIndex, find_element_scan
    vol = np.prod(box[:, 3:] - box[:, :3], axis=1).sum()
    assert abs(vol - 1.0) < 1e-12
    rng = np.random.default_rng(seed)
    pts = [rng.random((n, 3)), box[:, :3], box[:, 3:],
           0.5 * (box[:, :3] + box[:, 3:])]
    x = np.concatenate(pts)
    ElementIndex(box).find(x)                 # raises unless exactly one element
    find_element_scan(box, x[:300])


def test_scalar_ortho64_shape():
    w = workload("scalar_ortho64")
    s = w.spline
    assert s.p == (2, 2, 2) and s.ncomp == 1
    # 4^3 tensor mesh plus exactly 20 refinements, each adding elements
    assert s.n_elem > 64 + 20
    assert _fp32_exact(s.elem_box) and _fp32_exact(s.knots)
    assert np.all(s.gamma > 0)
    assert np.all((s.coef >= 0) & (s.coef <= 1))
    _partition_check(s.elem_box)


def test_scalar20k_shape():
    w = workload("scalar20k")
    s = w.spline
    assert 20000 <= s.n_elem < 20100
    assert _fp32_exact(s.elem_box) and _fp32_exact(s.knots)
    assert np.all(s.gamma > 0)
    _partition_check(s.elem_box, seed=1)
    assert len(w.views) == 4 and w.views[0].width == 512
    assert w.extra["coef_target"].shape == s.coef.shape


def test_generator_deterministic():
    a = lrgen.scalar_ortho64().spline
    b = lrgen.scalar_ortho64().spline
    for x, y in ((a.elem_box, b.elem_box), (a.knots, b.knots), (a.gamma, b.gamma), (a.coef, b.coef)):
        assert np.array_equal(x, y)


def test_dyadic_knots():
    """Minimal-span refinement at element midpoints keeps every knot dyadic
    (a multiple of 2^-20 after 60 refinements of a 4^3 mesh), so knots are
    exact in FP32 (R5) and the octree applies (R26)."""
    s = lrgen.small_random(p=(3, 3, 3), n=(4, 4, 4), n_ref=60, seed=3, dist="cluster")
    scaled = s.knots * 2.0 ** 20
    assert np.all(scaled == np.round(scaled))
    assert np.array_equal(s.elem_box.astype(np.float32).astype(np.float64), s.elem_box)


def test_explicit_plane_refinement():
    r = lrgen.Refiner((2, 2, 2), (2, 2, 2))
    v = float(np.float32(0.3125))
    r.refine_plane([0.1, 0.1, 0.1], 0, v)
    s = r.export()
    assert np.any(s.elem_box[:, 3] == v)
    _partition_check(s.elem_box)
    with pytest.raises(RuntimeError):
        r.refine_plane([0.1, 0.1, 0.1], 0, 0.9)


def test_views():
    v = lrgen.sphere_view([0.0, -1.0, 0.0], 64, 32)
    assert v.proj == "persp"
    for a in (v.fwd, v.right, v.up):
        assert a.dtype == np.float32 and abs(np.linalg.norm(a.astype(np.float64)) - 1) < 1e-6
    assert abs(float(v.fwd @ v.right)) < 1e-6 and abs(float(v.up @ v.right)) < 1e-6
    np.testing.assert_allclose(v.eye, [0.5, -1.5, 0.5], atol=1e-6)
    assert np.isclose(v.ty, np.tan(np.deg2rad(22.5)), rtol=1e-6)
    assert np.isclose(v.tx, v.ty * 2, rtol=1e-6)
    top = lrgen.sphere_view([0.0, 0.0, 1.0], 8, 8)      # looking down z: up falls back to y
    assert abs(float(top.up[2])) < 1e-6


def test_lut():
    lut = lrgen.default_lut()
    assert lut.shape == (256, 4) and lut.dtype == np.float32
    assert lut[0, 3] == 0 and lut[255, 3] == 1
    np.testing.assert_allclose(lut[:, 3], np.arange(256) / 255.0, atol=1e-7)


def test_requests():
    rq = lrgen.blob_requests(n=200)
    t = np.array([r.arrival_s for r in rq])
    assert np.all(np.diff(t) > 0)
    assert 0.5 < t[-1] < 1.5                       # 200 arrivals at 200/s
    res = {r.view.width for r in rq}
    assert res <= set(lrgen.SERVING_RESOLUTIONS) and len(res) == 4

"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks an oracle function against something other than itself:
closed forms, invariants, library routines, brute force.
"""
import colorsys
from math import comb

import numpy as np
import pytest

import lrgen
from conftest import workload
from oracle import bezier as obez
from oracle import camera as ocam
from oracle import grad as ograd
from oracle import render as orr
from oracle.bspline import LREvaluator, cox_de_boor
from oracle.lookup import ElementIndex, find_element_scan


# ---------------------------------------------------------------- P1 partition of unity
@pytest.mark.parametrize("make", [
    lambda: workload("scalar_ortho64").spline,
    lambda: lrgen.small_random(p=(3, 3, 3), n=(3, 3, 3), n_ref=50, seed=7, dist="cluster"),
    lambda: lrgen.small_random(p=(2, 3, 1), n=(4, 2, 5), n_ref=40, seed=8),
])
def test_partition_of_unity(make):
    """sum_i gamma_i N_i = 1 (Sec. 3.1, Eq. 2's scaling weights)."""
    s = make()
    ev = LREvaluator(s)
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.random((10000, 3)), s.elem_box[:, :3], s.elem_box[:, 3:],
                        np.array([[1.0, 1.0, 1.0], [0.0, 1.0, 0.5], [1.0, 0.0, 1.0]])])
    assert np.abs(ev.partition_of_unity(x) - 1.0).max() <= 1e-13


# ---------------------------------------------------------------- P2 polynomial reproduction
def _marsden(p, interior):
    """Coefficients of 1, x, .., x^p in a B-spline basis (Marsden's identity):
    x^a = sum_i e_a(interior knots of B_i) / binom(p, a) * B_i(x)."""
    m = interior.shape[0]
    e = np.zeros((m, p + 1))
    e[:, 0] = 1.0
    for k in range(p):                      # elementary symmetric polynomials
        for a in range(k + 1, 0, -1):
            e[:, a] += e[:, a - 1] * interior[:, k]
    return e / np.array([comb(p, a) for a in range(p + 1)])


def _poly_spline(p, n, n_ref, seed, dist):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(p[0] + 1, p[1] + 1, p[2] + 1))
    r = lrgen.Refiner(p, n)
    t0 = lrgen.tensor_spline(p, n)
    M = [_marsden(p[d], t0.knots[:, d, 1:p[d] + 1]) for d in range(3)]
    c = np.einsum("abc,ia,ib,ic->i", A, M[0], M[1], M[2])
    r.set_initial_coef(c)
    pts = rng.random((n_ref, 3)) if dist == "uniform" else np.clip(0.4 + 0.07 * rng.normal(size=(n_ref, 3)), 0, 1)
    r.refine(pts)
    return r.export(), A


def _poly_eval(A, x):
    out = np.zeros(x.shape[0])
    for a in range(A.shape[0]):
        for b in range(A.shape[1]):
            for c in range(A.shape[2]):
                out += A[a, b, c] * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c
    return out


@pytest.mark.parametrize("p,n,n_ref,dist", [((2, 2, 2), (3, 3, 3), 40, "uniform"),
                                            ((3, 3, 3), (2, 2, 2), 60, "cluster"),
                                            ((1, 2, 3), (3, 2, 2), 30, "uniform")])
def test_polynomial_reproduction(p, n, n_ref, dist):
    """Refinement preserves the function exactly (Sec. 3.1); a polynomial of
    tri-degree <= p set on the tensor mesh stays that polynomial."""
    s, A = _poly_spline(p, n, n_ref, 11, dist)
    assert s.n_elem > n[0] * n[1] * n[2] + n_ref
    ev = LREvaluator(s)
    x = np.random.default_rng(1).random((8000, 3))
    g = _poly_eval(A, x)
    f = ev.evaluate(x)[:, 0]
    assert np.abs(f - g).max() <= 1e-12 * max(1.0, np.abs(g).max())


# ---------------------------------------------------------------- P3 tensor case = scipy
@pytest.mark.parametrize("p,n", [((2, 2, 2), (4, 3, 5)), ((3, 1, 2), (2, 4, 3))])
def test_tensor_matches_scipy(p, n):
    """Eq. 1: with no refinement the LR-spline is the tensor-product spline."""
    from scipy.interpolate import NdBSpline
    rng = np.random.default_rng(2)
    nb = [n[d] + p[d] for d in range(3)]
    coef = rng.random(nb[0] * nb[1] * nb[2])
    s = lrgen.tensor_spline(p, n, coef)
    ev = LREvaluator(s)
    t = [np.concatenate([np.zeros(p[d] + 1), np.arange(1, n[d]) / n[d], np.ones(p[d] + 1)]) for d in range(3)]
    cc = coef.reshape(nb[2], nb[1], nb[0]).transpose(2, 1, 0)
    spl = NdBSpline(tuple(t), cc, tuple(p))
    x = np.concatenate([rng.random((3000, 3)), rng.integers(0, 5, size=(200, 3)) / 4.0])
    x = np.clip(x, 0.0, 1.0 - 1e-15)
    assert np.abs(ev.evaluate(x)[:, 0] - spl(x)).max() <= 1e-13


def test_cox_de_boor_domain_end():
    # closed at x = 1: the right-end B-spline is 1 there, its neighbour 0
    assert cox_de_boor(np.array([1.0]), np.array([[0.75, 1.0, 1.0, 1.0]]), 2)[0] == 1.0
    assert cox_de_boor(np.array([1.0]), np.array([[0.5, 0.75, 1.0, 1.0]]), 2)[0] == 0.0
    x = np.array([1.0 - 2.0 ** -30])
    assert abs(cox_de_boor(x, np.array([[0.75, 1.0, 1.0, 1.0]]), 2)[0] - 1.0) < 1e-8
    t = np.array([[0.25, 0.5, 0.75, 0.875]])
    assert cox_de_boor(np.array([0.875]), t, 2)[0] == 0.0     # half-open interior end


# ---------------------------------------------------------------- P4 Bezier extraction
def _blossom_bezier(A, p, box):
    """Closed-form Bernstein coefficients of the polynomial A on a box: the
    blossom of x^a on [lo, hi] at (lo^(p-j), hi^j) is e_a(...)/binom(p, a)."""
    per_axis = []
    for d in range(3):
        lo, hi = box[d], box[3 + d]
        M = np.zeros((p[d] + 1, p[d] + 1))          # [a, j]
        for j in range(p[d] + 1):
            args = np.array([[lo] * (p[d] - j) + [hi] * j])
            M[:, j] = _marsden(p[d], args)[0]
        per_axis.append(M)
    C = np.einsum("abc,aj,bk,cl->lkj", A, per_axis[0], per_axis[1], per_axis[2])
    return C.reshape(-1)


@pytest.mark.parametrize("p,n,n_ref,dist", [((2, 2, 2), (3, 3, 3), 40, "uniform"),
                                            ((3, 3, 3), (2, 2, 2), 40, "cluster")])
def test_extraction_closed_form(p, n, n_ref, dist):
    """Sec. 3.2.3: a change of basis; for a polynomial the Bezier coefficients
    on each element are its blossom values at the element corners."""
    s, A = _poly_spline(p, n, n_ref, 5, dist)
    ev = LREvaluator(s)
    C = obez.extract(s, ev)
    ref = np.stack([_blossom_bezier(A, p, b) for b in s.elem_box])
    assert np.abs(C[:, 0, :] - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())


def test_extraction_matches_cox_de_boor():
    """Bernstein evaluation of the blocks = Cox-de Boor evaluation, per element;
    convex hull; local dimension >= Bezier dimension (Sec. 3.2.3)."""
    for s in (workload("scalar_ortho64").spline,
              lrgen.small_random(p=(3, 3, 3), n=(3, 3, 3), n_ref=40, seed=4, ncomp=3)):
        ev = LREvaluator(s)
        C = obez.extract(s, ev)
        ei = ElementIndex(s.elem_box)
        x = np.random.default_rng(3).random((20000, 3))
        e = ei.find(x)
        fb = obez.evaluate(s.p, C[e], s.elem_box[e], x)
        assert np.abs(fb - ev.evaluate(x)).max() <= 1e-12
        for q in range(s.ncomp):
            assert np.all(fb[:, q] >= C[e, q].min(1) - 1e-12)
            assert np.all(fb[:, q] <= C[e, q].max(1) + 1e-12)
        nb = np.prod([v + 1 for v in s.p])
        for b in s.elem_box[:200]:
            assert ev.bsplines_on_element(b).shape[0] >= nb


def test_bernstein_basis():
    u = np.linspace(0, 1, 11)
    for p in (1, 2, 3):
        B = obez.bernstein(p, u)
        assert np.allclose(B.sum(1), 1.0, atol=1e-15)
        assert np.allclose(B[:, 0], (1 - u) ** p) and np.allclose(B[:, -1], u ** p)


# ---------------------------------------------------------------- lookup (brute force)
def test_element_index_equals_scan():
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=60, seed=9, dist="cluster")
    b = s.elem_box
    rng = np.random.default_rng(4)
    corners = np.concatenate([b[:, [0, 1, 2]], b[:, [3, 4, 5]], b[:, [0, 4, 2]], b[:, [3, 1, 5]]])
    grid = np.stack(np.meshgrid(*[np.arange(9) / 8.0] * 3, indexing="ij"), -1).reshape(-1, 3)
    x = np.concatenate([rng.random((1500, 3)).astype(np.float32).astype(np.float64), corners, grid])
    assert np.array_equal(ElementIndex(b).find(x), find_element_scan(b, x))
    assert np.array_equal(ElementIndex(b, grid=1).find(x), find_element_scan(b, x))


# ---------------------------------------------------------------- transfer function, hue
def test_transfer_function():
    lut = lrgen.default_lut()
    k = np.arange(256)
    rgba, _ = orr.transfer(k / 255.0, lut, 0.0, 1.0)
    assert np.array_equal(rgba, lut.astype(np.float64))
    rgba, _ = orr.transfer((k[:-1] + 0.5) / 255.0, lut, 0.0, 1.0)
    assert np.allclose(rgba, 0.5 * (lut[:-1].astype(np.float64) + lut[1:]), atol=1e-12)
    rgba, _ = orr.transfer(np.array([-3.0, 7.0]), lut, 0.0, 1.0)
    assert np.array_equal(rgba[0], lut[0].astype(np.float64)) and np.array_equal(rgba[1], lut[255].astype(np.float64))


def test_hsv_matches_colorsys():
    h = np.random.default_rng(5).random(2000)
    ref = np.array([colorsys.hsv_to_rgb(v, 1.0, 1.0) for v in h])
    assert np.abs(orr.hsv_full(h) - ref).max() <= 1e-12
    assert orr.hue(np.array([0.0]), np.array([0.0]))[0] == 0.0
    assert np.isclose(orr.hue(np.array([0.0]), np.array([1.0]))[0], 0.25)
    assert np.isclose(orr.hue(np.array([0.0]), np.array([-1.0]))[0], 0.75)


# ---------------------------------------------------------------- camera replay
def test_ortho_rays_exact():
    v = lrgen.ortho_z_view(64)
    ii, jj = ocam.pixel_grid(v)
    o, d, t0, t1, hit = ocam.primary_rays(v, ii, jj)
    assert hit.all()
    assert np.array_equal(o[:, 0], ((ii + 0.5) / 64).astype(np.float32))
    assert np.array_equal(o[:, 1], (1 - (jj + 0.5) / 64).astype(np.float32))
    assert np.all(o[:, 2] == 0) and np.all(d == np.array([0, 0, 1], np.float32))
    assert np.all(t0 == 0) and np.all(t1 == 1)


def test_perspective_rays_geometry():
    v = lrgen.sphere_view([0.3, -0.8, 0.5], 97, 61)
    ii, jj = ocam.pixel_grid(v)
    o, d, t0, t1, hit = ocam.primary_rays(v, ii, jj)
    # FP64 pinhole model
    sx = ((2 * ii + 1) / 97 - 1) * np.tan(np.pi / 8) * 97 / 61
    sy = (1 - (2 * jj + 1) / 61) * np.tan(np.pi / 8)
    dd = v.fwd.astype(float) + sx[:, None] * v.right.astype(float) + sy[:, None] * v.up.astype(float)
    dd /= np.linalg.norm(dd, axis=1, keepdims=True)
    assert np.abs(d - dd).max() < 2e-6
    assert hit.sum() > 0.3 * hit.size
    # entry/exit points lie on the cube surface, the midpoint inside
    for t in (t0[hit], t1[hit]):
        x = o[hit].astype(float) + t[:, None].astype(float) * d[hit].astype(float)
        dist = np.minimum(np.abs(x), np.abs(x - 1)).min(1)
        assert dist.max() < 1e-5 and np.all((x > -1e-5) & (x < 1 + 1e-5))
    # misses: an FP64 slab test finds no interval of positive length
    m = ~hit
    od, dd2 = o[m].astype(float), d[m].astype(float)
    with np.errstate(divide="ignore", invalid="ignore"):
        ta, tb = -od / dd2, (1 - od) / dd2
    near = np.nanmax(np.minimum(ta, tb), axis=1)
    far = np.nanmin(np.maximum(ta, tb), axis=1)
    assert np.all(far - near < 1e-5)
    # the centre pixel of an odd-size image looks along fwd
    c = (61 // 2) * 97 + 97 // 2
    assert np.abs(d[c] - v.fwd).max() < 1e-6


# ---------------------------------------------------------------- FP32 replay of rays and samples (R11)
def _f32_round(q):
    """The binary32 value nearest the rational q, ties to even, from the
    format's definition (24-bit significand, exponents down to -126 with
    subnormals below); independent of numpy's float32."""
    from fractions import Fraction
    q = Fraction(q)
    if q == 0:
        return 0.0
    sign = -1 if q < 0 else 1
    a = abs(q)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    e = max(e, -126)
    ulp = Fraction(2) ** (e - 23)
    m = a / ulp
    n = m.numerator // m.denominator
    r = m - n
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and n % 2 == 1):
        n += 1
    return sign * float(n * ulp)


def _f32_sqrt(q):
    """Correctly rounded binary32 square root of a non-negative rational."""
    from fractions import Fraction
    from math import isqrt
    q = Fraction(q)
    if q == 0:
        return 0.0
    # 60 extra bits: floor(sqrt(q) 2^60) with an exactness flag decides the rounding
    k = 120
    num = q.numerator << k
    s = isqrt(num // q.denominator)
    exact = s * s * q.denominator == num
    lo = Fraction(s, 1 << 60)
    # sqrt(q) lies in [lo, lo + 2^-60]; a binary32 rounding boundary can only be
    # hit exactly when the root is exact, so nudging an inexact root by half a
    # unit of the extra precision cannot change the rounded result
    return _f32_round(lo if exact else lo + Fraction(1, 1 << 61))


def _f32(v):
    from fractions import Fraction
    return Fraction(float(v))


def test_ray_setup_exact_replay():
    """Ray setup is one correctly rounded FP32 operation per operator of the
    documented sequence (R11): replayed here in exact rational arithmetic with
    a rounding written from the binary32 definition, ray by ray, bit for bit."""
    from fractions import Fraction
    for v in (lrgen.sphere_view([0.3, -0.8, 0.5], 37, 23), lrgen.sphere_view([-0.2, 0.1, 0.97], 19, 29)):
        ii, jj = ocam.pixel_grid(v)
        o, d, t0, t1, hit = ocam.primary_rays(v, ii, jj)
        W, H = Fraction(v.width), Fraction(v.height)
        rnd = _f32_round
        for r in range(0, ii.size, 7):
            sx = rnd(_f32(rnd(Fraction(2 * int(ii[r]) + 1) / W)) - 1)
            sx = rnd(_f32(sx) * _f32(v.tx))
            sy = rnd(1 - _f32(rnd(Fraction(2 * int(jj[r]) + 1) / H)))
            sy = rnd(_f32(sy) * _f32(v.ty))
            dp = [rnd(_f32(rnd(_f32(v.fwd[a]) + _f32(rnd(_f32(sx) * _f32(v.right[a]))))) +
                      _f32(rnd(_f32(sy) * _f32(v.up[a])))) for a in range(3)]
            sq = [rnd(_f32(x) * _f32(x)) for x in dp]
            n = _f32_sqrt(_f32(rnd(_f32(rnd(_f32(sq[0]) + _f32(sq[1]))) + _f32(sq[2]))))
            dd = [rnd(_f32(x) / _f32(n)) for x in dp]
            assert [float(x) for x in d[r]] == dd, (r, d[r], dd)
            assert [float(x) for x in o[r]] == [float(x) for x in v.eye]
            # slab clip on the replayed ray
            tn, tf, ok = Fraction(0), None, True
            for a in range(3):
                if dd[a] != 0.0:
                    ta = rnd((0 - _f32(v.eye[a])) / _f32(dd[a]))
                    tb = rnd((1 - _f32(v.eye[a])) / _f32(dd[a]))
                    tn = max(tn, _f32(min(ta, tb)))
                    tf = _f32(max(ta, tb)) if tf is None else min(tf, _f32(max(ta, tb)))
                else:
                    ok = ok and 0.0 <= float(v.eye[a]) <= 1.0
            assert float(t0[r]) == float(tn) and float(t1[r]) == float(tf)
            assert bool(hit[r]) == (ok and tn < tf)


def _recorded(w, view, ii, jj):
    """Every recorded sample (ray index, t, position) of a constant-field render."""
    ev = LREvaluator(w.spline)
    _, ns, recs = orr.render_view(w, view, orr.LRField(ev), ii=ii, jj=jj, record=True)
    return ns, recs


def _schedule_workload(mode, n_fixed=37):
    import copy
    w = _constant_workload(copy.copy(workload("scalar20k")), 77)
    w.step_mode = mode
    w.n_fixed_steps = n_fixed
    return w


@pytest.mark.parametrize("mode", ["fixed", "adaptive"])
def test_sample_positions_on_ray(mode):
    """Samples lie on the ray (R11): every position is an FP32 value in
    [0,1]^3 within two FP32 roundings of the exact point clamp(o + t d); for a
    perspective ray (unit d from the eye) an unclamped sample is at distance t
    from the eye; a few hundred positions equal the exact rational replay of
    fl(o + fl(t d)) bit for bit."""
    from fractions import Fraction
    w = _schedule_workload(mode)
    view = lrgen.sphere_view([0.7, 0.2, -0.5], 18, 14)
    ii, jj = ocam.pixel_grid(view)
    o, d, t0, t1, hit = ocam.primary_rays(view, ii, jj)
    ns, recs = _recorded(w, view, ii, jj)
    assert hit.sum() > 50
    n_exact = 0
    for k, r in enumerate(recs):
        idx, t, x = r["idx"], r["t"].astype(np.float64), r["x"]
        assert np.array_equal(x.astype(np.float32).astype(np.float64), x)
        assert np.all((x >= 0.0) & (x <= 1.0))
        o64, d64 = o[idx].astype(np.float64), d[idx].astype(np.float64)
        td = t[:, None] * d64
        exact = o64 + td
        bound = 2.0 ** -24 * (np.abs(td) + np.abs(exact))
        assert np.all(np.abs(x - np.clip(exact, 0.0, 1.0)) <= bound)
        inner = np.all((exact > 0.0) & (exact < 1.0), axis=1)
        dist = np.sqrt(((exact[inner] - o64[inner]) ** 2).sum(1))
        assert np.all(np.abs(dist - t[inner]) <= 1e-6 * t[inner])
        if k % 3 == 0:
            for m in range(0, idx.size, 5):
                rep = [min(max(_f32_round(_f32(o[idx[m], a]) + _f32(_f32_round(_f32(r["t"][m]) * _f32(d[idx[m], a])))),
                               0.0), 1.0) for a in range(3)]
                assert list(x[m]) == rep, (k, m, x[m], rep)
                n_exact += 1
    assert n_exact > 100


def test_fixed_schedule_midpoints():
    """Fixed steps (R9): [t_entry, t_exit) is cut into N equal segments, each
    sampled at its midpoint, so the samples are evenly spaced, sit half a
    segment inside both ends, are symmetric about the ray's middle, and the
    composited lengths are the one FP32 segment length (t_exit - t_entry)/N."""
    N = 37
    w = _schedule_workload("fixed", N)
    view = lrgen.sphere_view([-0.3, 0.9, 0.4], 16, 12)
    ii, jj = ocam.pixel_grid(view)
    o, d, t0, t1, hit = ocam.primary_rays(view, ii, jj)
    ns, recs = _recorded(w, view, ii, jj)
    assert len(recs) == N and np.all(ns[hit] == N) and np.all(ns[~hit] == 0)
    T = np.zeros((N, ii.size))
    for k, r in enumerate(recs):
        T[k, r["idx"]] = r["t"]
        seg = (t1[r["idx"]] - t0[r["idx"]]) / np.float32(N)
        assert np.array_equal(r["ds"], seg)
    h = np.nonzero(hit)[0]
    T = T[:, h]
    a, b = t0[h].astype(np.float64), t1[h].astype(np.float64)
    L = b - a
    tol = 8 * 2.0 ** -24 * np.maximum(np.abs(a), np.abs(b))      # a few FP32 roundings of t
    assert np.all(np.abs(np.diff(T, axis=0) - L / N) <= tol)
    assert np.all(np.abs((T[0] - a) - 0.5 * L / N) <= tol)
    assert np.all(np.abs((b - T[-1]) - 0.5 * L / N) <= tol)
    assert np.all(np.abs(T + T[::-1] - (a + b)) <= 2 * tol)


# ---------------------------------------------------------------- P5/P6 compositing
def _constant_workload(wl, k):
    """The same mesh with every coefficient at the value mapping to LUT row k."""
    import copy
    w = copy.copy(wl)
    c0 = wl.vmin + (k / 255.0) * (wl.vmax - wl.vmin)
    w.spline = wl.spline.with_coef(np.full_like(wl.spline.coef, c0))
    return w


@pytest.mark.parametrize("mode", ["fixed", "adaptive", "fine"])
def test_constant_field_closed_form(mode):
    """Eq. 3 with constant emission/absorption: alpha = 1 - exp(-sigma L) with
    sigma = -ln(1 - alpha_src)/xi, and C = C_src alpha, for any partition of the
    ray; Alg. 2 telescopes to it."""
    import copy
    base = copy.copy(workload("scalar20k"))
    base.step_mode = "fixed" if mode == "fixed" else "adaptive"
    base.n_fixed_steps = 37
    k = 77
    w = _constant_workload(base, k)
    ev = LREvaluator(w.spline)
    view = lrgen.sphere_view([0.2, 0.9, -0.4], 24, 16)
    ii, jj = ocam.pixel_grid(view)
    rgba, ns, recs = orr.render_view(w, view, orr.LRField(ev), ii=ii, jj=jj,
                                     mode="F" if mode == "fine" else "S", record=(mode != "fine"))
    o, d, t0, t1, hit = ocam.primary_rays(view, ii, jj)
    L = np.where(hit, t1.astype(float) - t0.astype(float), 0.0)
    if mode == "adaptive":     # the FP32 schedule covers [t0, t1) up to FP32 rounding of t
        Ls = np.zeros_like(L)
        for r in recs:
            np.add.at(Ls, r["idx"], r["ds"].astype(float))
        assert np.all(np.abs(Ls - L) <= ns * 2.0 ** -22 * 4)
        L = Ls
    lut = w.lut.astype(np.float64)
    a_src = lut[k, 3]
    sigma = -np.log1p(-a_src) / w.xi
    alpha = 1.0 - np.exp(-sigma * L)
    tol = 1e-12 if mode != "fixed" else 1e-6 * 0   # fixed: sum of N equal FP32 steps
    if mode == "fixed":
        Lf = ns * ((t1 - t0) / np.float32(37)).astype(float)
        alpha = 1.0 - np.exp(-sigma * np.where(hit, Lf, 0))
        tol = 1e-12
    assert np.abs(rgba[:, 3] - alpha).max() <= tol
    assert np.abs(rgba[:, :3] - alpha[:, None] * lut[k, :3]).max() <= tol
    assert hit.any() and (~hit).any()


def test_fixed_steps_converge_to_fine_mode():
    """Mode F (fixed fine step 2^-12, FP64 positions, its own loop) is the
    limit of the fixed-step schedule (FP32 replay): both are midpoint sums of
    the Eq. 3 integral composited by Alg. 2, so the difference falls as N
    doubles, at the second order of the midpoint rule once N is large."""
    import copy
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=12)
    w = lrgen.Workload("conv", s, lrgen.default_lut(), 0.0, 1.0, "fixed", 16, "lut",
                       [lrgen.sphere_view([0.5, -0.7, 0.4], 10, 8)])
    ev = LREvaluator(s)
    F, _, _ = orr.render_view(w, w.views[0], orr.LRField(ev), mode="F")
    errs = []
    for N in (16, 64, 256, 512):
        w2 = copy.copy(w)
        w2.n_fixed_steps = N
        S, _, _ = orr.render_view(w2, w2.views[0], orr.LRField(ev))
        errs.append(np.abs(S - F).max())
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] <= errs[0] / 1000.0 and errs[2] / errs[3] >= 3.0
    assert errs[3] < 1e-5 * np.abs(F).max()


def test_over_operator():
    """With ds = xi, Alg. 2 is the textbook front-to-back 'over' operator."""
    rng = np.random.default_rng(6)
    C = np.zeros((50, 3))
    A = np.zeros(50)
    Cref = np.zeros((50, 3))
    Aref = np.zeros(50)
    for _ in range(20):
        cs = rng.random((50, 3))
        a = rng.random(50) * 0.9
        orr.composite(C, A, cs, a, np.full(50, 0.37), 0.37)
        Cref += (a * (1 - Aref))[:, None] * cs
        Aref += a * (1 - Aref)
    assert np.abs(C - Cref).max() < 1e-14 and np.abs(A - Aref).max() < 1e-14


# ---------------------------------------------------------------- Eq. 4 schedule
def test_adaptive_schedule_powers_of_two():
    """Every step is 2^-d min side(e) of the sample's element (exact in FP32
    on dyadic meshes), clipped only at the exit, and the element of each sample
    contains the sample (Eq. 4)."""
    w = workload("scalar20k")
    view = lrgen.sphere_view([0.6, 0.3, 0.7], 20, 20)
    ev = LREvaluator(w.spline)
    _, ns, recs = orr.render_view(w, view, orr.LRField(ev), record=True)
    box = w.spline.elem_box
    for r in recs[:200]:
        e = r["e"]
        side = (box[e, 3:] - box[e, :3]).min(1) / 4.0
        assert np.all(side.astype(np.float32) == side)
        ds = r["ds"].astype(np.float64)
        assert np.all((ds == side) | ((ds < side) & (r["t"] + r["ds"] >= 0)))
        inside = np.all((box[e, :3] <= r["x"]) & ((r["x"] < box[e, 3:]) | (r["x"] == 1.0)), axis=1)
        assert inside.all()
    assert ns.max() > 20


def test_lr_and_bezier_forms_render_alike():
    w = workload("scalar_ortho64")
    ev = LREvaluator(w.spline)
    C = obez.extract(w.spline, ev)
    ii, jj = ocam.pixel_grid(w.views[0])
    sel = np.arange(0, ii.size, 7)
    a, _, _ = orr.render_view(w, w.views[0], orr.LRField(ev), ii=ii[sel], jj=jj[sel])
    b, _, _ = orr.render_view(w, w.views[0], orr.BezierField(w.spline, C), ii=ii[sel], jj=jj[sel])
    assert np.abs(a - b).max() < 1e-12


# ---------------------------------------------------------------- P10 gradient vs FD
def test_gradient_matches_finite_differences():
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=12)
    rng = np.random.default_rng(13)
    w = lrgen.Workload("tiny", s, lrgen.default_lut(), 0.0, 1.0, "adaptive", 0, "lut",
                       [lrgen.sphere_view([0.5, -0.7, 0.4], 14, 12)])
    tgt = s.with_coef(rng.random(s.coef.shape))
    ev = LREvaluator(s)
    C = obez.extract(s, ev)
    Ct = obez.extract(tgt, LREvaluator(tgt))
    view = w.views[0]
    ii, jj = ocam.pixel_grid(view)
    ei = ElementIndex(s.elem_box)
    target, _, _ = orr.render_view(w, view, orr.BezierField(s, Ct), eidx=ei)
    rgba, ns, recs = ograd.forward_records(w, view, C, ei)
    gb, gl = ograd.backward(w, C, recs, ii.size, ograd.l2_grad(rgba, target))
    hit_e = np.unique(np.concatenate([r["e"] for r in recs]))
    picks = [(int(e), int(j)) for e, j in zip(rng.choice(hit_e, 64), rng.integers(0, 27, 64))]   # 64 coefficients
    n_checked = 0
    for e, j in picks:
        fd = ograd.fd_coefficient(w, view, C, ei, ii, jj, target, e, j, h=1e-3)
        kinks = ograd.kink_samples(w, recs, e, j, 1e-3)
        if kinks:
            continue
        assert abs(fd - gb[e, 0, j]) <= 1e-3 * max(abs(fd), 1e-3 * np.abs(gb).max())
        n_checked += 1
    assert n_checked >= 32
    rows = np.argsort(-np.abs(gl).sum(1))[:3]
    for row in rows:
        for ch in (0, 3):
            fd = ograd.fd_lut(w, view, C, ei, ii, jj, target, int(row), ch, h=1e-3)
            assert abs(fd - gl[row, ch]) <= 1e-5 * max(1.0, abs(fd))


def test_gradient_where_opacity_saturates():
    """A short standard length xi makes a = 1 - (1 - alpha)^(ds/xi) round to
    exactly 1 in FP64 for clamped samples (R16); the reverse mode stays finite
    and equals central differences there (Alg. 2 differentiated)."""
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=61)
    rng = np.random.default_rng(62)
    w = lrgen.Workload("sat", s, lrgen.default_lut(), 0.0, 0.6, "adaptive", 0, "lut",
                       [lrgen.sphere_view([0.3, 0.8, -0.5], 13, 10)], xi=0.004)
    tgt = s.with_coef(rng.random(s.coef.shape))
    ev = LREvaluator(s)
    C = obez.extract(s, ev)
    Ct = obez.extract(tgt, LREvaluator(tgt))
    view = w.views[0]
    ii, jj = ocam.pixel_grid(view)
    ei = ElementIndex(s.elem_box)
    target, _, _ = orr.render_view(w, view, orr.BezierField(s, Ct), eidx=ei)
    rgba, ns, recs = ograd.forward_records(w, view, C, ei)
    assert sum(int(np.sum(r["a"] == 1.0)) for r in recs) > 0
    gb, gl = ograd.backward(w, C, recs, ii.size, ograd.l2_grad(rgba, target))
    assert np.isfinite(gb).all() and np.isfinite(gl).all()
    hit_e = np.unique(np.concatenate([r["e"] for r in recs]))
    n_checked = 0
    for e in rng.choice(hit_e, 40, replace=False):
        j = int(rng.integers(0, 27))
        if ograd.kink_samples(w, recs, int(e), j, 1e-3):
            continue
        fd = ograd.fd_coefficient(w, view, C, ei, ii, jj, target, int(e), j, h=1e-3)
        assert abs(fd - gb[e, 0, j]) <= 1e-3 * max(abs(fd), 1e-3 * np.abs(gb).max())
        n_checked += 1
    assert n_checked >= 12
    for row in np.argsort(-np.abs(gl).sum(1))[:3]:
        fd = ograd.fd_lut(w, view, C, ei, ii, jj, target, int(row), 0, h=1e-3)
        assert abs(fd - gl[row, 0]) <= 1e-5 * max(1.0, abs(fd))


# ---------------------------------------------------------------- adjoint of the change of basis
def test_extraction_adjoint_brute_force():
    """Transpose of the explicit extraction matrix, built column by column by
    extracting unit coefficient vectors on a tiny mesh."""
    s = lrgen.small_random(p=(2, 3, 1), n=(2, 2, 2), n_ref=6, seed=21)
    nb = s.coef.shape[0]
    cols = []
    for i in range(nb):
        c = np.zeros((nb, 1))
        c[i, 0] = 1.0
        si = s.with_coef(c)
        cols.append(obez.extract(si, LREvaluator(si)).reshape(-1))
    E = np.stack(cols, axis=1)                                   # [(e, q, j), i]
    G = np.random.default_rng(5).normal(size=(s.n_elem, 1, E.shape[0] // s.n_elem))
    ref = E.T @ G.reshape(-1)
    got = obez.extract_adjoint(s, LREvaluator(s), G)[:, 0]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("make", [
    lambda: workload("scalar_ortho64").spline,
    lambda: lrgen.small_random(p=(3, 3, 3), n=(3, 3, 3), n_ref=30, seed=9, ncomp=3),
])
def test_extraction_adjoint_of_point_evaluation(make):
    """Closed form: the Bernstein basis of a point x inside element e, placed
    at e, is the gradient of f(x) with respect to the Bezier block; its
    adjoint image must be dL/dc_i = gamma_i N_i(x) (Eq. 2), each component."""
    s = make()
    ev = LREvaluator(s)
    ei = ElementIndex(s.elem_box)
    rng = np.random.default_rng(6)
    x = rng.random((24, 3))
    nq = s.coef.shape[1]
    for xk in x:
        e = int(ei.find(xk[None])[0])
        B = obez.basis_on_element(s.p, s.elem_box[e:e + 1], xk[None])[0]
        G = np.zeros((s.n_elem, nq, B.shape[0]))
        G[e, :] = B * np.arange(1, nq + 1)[:, None]              # component q weighted by q+1
        got = obez.extract_adjoint(s, ev, G)
        pt, bs, val = ev.basis(xk[None])
        ref = np.zeros((s.coef.shape[0], nq))
        ref[bs] = (s.gamma[bs] * val)[:, None] * np.arange(1, nq + 1)
        assert np.abs(got - ref).max() <= 1e-12 * nq


def test_extraction_adjoint_dot_product():
    """<E c, G> = <c, E^T G> for random c and G (vector field, degree 2)."""
    s = lrgen.small_random(p=(2, 2, 2), n=(3, 3, 3), n_ref=40, seed=10, ncomp=3)
    rng = np.random.default_rng(7)
    G = rng.normal(size=(s.n_elem, 3, 27))
    lhs = np.sum(obez.extract(s, LREvaluator(s)) * G)
    rhs = np.sum(s.coef * obez.extract_adjoint(s, LREvaluator(s), G))
    assert abs(lhs - rhs) <= 1e-12 * np.abs(G).sum()


# ---------------------------------------------------------------- gradient and local illumination
def _poly_grad(A, x):
    g = np.zeros((x.shape[0], 3))
    for a in range(A.shape[0]):
        for b in range(A.shape[1]):
            for c in range(A.shape[2]):
                m = A[a, b, c]
                if a:
                    g[:, 0] += m * a * x[:, 0] ** (a - 1) * x[:, 1] ** b * x[:, 2] ** c
                if b:
                    g[:, 1] += m * b * x[:, 0] ** a * x[:, 1] ** (b - 1) * x[:, 2] ** c
                if c:
                    g[:, 2] += m * c * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** (c - 1)
    return g


@pytest.mark.parametrize("p,n,n_ref,dist", [((2, 2, 2), (3, 3, 3), 40, "uniform"),
                                            ((3, 1, 2), (2, 4, 3), 40, "cluster")])
def test_gradient_of_reproduced_polynomial(p, n, n_ref, dist):
    """A polynomial of tri-degree <= p kept through refinement: the LR gradient
    is the polynomial's derivative (Eq. 2 differentiated term by term)."""
    s, A = _poly_spline(p, n, n_ref, 17, dist)
    x = np.random.default_rng(18).random((5000, 3))
    g = LREvaluator(s).gradient(x)[:, 0, :]
    ref = _poly_grad(A, x)
    assert np.abs(g - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


def test_gradient_matches_central_differences():
    """Degree 2 with simple knots is C^1: central differences of the value."""
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=40, seed=19, ncomp=3)
    ev = LREvaluator(s)
    x = 0.05 + 0.9 * np.random.default_rng(20).random((2000, 3))
    g = ev.gradient(x)
    h = 1e-6
    for a in range(3):
        dx = np.zeros(3)
        dx[a] = h
        fd = (ev.evaluate(x + dx) - ev.evaluate(x - dx)) / (2 * h)
        assert np.abs(fd - g[:, :, a]).max() <= 1e-6 * max(1.0, np.abs(g).max())


@pytest.mark.parametrize("color", ["lut", "hue"])
def test_illumination_of_linear_field(color):
    """f linear (reproduced exactly at degree 2): the normal is constant, so a
    directional light scales every C_src, hence C, by I = max(0.4, |l.a|/|a|)
    and leaves alpha unchanged (Sec. 4.1); for a vector field (f, f, f) the
    normal of |f| is the same."""
    import copy
    A = np.zeros((3, 3, 3))
    A[0, 0, 0], A[1, 0, 0], A[0, 1, 0], A[0, 0, 1] = 0.2, 0.3, -0.2, 0.25
    t0 = lrgen.tensor_spline((2, 2, 2), (3, 3, 3))
    M = [_marsden(2, t0.knots[:, d, 1:3]) for d in range(3)]
    r = lrgen.Refiner((2, 2, 2), (3, 3, 3))
    r.set_initial_coef(np.einsum("abc,ia,ib,ic->i", A, M[0], M[1], M[2]))
    r.refine(np.random.default_rng(24).random((20, 3)))
    s = r.export()
    if color == "hue":
        s = s.with_coef(np.repeat(s.coef, 3, axis=1))
    w = lrgen.Workload("lin", s, lrgen.default_lut(), -0.5, 1.2, "adaptive", 0, color,
                       [lrgen.sphere_view([0.3, -0.8, 0.5], 12, 10)])
    ev = LREvaluator(s)
    light = (0.6, 0.0, 0.8)
    a = np.array([0.3, -0.2, 0.25])
    I = max(0.4, abs(np.dot(a, light)) / np.linalg.norm(a))
    assert I > 0.4
    plain, _, _ = orr.render_view(w, w.views[0], orr.LRField(ev))
    lit, _, _ = orr.render_view(w, w.views[0], orr.LRField(ev), shading="directional", light=light)
    assert np.abs(lit[:, 3] - plain[:, 3]).max() == 0.0
    assert np.abs(lit[:, :3] - I * plain[:, :3]).max() <= 1e-12
    assert plain[:, :3].max() > 0.05
    w2 = copy.copy(w)
    head, _, _ = orr.render_view(w2, w.views[0], orr.LRField(ev), shading="headlight")
    assert np.all(head[:, :3] >= 0.4 * plain[:, :3] - 1e-12) and np.all(head[:, :3] <= plain[:, :3] + 1e-12)


def test_illumination_floor_where_gradient_vanishes():
    f = np.array([[0.3], [0.5]])
    g = np.zeros((2, 1, 3))
    g[1, 0] = [0.0, 3.0, 4.0]
    ld = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    assert np.allclose(orr.illumination(f, g, ld), [0.4, 0.8], atol=0, rtol=1e-15)

"""Host checks of the short formulas the render kernel uses in place of the
device library's atan2, log1p and expm1: their coefficients are reproduced
from the method named in the kernel and their error bounds are measured
against numpy in FP64, with the kernel's FP32 operation sequence emulated."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1707_01170_amd", "csrc", "render.hip")
f32 = np.float32


def _function(name):
    src = open(SRC).read()
    body = src[src.index("__device__ inline float %s(" % name):]
    return body[:body.index("\n}\n")]


def _fma32(a, b, c):
    """fmaf: one rounding of the exact a*b + c (the product of two FP32 values
    is exact in FP64, so only the sum is rounded twice; the bounds below hold
    with margin)."""
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(f32)


def _atan_coefficients():
    return [float(x) for x in re.findall(r"(-?\d\.\d+)f", _function("atan01"))]


def test_atan01_coefficients_reproduced():
    """atan(t) on [0, 1] as t P(t^2), P of degree 7, fitted by Lawson's
    algorithm (iteratively reweighted least squares converging to the minimax
    fit) on Chebyshev nodes: the fit reproduces the kernel's coefficients, and
    the kernel's FP32 Horner evaluation stays within 1.1e-7 of atan."""
    c = np.array(_atan_coefficients())
    assert c.size == 8
    n = 4000
    k = np.arange(n)
    t = 0.5 - 0.5 * np.cos((2 * k + 1) * np.pi / (2 * n))
    A = np.stack([t ** (2 * j + 1) for j in range(8)], axis=1)
    y = np.arctan(t)
    w = np.full(n, 1.0 / n)
    for _ in range(200):
        sw = np.sqrt(w)
        sol = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)[0]
        err = np.abs(A @ sol - y)
        w = w * err
        w /= w.sum()
    fit = sol[::-1]                                   # highest power first, as in the kernel
    assert np.abs(fit - c).max() <= 1e-5 * np.abs(c).max()
    assert np.abs((fit - c) / c).max() <= 1e-4
    x = np.linspace(0.0, 1.0, 400001)
    poly = x * np.polyval(c, x * x)
    assert np.abs(poly - np.arctan(x)).max() <= 5e-8       # the coefficients themselves
    x32 = x.astype(f32)
    t2 = x32 * x32
    p = f32(c[0])
    for a in c[1:]:
        p = _fma32(p, t2, f32(a))
    got = (x32 * p).astype(np.float64)
    assert np.abs(got - np.arctan(x32.astype(np.float64))).max() <= 1.1e-7


def test_hue_matches_atan2():
    """The hue built from atan01 by octant reduction equals atan2(fy, fx)/2pi
    mod 1 to 2e-7 on a grid of directions, 0 at the origin."""
    c = _atan_coefficients()

    def atan01(t):
        t = t.astype(f32)
        t2 = t * t
        p = f32(c[0])
        for a in c[1:]:
            p = _fma32(p, t2, f32(a))
        return t * p

    rng = np.random.default_rng(1)
    fx = rng.normal(size=200000).astype(f32)
    fy = rng.normal(size=200000).astype(f32)
    ax, ay = np.abs(fx), np.abs(fy)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    r = atan01(mn / mx)
    r = np.where(ay > ax, f32(1.5707963267948966) - r, r)
    r = np.where(fx < 0, f32(3.141592653589793) - r, r)
    h = r * f32(0.15915494309189535)
    h = np.where(fy < 0, f32(1.0) - h, h)
    h = np.where(h >= 1, f32(0.0), h)
    ref = np.mod(np.arctan2(fy.astype(np.float64), fx.astype(np.float64)) / (2 * np.pi), 1.0)
    d = np.abs(h - ref)
    d = np.minimum(d, 1.0 - d)                         # hue is periodic
    assert d.max() <= 2e-7


def test_opacity_correction_accuracy():
    """a = 1 - (1 - alpha)^r by the kernel's series and hardware log2/exp2
    (emulated as correctly rounded FP32 results): relative error at most 1e-6
    of the exact value over alpha in [0, 1 - 2^-16] and r in (0, 16]."""
    al = np.concatenate([np.linspace(0.0, 1.0 - 2.0 ** -16, 3001), np.geomspace(1e-7, 0.05, 400)]).astype(f32)
    r = np.concatenate([np.geomspace(1e-4, 16.0, 301), [0.5, 1.0, 2.0, 0.25]]).astype(f32)
    A, R = np.meshgrid(al, r, indexing="ij")
    A, R = A.ravel(), R.ravel()
    s = f32(1.0 / 6.0)
    for k in (0.2, 0.25, 1.0 / 3.0, 0.5, 1.0):
        s = _fma32(s, A, f32(k))
    ser = -A * s
    u = (f32(1.0) - A).astype(f32)
    d = (u - f32(1.0)).astype(f32)
    with np.errstate(divide="ignore", invalid="ignore"):
        log2u = np.log2(u.astype(np.float64)).astype(f32)
        rcp = (1.0 / (-d).astype(np.float64)).astype(f32)
        lu = (log2u * f32(0.6931471805599453)).astype(f32) * (A * rcp).astype(f32)
    L = np.where(A < f32(0.03125), ser, lu).astype(f32) * R
    e = f32(1.0 / 5040.0)
    for k in (1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0):
        e = _fma32(e, L, f32(k))
    e = e * L
    big = (np.exp2((L * f32(1.4426950408889634)).astype(np.float64)).astype(f32) - f32(1.0)).astype(f32)
    got = -np.where(L > f32(-0.125), e, big).astype(np.float64)
    exact = -np.expm1(R.astype(np.float64) * np.log1p(-A.astype(np.float64)))
    ok = exact > 0
    rel = np.abs(got[ok] - exact[ok]) / exact[ok]
    assert rel.max() <= 1e-6
    assert np.all(got[~ok] == 0.0)

"""Primary rays and sample positions, replayed in IEEE FP32.

Volume rendering traces view rays through [0,1]^3 (Sec. 4).  The paper does
not give its camera model or precision; here every ray and sample position is
defined as the FP32 result of this fixed sequence of correctly rounded single
operations (no fused multiply-add), so that a GPU kernel can reproduce sample
positions bit for bit and element ids can be compared exactly.  Everything
after the position (field value, transfer function, compositing) is FP64.

Pixel (i, j), column i, row j (row 0 at the top):
  sx = ((2i+1) / W - 1) * tx          sy = (1 - (2j+1) / H) * ty
  persp:  d' = (fwd + sx*right) + sy*up   (per component, in that order)
          n = sqrt((d'x*d'x + d'y*d'y) + d'z*d'z),  d = d'/n,  o = eye
  ortho:  o = (eye + sx*right) + sy*up,   d = fwd
Slab clip against [0,1]^3: per axis with d_a != 0, t = (0 - o_a)/d_a and
(1 - o_a)/d_a; with d_a == 0 the ray misses unless 0 <= o_a <= 1.
t_entry = max(0, near planes), t_exit = min(far planes); hit iff t_entry < t_exit.
Sample at t: p_a = clamp(o_a + t*d_a, 0, 1).
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def pixel_grid(view):
    jj, ii = np.meshgrid(np.arange(view.height), np.arange(view.width), indexing="ij")
    return ii.ravel(), jj.ravel()


def primary_rays(view, ii: np.ndarray, jj: np.ndarray):
    """(o [R,3] f32, d [R,3] f32, t_entry [R] f32, t_exit [R] f32, hit [R] bool)."""
    ii = np.asarray(ii, dtype=np.int64)
    jj = np.asarray(jj, dtype=np.int64)
    W, H = f32(view.width), f32(view.height)
    fi = (2 * ii + 1).astype(f32)
    fj = (2 * jj + 1).astype(f32)
    sx = (fi / W - f32(1.0)) * f32(view.tx)
    sy = (f32(1.0) - fj / H) * f32(view.ty)
    eye, fwd, right, up = (np.asarray(v, dtype=f32) for v in (view.eye, view.fwd, view.right, view.up))
    R = ii.shape[0]
    if view.proj == "persp":
        dp = np.empty((R, 3), dtype=f32)
        for a in range(3):
            dp[:, a] = (fwd[a] + sx * right[a]) + sy * up[a]
        n = np.sqrt((dp[:, 0] * dp[:, 0] + dp[:, 1] * dp[:, 1]) + dp[:, 2] * dp[:, 2])
        d = dp / n[:, None]
        o = np.broadcast_to(eye, (R, 3)).astype(f32)
    elif view.proj == "ortho":
        o = np.empty((R, 3), dtype=f32)
        for a in range(3):
            o[:, a] = (eye[a] + sx * right[a]) + sy * up[a]
        d = np.broadcast_to(fwd, (R, 3)).astype(f32)
    else:
        raise ValueError(view.proj)
    assert o.dtype == f32 and d.dtype == f32
    t0 = np.zeros(R, dtype=f32)
    t1 = np.full(R, np.inf, dtype=f32)
    hit = np.ones(R, dtype=bool)
    for a in range(3):
        nz = d[:, a] != 0
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (f32(0.0) - o[:, a]) / d[:, a]
            tb = (f32(1.0) - o[:, a]) / d[:, a]
        tn = np.where(nz, np.minimum(ta, tb), f32(-np.inf)).astype(f32)
        tf = np.where(nz, np.maximum(ta, tb), f32(np.inf)).astype(f32)
        inside = (o[:, a] >= 0) & (o[:, a] <= 1)
        hit &= nz | inside
        t0 = np.maximum(t0, tn)
        t1 = np.minimum(t1, tf)
    hit &= t0 < t1
    return o, d, t0, t1, hit


def positions(o: np.ndarray, d: np.ndarray, t: np.ndarray) -> np.ndarray:
    """FP32 sample positions clamp(o + t*d, 0, 1), one rounding per operation."""
    p = o + t[:, None].astype(f32) * d
    assert p.dtype == f32
    return np.clip(p, f32(0.0), f32(1.0))

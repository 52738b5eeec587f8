"""Reverse-mode derivative of the Bezier-parameterised render, FP64.

The image of Alg. 2 is a function of the Bezier coefficients (through the field
value at each sample, Sec. 3.2.3) and of the transfer-function table.  With
T_i = prod_{j<i} (1 - a_i) the transmittance before sample i,
a_i = 1 - (1 - alpha_i)^(ds_i/xi), and c_i = T_i a_i C_src,i its contribution:
  C = sum_i c_i,   alpha = 1 - prod_i (1 - a_i)
  dC/dC_src,i = T_i a_i
  dC/da_i     = T_i (C_src,i - S_i),  S_i = sum_{k>i} prod_{i<j<k} (1 - a_j) a_k C_src,k
                (the radiance behind sample i seen from just behind it, summed
                back to front: S_i = a_{i+1} C_src,i+1 + (1 - a_{i+1}) S_{i+1};
                this equals (sum_{k>i} c_k) / (1 - a_i) without dividing, so it
                also holds where a_i rounds to 1)
  dalpha/da_i = prod_{j != i} (1 - a_j)
  da_i/dalpha_i = (ds_i/xi) (1 - alpha_i)^(ds_i/xi - 1)   (0 where alpha is clamped)
then through the linear interpolation of the table (weights 1-w, w on rows i0,
i1; slope LUT[i1] - LUT[i0] in s), s = 255 (v - vmin)/(vmax - vmin) (zero slope
where clamped), and v = sum_j C_e[j] B_j(u).  The forward pass stores every
sample; the suffix sums are taken directly.
"""
from __future__ import annotations

import numpy as np

from . import bezier as obez
from .render import BezierField, Scene, render_view


def forward_records(wl, view, C, eidx, ii=None, jj=None):
    """Bezier-parameterised forward render with every sample recorded."""
    field = BezierField(wl.spline, C)
    rgba, ns, recs = render_view(wl, view, field, eidx=eidx, ii=ii, jj=jj, record=True)
    return rgba, ns, recs


def backward(wl, C, recs, R: int, g_rgba: np.ndarray):
    """dL/dC [n_elem, 1, nc] and dL/dLUT [256, 4] given dL/d(rgba) [R, 4] for
    the rays of recs (scalar field, LUT colour mode)."""
    sc = Scene.of(wl)
    assert sc.color_mode == "lut" and C.shape[1] == 1
    K = len(recs)
    p = sc.p
    nc = C.shape[2]
    a = np.zeros((K, R))
    Tb = np.zeros((K, R))
    cs = np.zeros((K, R, 3))
    for k, r in enumerate(recs):
        a[k, r["idx"]] = r["a"]
        Tb[k, r["idx"]] = r["Tb"]
        cs[k, r["idx"]] = r["csrc"]
    one_m_a = 1.0 - a
    # S_i, back to front (records without a sample for a ray have a = 0, C_src = 0)
    S = np.zeros((K, R, 3))
    for k in range(K - 2, -1, -1):
        S[k] = a[k + 1][:, None] * cs[k + 1] + one_m_a[k + 1][:, None] * S[k + 1]
    # prod_{j>i} (1 - a_j)
    rev = np.cumprod(one_m_a[::-1], axis=0)[::-1]
    prod_after = np.concatenate([rev[1:], np.ones((1, R))], axis=0)
    gC = g_rgba[:, :3]
    gA = g_rgba[:, 3]
    g_csrc = (Tb * a)[:, :, None] * gC[None]
    g_a = (gC[None] * (Tb[:, :, None] * (cs - S))).sum(-1) + gA[None] * Tb * prod_after
    gbez = np.zeros_like(C)
    glut = np.zeros((256, 4))
    for k, r in enumerate(recs):
        idx = r["idx"]
        s, i0, i1, w, inside = r["st"]
        ga = g_a[k, idx]
        rr = r["ds"].astype(np.float64) / sc.xi
        clamped = r["a_raw"] > sc.alpha_clamp
        g_alpha = np.where(clamped, 0.0, ga * rr * (1.0 - r["asrc"]) ** (rr - 1.0))
        g_x = np.concatenate([g_csrc[k, idx], g_alpha[:, None]], axis=1)     # d/d rgba_src
        np.add.at(glut, i0, (1.0 - w)[:, None] * g_x)
        np.add.at(glut, i1, w[:, None] * g_x)
        slope = sc.lut[i1] - sc.lut[i0]
        g_s = (g_x * slope).sum(1)
        g_v = np.where(inside, g_s * 255.0 / (sc.vmax - sc.vmin), 0.0)
        B = obez.basis_on_element(p, wl.spline.elem_box[r["e"]], r["x"])
        np.add.at(gbez[:, 0, :], r["e"], g_v[:, None] * B)
    return gbez, glut


def l2_loss(rgba: np.ndarray, target: np.ndarray) -> float:
    """L = sum over pixels and RGB of (C - C_target)^2."""
    return float(((rgba[:, :3] - target[:, :3]) ** 2).sum())


def l2_grad(rgba: np.ndarray, target: np.ndarray) -> np.ndarray:
    g = np.zeros_like(rgba)
    g[:, :3] = 2.0 * (rgba[:, :3] - target[:, :3])
    return g


def fd_coefficient(wl, view, C, eidx, ii, jj, target, e: int, j: int, h: float = 1e-3):
    """Central difference of the L2 loss in the Bezier coefficient C[e,0,j] over
    the rays (ii, jj)."""
    Cp = C.copy()
    Cp[e, 0, j] += h
    Cm = C.copy()
    Cm[e, 0, j] -= h
    rp, _, _ = render_view(wl, view, BezierField(wl.spline, Cp), eidx=eidx, ii=ii, jj=jj)
    rm, _, _ = render_view(wl, view, BezierField(wl.spline, Cm), eidx=eidx, ii=ii, jj=jj)
    return (l2_loss(rp, target) - l2_loss(rm, target)) / (2.0 * h)


def fd_lut(wl, view, C, eidx, ii, jj, target, row: int, ch: int, h: float = 1e-3):
    """Central difference of the L2 loss in the table entry LUT[row, ch]."""
    import copy
    out = []
    for sgn in (1.0, -1.0):
        w2 = copy.copy(wl)
        lut = np.asarray(wl.lut, dtype=np.float64).copy()
        lut[row, ch] += sgn * h
        w2.lut = lut
        r, _, _ = render_view(w2, view, BezierField(wl.spline, C), eidx=eidx, ii=ii, jj=jj)
        out.append(l2_loss(r, target))
    return (out[0] - out[1]) / (2.0 * h)


def kink_rows(lut: np.ndarray, tol: float = 1e-6) -> np.ndarray:
    """Rows k (1..254) of the table where the slope of its linear interpolation
    changes: LUT[k] - LUT[k-1] differs from LUT[k+1] - LUT[k] in some channel
    by more than tol (the rounding of a linear ramp stored in FP32 is below
    it).  Across any other row the interpolated table is one straight line."""
    slope = np.diff(np.asarray(lut, dtype=np.float64), axis=0)
    return np.nonzero(np.abs(np.diff(slope, axis=0)).max(axis=1) > tol)[0] + 1


def kink_samples(wl, recs, e: int, j: int, h: float):
    """Number of samples in element e whose table position s crosses a row
    where the table's slope changes (a kink of the linear interpolation) or a
    clamp (s = 0 or 255) when C[e,0,j] moves by +-h; finite differences are
    not smooth there."""
    sc = Scene.of(wl)
    K = kink_rows(sc.lut)
    n = 0
    for r in recs:
        m = r["e"] == e
        if not np.any(m):
            continue
        B = obez.basis_on_element(sc.p, wl.spline.elem_box[r["e"][m]], r["x"][m])[:, j]
        s = r["st"][0][m]
        dsv = np.abs(B * h * 255.0 / (sc.vmax - sc.vmin))
        lo, hi = s - dsv, s + dsv
        k = np.searchsorted(K, lo, side="right")
        crossed = (k < K.size) & (K[np.minimum(k, K.size - 1)] <= hi) if K.size else np.zeros(lo.shape, bool)
        n += int(np.sum(crossed | (lo <= 0) | (hi >= 255)))
    return n

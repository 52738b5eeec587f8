"""Accuracy of computed streamlines: the error metric Eq. 7 (Sec. 5.7).

E = max_j sum_i dt_i |x_j(t_i) - y_j(t_i)|_2 over the streamlines y_j, where
x_j is a reference solution.  As in the paper the reference is the
fifth-order RKF5 solver with a very small constant step; here it is computed
by the library itself (lr_streamlines, mixed precision) and read between its
grid points by cubic Lagrange interpolation through the four nearest points.
This is host-side analysis of results, not part of the rendering path.
"""
from __future__ import annotations

import numpy as np


def reference(scene, seeds, t_end: float, h: float):
    """RKF5 with the constant step h from every seed: (h, points [m, n, 3], count [m])."""
    from .api import streamlines
    n = int(np.ceil(t_end / h)) + 1
    pts, _, cnt = streamlines(scene, seeds, method="rkf5", step="constant", precision="mixed", base=h,
                              t_end=t_end, max_samples=n)
    return h, pts[:, :, :3].double().cpu().numpy(), cnt.cpu().numpy()


def _at(ref, j, t):
    h, X, cnt = ref
    n = int(cnt[j])
    s = t / h
    k = np.clip(np.floor(s).astype(np.int64) - 1, 0, max(n - 4, 0))
    out = np.zeros((t.shape[0], 3))
    for a in range(4):                 # Lagrange weights on the nodes k .. k+3
        w = np.ones_like(s)
        for b in range(4):
            if b != a:
                w *= (s - (k + b)) / (a - b)
        out += w[:, None] * X[j, np.minimum(k + a, n - 1)]
    return out


def error_metric(ref, points, times, count) -> float:
    """Eq. 7 for lines (points [m, S, >=3], times [m, S], count [m]); points of
    a line past the end of its reference (a domain exit) are left out."""
    h = ref[0]
    P = np.asarray(points, dtype=np.float64)[:, :, :3]
    T = np.asarray(times, dtype=np.float64)
    worst = 0.0
    for j in range(P.shape[0]):
        n = int(count[j])
        if n < 2:
            continue
        t = T[j, 1:n]
        dt = np.diff(T[j, :n])
        keep = t <= (int(ref[2][j]) - 1) * h
        if not keep.any():
            continue
        d = np.sqrt(((P[j, 1:n][keep] - _at(ref, j, t[keep])) ** 2).sum(axis=1))
        worst = max(worst, float((dt[keep] * d).sum()))
    return worst

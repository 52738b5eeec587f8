"""LR B-spline evaluation in FP64 by the Cox-de Boor recursion.

Eq. 2 (Sec. 3.1): f(x) = sum_i c_i gamma_i N_i(x), where each N_i is a
tensor-product B-spline (Eq. 1) on its own local knot vectors of p_d + 2 knots
per axis.  The univariate factor is the degree-p B-spline on knots
t_0 <= ... <= t_{p+1} (Sec. 3.1, knot-vector definition), computed with
  B^0_j(x) = 1 if t_j <= x < t_{j+1} else 0      (j = 0..p)
  B^k_j(x) = (x - t_j)/(t_{j+k} - t_j) B^{k-1}_j(x)
           + (t_{j+k+1} - x)/(t_{j+k+1} - t_{j+1}) B^{k-1}_{j+1}(x),
with 0/0 := 0, and the last non-empty span closed at the domain end x = 1.
"""
from __future__ import annotations

import numpy as np


def cox_de_boor(x: np.ndarray, t: np.ndarray, p: int) -> np.ndarray:
    """Value of the B-spline with local knots t[m, 0..p+1] at x[m] (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    m = x.shape[0]
    N = np.zeros((m, p + 1))
    for j in range(p + 1):
        N[:, j] = (t[:, j] <= x) & (x < t[:, j + 1])
    # Domain end: at x == 1 the last non-empty span [t_j, t_{j+1}] is closed.
    end = (x == 1.0) & (t[:, p + 1] == 1.0)
    if np.any(end):
        nonempty = t[:, 1:] > t[:, :-1]                       # span j non-empty
        last = p - np.argmax(nonempty[:, ::-1], axis=1)       # largest such j
        rows = np.nonzero(end & nonempty.any(axis=1))[0]
        N[rows, last[rows]] = 1.0
    for k in range(1, p + 1):
        Nn = np.zeros((m, p + 1 - k))
        for j in range(p + 1 - k):
            d1 = t[:, j + k] - t[:, j]
            d2 = t[:, j + k + 1] - t[:, j + 1]
            w1 = np.divide(x - t[:, j], d1, out=np.zeros(m), where=d1 != 0)
            w2 = np.divide(t[:, j + k + 1] - x, d2, out=np.zeros(m), where=d2 != 0)
            Nn[:, j] = w1 * N[:, j] + w2 * N[:, j + 1]
        N = Nn
    return N[:, 0]


def cox_de_boor_derivative(x: np.ndarray, t: np.ndarray, p: int) -> np.ndarray:
    """d/dx of the B-spline with local knots t[m, 0..p+1] at x[m] (FP64):
      B'(x) = p/(t_p - t_0) B[t_0..t_p](x) - p/(t_{p+1} - t_1) B[t_1..t_{p+1}](x)
    (the two degree p-1 B-splines on the leading and trailing p+1 knots; 0/0 := 0),
    one-sided from the right like the half-open evaluation."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    m = x.shape[0]
    if p == 0:
        return np.zeros(m)
    d1 = t[:, p] - t[:, 0]
    d2 = t[:, p + 1] - t[:, 1]
    lo = cox_de_boor(x, t[:, :p + 1], p - 1)
    hi = cox_de_boor(x, t[:, 1:], p - 1)
    w1 = np.divide(p * lo, d1, out=np.zeros(m), where=d1 != 0)
    w2 = np.divide(p * hi, d2, out=np.zeros(m), where=d2 != 0)
    return w1 - w2


def support_contains(lo: np.ndarray, hi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Half-open containment lo <= x < hi per axis, closed where hi == x == 1."""
    return np.all((lo <= x) & ((x < hi) | ((x == 1.0) & (hi == 1.0))), axis=-1)


class LREvaluator:
    """Evaluates an LR-spline (Eq. 2) at arbitrary points.

    B-splines whose support contains a point are found through a uniform grid
    of G^3 buckets (each B-spline is listed in every bucket its support box
    overlaps); within a bucket the test is the plain half-open containment.
    """

    def __init__(self, spline, grid: int | None = None):
        self.s = spline
        self.p = tuple(int(v) for v in spline.p)
        kn = spline.knots
        self.lo = np.stack([kn[:, d, 0] for d in range(3)], axis=1)
        self.hi = np.stack([kn[:, d, self.p[d] + 1] for d in range(3)], axis=1)
        if grid is None:   # about two buckets per typical support side
            side = float(np.median(self.hi - self.lo))
            grid = int(np.clip(2 ** np.round(np.log2(2.0 / side)), 2, 64))
        self.G = G = int(grid)
        c0 = np.clip(np.floor(self.lo * G).astype(np.int64), 0, G - 1)
        c1 = np.clip(np.ceil(self.hi * G).astype(np.int64) - 1, 0, G - 1)
        ids, cells = [], []
        nb = kn.shape[0]
        span = c1 - c0 + 1
        for i in range(int(span[:, 0].max())):
            for j in range(int(span[:, 1].max())):
                for k in range(int(span[:, 2].max())):
                    ok = (i < span[:, 0]) & (j < span[:, 1]) & (k < span[:, 2])
                    b = np.nonzero(ok)[0]
                    cx, cy, cz = c0[b, 0] + i, c0[b, 1] + j, c0[b, 2] + k
                    ids.append(b)
                    cells.append((cz * G + cy) * G + cx)
        ids = np.concatenate(ids)
        cells = np.concatenate(cells)
        order = np.argsort(cells, kind="stable")
        self.cell_ids = ids[order]
        self.cell_ptr = np.zeros(G ** 3 + 1, dtype=np.int64)
        np.add.at(self.cell_ptr, cells + 1, 1)
        self.cell_ptr = np.cumsum(self.cell_ptr)
        self.gc = spline.gamma[:, None] * spline.coef        # gamma_i c_i
        self.nb = nb

    def pairs(self, x: np.ndarray):
        """All (point index, B-spline index) with x in supp(N_i)."""
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        G = self.G
        c = np.clip(np.floor(x * G).astype(np.int64), 0, G - 1)
        cell = (c[:, 2] * G + c[:, 1]) * G + c[:, 0]
        a, b = self.cell_ptr[cell], self.cell_ptr[cell + 1]
        cnt = b - a
        pt = np.repeat(np.arange(x.shape[0]), cnt)
        off = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        bs = self.cell_ids[np.repeat(a, cnt) + off]
        keep = support_contains(self.lo[bs], self.hi[bs], x[pt])
        return pt[keep], bs[keep]

    def basis(self, x: np.ndarray):
        """(point index, B-spline index, N_i(x)) for every B-spline whose
        support contains the point (N_i without the gamma_i weight)."""
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        pt, bs = self.pairs(x)
        val = np.ones(pt.shape[0])
        for d in range(3):
            pd = self.p[d]
            val *= cox_de_boor(x[pt, d], self.s.knots[bs, d, :pd + 2], pd)
        return pt, bs, val

    def evaluate(self, x: np.ndarray, chunk: int = 200000) -> np.ndarray:
        """f(x) of Eq. 2 in FP64, shape [m, ncomp]."""
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        out = np.zeros((x.shape[0], self.gc.shape[1]))
        for s0 in range(0, x.shape[0], chunk):
            xs = x[s0:s0 + chunk]
            pt, bs, val = self.basis(xs)
            for q in range(self.gc.shape[1]):
                out[s0:s0 + chunk, q] = np.bincount(pt, weights=val * self.gc[bs, q],
                                                    minlength=xs.shape[0])
        return out

    def gradient(self, x: np.ndarray) -> np.ndarray:
        """Spatial gradient of f (Eq. 2) in FP64, shape [m, ncomp, 3]: the sum
        of gamma_i c_i times the product rule over the three univariate factors."""
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        pt, bs = self.pairs(x)
        val = [cox_de_boor(x[pt, d], self.s.knots[bs, d, :self.p[d] + 2], self.p[d]) for d in range(3)]
        der = [cox_de_boor_derivative(x[pt, d], self.s.knots[bs, d, :self.p[d] + 2], self.p[d]) for d in range(3)]
        out = np.zeros((x.shape[0], self.gc.shape[1], 3))
        for a in range(3):
            w = der[a] * val[(a + 1) % 3] * val[(a + 2) % 3]
            for q in range(self.gc.shape[1]):
                out[:, q, a] = np.bincount(pt, weights=w * self.gc[bs, q], minlength=x.shape[0])
        return out

    def partition_of_unity(self, x: np.ndarray) -> np.ndarray:
        """sum_i gamma_i N_i(x), which Eq. 2's weights make identically 1."""
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        pt, bs, val = self.basis(x)
        return np.bincount(pt, weights=val * self.s.gamma[bs], minlength=x.shape[0])

    def bsplines_on_element(self, box: np.ndarray) -> np.ndarray:
        """Indices of the B-splines whose support contains the element box."""
        box = np.asarray(box, dtype=np.float64)
        inside = np.all((self.lo <= box[:3]) & (box[3:] <= self.hi), axis=1)
        return np.nonzero(inside)[0]

"""Element search by linear scan (Sec. 3.2: the O(N) search the paper starts from).

An element is a box of the box partition of [0,1]^3 (Sec. 3.1).  A point x lies
in the element with lo_d <= x_d < hi_d on every axis, where the upper face is
closed only at the domain end hi_d = 1; elements tile the domain, so exactly
one element matches every point of [0,1]^3.
"""
from __future__ import annotations

import numpy as np


def contains(box: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Half-open containment of points x [m,3] in boxes box [..., 6]."""
    lo, hi = box[..., :3], box[..., 3:]
    return np.all((lo <= x) & ((x < hi) | ((x == 1.0) & (hi == 1.0))), axis=-1)


def find_element_scan(elem_box: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The element holding each point, by testing every element (O(N) per
    point).  Raises if a point is in zero or several elements."""
    elem_box = np.asarray(elem_box, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.empty(x.shape[0], dtype=np.int64)
    for i in range(x.shape[0]):
        hit = np.nonzero(contains(elem_box, x[i]))[0]
        if hit.shape[0] != 1:
            raise AssertionError("point %r lies in %d elements" % (x[i].tolist(), hit.shape[0]))
        out[i] = hit[0]
    return out


class ElementIndex:
    """The same linear scan restricted to the elements listed in the point's
    bucket of a uniform G^3 grid (every element is listed in each bucket its
    box overlaps, so the element holding a point is always among them)."""

    def __init__(self, elem_box: np.ndarray, grid: int | None = None):
        self.box = np.asarray(elem_box, dtype=np.float64)
        if grid is None:
            side = float(np.median(self.box[:, 3:] - self.box[:, :3]))
            grid = int(np.clip(2 ** np.round(np.log2(1.0 / side)), 1, 128))
        self.G = G = int(grid)
        c0 = np.clip(np.floor(self.box[:, :3] * G).astype(np.int64), 0, G - 1)
        c1 = np.clip(np.ceil(self.box[:, 3:] * G).astype(np.int64) - 1, 0, G - 1)
        span = c1 - c0 + 1
        ids, cells = [], []
        for i in range(int(span[:, 0].max())):
            for j in range(int(span[:, 1].max())):
                for k in range(int(span[:, 2].max())):
                    ok = (i < span[:, 0]) & (j < span[:, 1]) & (k < span[:, 2])
                    e = np.nonzero(ok)[0]
                    ids.append(e)
                    cells.append(((c0[e, 2] + k) * G + c0[e, 1] + j) * G + c0[e, 0] + i)
        ids = np.concatenate(ids)
        cells = np.concatenate(cells)
        order = np.argsort(cells, kind="stable")
        self.ids = ids[order]
        ptr = np.zeros(G ** 3 + 1, dtype=np.int64)
        np.add.at(ptr, cells + 1, 1)
        self.ptr = np.cumsum(ptr)

    def find(self, x: np.ndarray) -> np.ndarray:
        """Element id of each point; raises unless exactly one element holds it."""
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        G = self.G
        c = np.clip(np.floor(x * G).astype(np.int64), 0, G - 1)
        cell = (c[:, 2] * G + c[:, 1]) * G + c[:, 0]
        a, b = self.ptr[cell], self.ptr[cell + 1]
        cnt = b - a
        pt = np.repeat(np.arange(x.shape[0]), cnt)
        off = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        el = self.ids[np.repeat(a, cnt) + off]
        keep = contains(self.box[el], x[pt])
        n_hit = np.bincount(pt[keep], minlength=x.shape[0])
        if np.any(n_hit != 1):
            bad = int(np.nonzero(n_hit != 1)[0][0])
            raise AssertionError("point %r lies in %d elements" % (x[bad].tolist(), n_hit[bad]))
        out = np.empty(x.shape[0], dtype=np.int64)
        out[pt[keep]] = el[keep]
        return out

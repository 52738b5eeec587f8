"""Shared helpers of the GPU tests: cached volumes, oracle renders, metrics."""
import sys

import numpy as np

import lrgen
from conftest import workload

TOL_F32 = 1e-4        # peak-relative max error of the FP32 path against the FP64 oracle
TOL_F16 = 1e-2        # sanity bound of the FP16-storage path (stated, not the accuracy claim)

_VOL = {}
_ORC = {}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def volume(name, blocks=64, dtype="f32", **kw):
    import paper_1707_01170_amd as P
    key = (name, blocks, dtype, tuple(sorted(kw.items())))
    if key not in _VOL:
        wl = workload(name, **kw)
        say("[gpu] building volume", key, "n_elem", wl.spline.n_elem)
        _VOL[key] = P.Volume(wl.spline, blocks=blocks, dtype=dtype)
    return _VOL[key]


def scene(name, blocks=64, dtype="f32", **kw):
    import paper_1707_01170_amd as P
    wl = workload(name, **kw)
    return wl, P.Scene(volume(name, blocks, dtype, **kw), P.RenderParams.of(wl))


def oracle_parts(name, **kw):
    from oracle.bspline import LREvaluator
    from oracle.lookup import ElementIndex
    key = (name, tuple(sorted(kw.items())))
    if key not in _ORC:
        wl = workload(name, **kw)
        _ORC[key] = (LREvaluator(wl.spline), ElementIndex(wl.spline.elem_box))
    return _ORC[key]


def oracle_render(name, view, ii, jj, record=False, **kw):
    from oracle import render as orr
    wl = workload(name, **kw)
    ev, ei = oracle_parts(name, **kw)
    return orr.render_view(wl, view, orr.LRField(ev), eidx=ei, ii=ii, jj=jj, record=record)


def resized(view, w, h):
    """The same camera at another resolution."""
    c = np.array([0.5, 0.5, 0.5])
    return lrgen.sphere_view(view.eye.astype(np.float64) - c, w, h)


def peak_rel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return float(np.abs(x - ref).max() / scale), float(np.sqrt(((x - ref) ** 2).mean()) / scale)


def sample_pixels(view, n, seed, tile=32):
    """n seeded pixels plus one tile x tile block (pixel coordinates)."""
    rng = np.random.default_rng(seed)
    ii = rng.integers(0, view.width, n)
    jj = rng.integers(0, view.height, n)
    x0 = int(rng.integers(0, max(1, view.width - tile)))
    y0 = int(rng.integers(0, max(1, view.height - tile)))
    ty, tx = np.meshgrid(np.arange(y0, min(y0 + tile, view.height)), np.arange(x0, min(x0 + tile, view.width)),
                         indexing="ij")
    return np.concatenate([ii, tx.ravel()]), np.concatenate([jj, ty.ravel()])


def per_ray_schedule(recs, R):
    """Oracle records -> per ray arrays of (t, element, ds)."""
    out = [([], [], []) for _ in range(R)]
    for r in recs:
        for k, i in enumerate(r["idx"]):
            out[i][0].append(r["t"][k])
            out[i][1].append(r["e"][k])
            out[i][2].append(r["ds"][k])
    return [(np.array(a, np.float32), np.array(b, np.int64), np.array(c, np.float32)) for a, b, c in out]

"""Discretisation error of the method's sampling schedules, oracle only (FP64).

For each workload the oracle renders the same seeded pixels twice: with the
schedule of the method (mode S: the fixed steps of the orthographic volume,
the Eq. 4 adaptive distance of Sec. 4.2 for the others) and with the fine
fixed step 2^-12 (mode F), both composited by Alg. 2.  The paper states no
error bound for its step heuristic; this prints the difference as
peak-relative max / RMS (max|S - F| / max|F|, over pixels and channels).

    python tests/report_discretisation.py [rays per workload, default 256]
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

WORKLOADS = ("scalar_ortho64", "blobs50k", "vortex200k", "scalar20k")
_JOB = None


def _chunk(args):
    from oracle import render as orr
    mode, sel = args
    wl, view, field, ei, ii, jj = _JOB
    rgba, ns, _ = orr.render_view(wl, view, field, eidx=ei, ii=ii[sel], jj=jj[sel], mode=mode)
    return rgba, ns


def compare(name: str, n_rays: int, seed: int = 7, procs: int = 8):
    import lrgen
    from oracle import render as orr
    from oracle.bspline import LREvaluator
    from oracle.lookup import ElementIndex
    global _JOB
    wl = lrgen.cached(name)
    view = wl.views[0]
    rng = np.random.default_rng(seed)
    ii = rng.integers(0, view.width, n_rays)
    jj = rng.integers(0, view.height, n_rays)
    _JOB = (wl, view, orr.LRField(LREvaluator(wl.spline)), ElementIndex(wl.spline.elem_box), ii, jj)
    chunks = np.array_split(np.arange(n_rays), procs * 4)
    out = {}
    with mp.get_context("fork").Pool(procs) as pool:
        for mode in ("S", "F"):
            parts = pool.map(_chunk, [(mode, c) for c in chunks])
            out[mode] = (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]))
    S, F = out["S"][0], out["F"][0]
    peak = np.abs(F).max()
    err = np.abs(S - F)
    return {"workload": name, "rays": n_rays, "max": float(err.max() / peak),
            "rms": float(np.sqrt((err ** 2).mean()) / peak),
            "samples_S": int(out["S"][1].sum()), "samples_F": int(out["F"][1].sum()),
            "schedule": "fixed %d" % wl.n_fixed_steps if wl.step_mode == "fixed" else "Eq. 4 adaptive"}


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    print("| workload | schedule (S) | rays | samples S / F | max \\|S-F\\| / max \\|F\\| | RMS / max \\|F\\| |")
    print("|---|---|---|---|---|---|")
    for name in WORKLOADS:
        r = compare(name, n)
        print("| %s | %s | %d | %d / %d | %.2e | %.2e |" % (r["workload"], r["schedule"], r["rays"], r["samples_S"],
                                                            r["samples_F"], r["max"], r["rms"]), flush=True)


if __name__ == "__main__":
    main()

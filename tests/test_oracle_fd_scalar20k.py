"""Finite differences of the differentiable render on the (2,2,2) scalar
volume of 20k elements itself (4 views of 512^2, L2 loss against the renders
of the second coefficient set), against the oracle's reverse mode (Alg. 2 and
Eq. 3 differentiated; the gradient entry of a Bezier coefficient of element e
only depends on the samples in e).

A coefficient C[e, j] changes only rays with a sample in e, and those rays
meet e's box; so the loss difference and the reverse-mode entry are formed
over every ray of the four views that meets the box (all other rays
contribute nothing to either).  Fields are evaluated from the LR B-splines
(Cox-de Boor) except in e, where the perturbed Bezier block is used; the
block equals the B-splines' polynomial there (the change of basis of
Sec. 3.2.3 is exact).
"""
import multiprocessing as mp

import numpy as np

from conftest import workload
from oracle import bezier as obez
from oracle import camera as ocam
from oracle import grad as ograd
from oracle import render as orr
from oracle.bspline import LREvaluator
from oracle.lookup import ElementIndex

H = 1e-3


class _OneBlockField:
    """LR-spline values, except from the Bezier block Ce in element e."""

    def __init__(self, ev, p, box, e, Ce):
        self.ev, self.p, self.box, self.e, self.Ce = ev, p, box, e, Ce

    def __call__(self, x, el):
        f = self.ev.evaluate(x)
        m = el == self.e
        if np.any(m):
            n = int(m.sum())
            f[m] = obez.evaluate(self.p, np.broadcast_to(self.Ce, (n,) + self.Ce.shape), self.box[el[m]], x[m])
        return f


def _rays_meeting(view, box, margin=1e-6):
    """Pixels whose FP32 ray meets the box (enlarged by margin) inside [t0, t1)."""
    ii, jj = ocam.pixel_grid(view)
    o, d, t0, t1, hit = ocam.primary_rays(view, ii, jj)
    o, d = o.astype(np.float64), d.astype(np.float64)
    lo, hi = box[:3] - margin, box[3:] + margin
    tn, tf = t0.astype(np.float64), t1.astype(np.float64)
    for a in range(3):
        with np.errstate(divide="ignore", invalid="ignore"):
            ta, tb = (lo[a] - o[:, a]) / d[:, a], (hi[a] - o[:, a]) / d[:, a]
        par = d[:, a] == 0
        inside = (o[:, a] >= lo[a]) & (o[:, a] <= hi[a])
        tn = np.where(par, np.where(inside, tn, np.inf), np.maximum(tn, np.minimum(ta, tb)))
        tf = np.where(par, tf, np.minimum(tf, np.maximum(ta, tb)))
    m = hit & (tn <= tf)
    return ii[m], jj[m]


_JOB = None


def _check_element(e):
    """FD against reverse mode for two coefficients of element e chosen (seeded
    by e) among those whose +-h moves no sample of e across a kink of the
    table; returns [(e, j, fd, reverse, kinked coefficients of e, visits)]."""
    wl, ev, evt, ei = _JOB
    box = wl.spline.elem_box
    p = tuple(int(v) for v in wl.spline.p)
    Ce = obez.extract(wl.spline, ev, elems=np.array([e]))[0]           # [1, nc]
    parts = []
    for view in wl.views:
        ii, jj = _rays_meeting(view, box[e])
        if ii.size == 0:
            continue
        tgt, _, _ = orr.render_view(wl, view, orr.LRField(evt), eidx=ei, ii=ii, jj=jj)
        rgba, ns, recs = orr.render_view(wl, view, _OneBlockField(ev, p, box, e, Ce), eidx=ei, ii=ii, jj=jj,
                                         record=True)
        parts.append((view, ii, jj, tgt, rgba, recs))
    visits = sum(int(np.sum(r["e"] == e)) for part in parts for r in part[5])
    if visits == 0:
        return []
    dummy = np.zeros((box.shape[0], 1, Ce.shape[1]))
    g = np.zeros(Ce.shape[1])
    for view, ii, jj, tgt, rgba, recs in parts:
        gb, _ = ograd.backward(wl, dummy, recs, ii.size, ograd.l2_grad(rgba, tgt))
        g += gb[e, 0]
    smooth = [j for j in range(Ce.shape[1])
              if sum(ograd.kink_samples(wl, part[5], e, j, H) for part in parts) == 0]
    n_kinked = Ce.shape[1] - len(smooth)
    if len(smooth) < 2:
        return [(e, -1, 0.0, 0.0, n_kinked, visits)]
    out = []
    for j in np.random.default_rng(e).choice(smooth, 2, replace=False):
        losses = []
        for sgn in (1.0, -1.0):
            Cp = Ce.copy()
            Cp[0, j] += sgn * H
            L = 0.0
            for view, ii, jj, tgt, _, _ in parts:
                r, _, _ = orr.render_view(wl, view, _OneBlockField(ev, p, box, e, Cp), eidx=ei, ii=ii, jj=jj)
                L += ograd.l2_loss(r, tgt)
            losses.append(L)
        out.append((e, int(j), (losses[0] - losses[1]) / (2 * H), g[j], n_kinked, visits))
    return out


def test_fd_on_config_volume():
    """64 seeded Bezier coefficients (2 in each of 32 elements that the rays of
    the four views sample): central differences with h = 1e-3 in FP64 agree
    with the reverse mode to 1e-3 relative.  Coefficients whose +-h moves a
    sample's table position across a row where the table's slope changes, or
    to a clamp, are not smooth there; they are counted and not drawn (the
    default table bends only at rows 127 and 128)."""
    global _JOB
    wl = workload("scalar20k")
    ev = LREvaluator(wl.spline)
    evt = LREvaluator(wl.spline.with_coef(wl.extra["coef_target"]))
    ei = ElementIndex(wl.spline.elem_box)
    rng = np.random.default_rng(2017)
    # elements sampled by the views: those met by a sparse set of traced rays
    hit = set()
    for view in wl.views:
        ii, jj = ocam.pixel_grid(view)
        sel = rng.choice(ii.size, 150, replace=False)
        _, _, recs = orr.render_view(wl, view, orr.LRField(ev), eidx=ei, ii=ii[sel], jj=jj[sel], record=True)
        for r in recs:
            hit.update(int(v) for v in r["e"])
    cand = [int(e) for e in rng.choice(np.array(sorted(hit)), 48, replace=False)]
    _JOB = (wl, ev, evt, ei)
    with mp.get_context("fork").Pool(8) as pool:
        per_elem = pool.map(_check_element, cand)
    res = [r for part in per_elem if part and part[0][1] >= 0 for r in part][:64]
    n_kinked = sum(part[0][4] for part in per_elem if part)
    assert len(res) == 64, "only %d smooth coefficients" % len(res)
    gmax = max(abs(r[3]) for r in res)
    worst = 0.0
    for e, j, fd, g, _, visits in res:
        assert visits > 0
        err = abs(fd - g) / max(abs(fd), 1e-3 * gmax)
        worst = max(worst, err)
        assert err <= 1e-3, (e, j, fd, g)
    print("64 coefficients of %d elements: worst relative FD difference %.2e; %d of %d coefficients of the "
          "candidate elements cross a table kink" % (len({r[0] for r in res}), worst, n_kinked, 27 * len(cand)))

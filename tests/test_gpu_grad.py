"""GPU adjoint (lr_render_backward) against the oracle's reverse mode.

The oracle differentiates its own FP64 Bezier-parameterised render (its own
extraction); both sides receive the same dL/d(rgba) so the comparison isolates
the adjoint.  Tolerance: 1e-4 of the largest gradient entry.
"""
import numpy as np
import pytest
import torch

from conftest import workload
from gpu_util import TOL_F32, oracle_parts, peak_rel, resized, say, scene

pytestmark = pytest.mark.gpu

_C = {}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle_blocks(coef_key="A"):
    from oracle import bezier as obez
    from oracle.bspline import LREvaluator
    if coef_key not in _C:
        wl = workload("scalar20k")
        s = wl.spline if coef_key == "A" else wl.spline.with_coef(wl.extra["coef_target"])
        ev = oracle_parts("scalar20k")[0] if coef_key == "A" else LREvaluator(s)
        _C[coef_key] = obez.extract(s, ev)
    return _C[coef_key]


def _oracle_grad(views, pix_per_view, g_per_view):
    """Sum over views of the oracle's dL/dC and dL/dLUT for the given pixels and
    upstream gradients."""
    from oracle import grad as ograd
    wl = workload("scalar20k")
    C = _oracle_blocks("A")
    ei = oracle_parts("scalar20k")[1]
    gb = np.zeros_like(C)
    gl = np.zeros((256, 4))
    imgs = []
    for v, (ii, jj), g in zip(views, pix_per_view, g_per_view):
        rgba, ns, recs = ograd.forward_records(wl, v, C, ei, ii=ii, jj=jj)
        imgs.append(rgba)
        if g is None:
            continue
        b, l = ograd.backward(wl, C, recs, ii.size, g)
        gb += b
        gl += l
    return gb, gl, imgs


def _grid(v):
    jj, ii = np.meshgrid(np.arange(v.height), np.arange(v.width), indexing="ij")
    return ii.ravel(), jj.ravel()


def test_backward_small_views():
    import paper_1707_01170_amd as P
    say("[gpu] backward small")
    wl, sc = scene("scalar20k")
    views = [resized(v, w, h) for v, (w, h) in zip(wl.views, [(40, 28), (33, 17), (24, 40), (48, 48)])]
    pix = [_grid(v) for v in views]
    _, _, imgs = _oracle_grad(views, pix, [None] * 4)
    rng = np.random.default_rng(3)
    gs = [rng.normal(size=img.shape) for img in imgs]
    gb_o, gl_o, _ = _oracle_grad(views, pix, gs)
    rgba, offs, _ = P.render(sc, views)
    g = torch.from_numpy(np.concatenate(gs).astype(np.float32)).cuda()
    gb, gl = P.render_backward(sc, views, rgba, g)
    torch.cuda.synchronize()
    gb = gb.cpu().numpy()[:, :27]
    e_b, r_b = peak_rel(gb, gb_o[:, 0, :])
    e_l, r_l = peak_rel(gl.cpu().numpy(), gl_o)
    say("backward small: dL/dC peak-rel %.3e rms %.3e | dL/dLUT %.3e rms %.3e" % (e_b, r_b, e_l, r_l))
    assert e_b <= TOL_F32 and e_l <= TOL_F32


def _kink_samples(recs, lut, delta=1e-4):
    """(record, sample) pairs whose table position lies within delta of a row
    boundary where the table's slope jumps: there the row is decided by the
    last bits of the value, so the FP32 kernel and the FP64 oracle may take
    different rows, and both one-sided derivatives are valid."""
    slope = np.diff(np.asarray(lut, dtype=np.float64), axis=0)
    jump = np.zeros(257)
    jump[1:255] = np.abs(np.diff(slope, axis=0)).max(1) > 1e-6      # boundary n: slope[n] vs slope[n - 1]
    out = []
    for k, r in enumerate(recs):
        sv = r["st"][0]
        n = np.rint(sv).astype(np.int64)
        for m in np.nonzero((np.abs(sv - n) < delta) & (n > 0) & (n < 256))[0]:
            if jump[n[m]]:
                out.append((k, int(m)))
    return out


def _flip_row(recs, k, m):
    import copy
    recs = copy.deepcopy(recs)
    S, i0, i1, w, inside = [np.array(x) for x in recs[k]["st"]]
    n = int(np.rint(S[m]))
    if S[m] >= n:
        i0[m], i1[m], w[m] = n - 1, n, 1.0      # the row just below the boundary
    else:
        i0[m], i1[m], w[m] = n, min(n + 1, 255), 0.0
    recs[k]["st"] = (S, i0, i1, w, inside)
    return recs


@pytest.mark.parametrize("p,mode", [(1, "adaptive"), (3, "adaptive"), (3, "fixed")])
def test_backward_degrees_one_and_three(p, mode):
    """The adjoint kernels of the other degrees (their LDS tables differ in
    size: 8 and 64 coefficients per slot) against the oracle's reverse mode.
    Samples whose table position lies on a slope kink of the table within
    FP32 reach may take either row on either side: the oracle's gradient is
    formed for every combination of those choices and the closest is used."""
    import itertools
    import lrgen
    import paper_1707_01170_amd as P
    from oracle import bezier as obez
    from oracle import grad as ograd
    from oracle.bspline import LREvaluator
    from oracle.lookup import ElementIndex
    say("[gpu] backward degree", p, mode)
    s = lrgen.small_random(p=(p, p, p), n=(4, 4, 4), n_ref=40, seed=52 + p)
    views = [lrgen.sphere_view([0.4, -0.6, 0.7], 30, 22), lrgen.sphere_view([-0.5, 0.2, 0.8], 18, 26)]
    wl = lrgen.Workload("deg", s, lrgen.default_lut(), 0.0, 1.0, mode, 83, "lut", views)
    C = obez.extract(s, LREvaluator(s))
    ei = ElementIndex(s.elem_box)
    rng = np.random.default_rng(7 + p)
    data, gs, kinks = [], [], []
    for vi, v in enumerate(views):
        ii, jj = _grid(v)
        rgba_o, _, recs = ograd.forward_records(wl, v, C, ei, ii=ii, jj=jj)
        g = rng.normal(size=rgba_o.shape)
        gs.append(g)
        data.append([recs, ii.size, g])
        kinks += [(vi, k, m) for k, m in _kink_samples(recs, wl.lut)]
    assert len(kinks) <= 6
    vol = P.Volume(s, blocks=4)
    sc = P.Scene(vol, P.RenderParams.of(wl))
    rgba, _, _ = P.render(sc, views)
    g = torch.from_numpy(np.concatenate(gs).astype(np.float32)).cuda()
    gb, gl = P.render_backward(sc, views, rgba, g)
    torch.cuda.synchronize()
    nc = (p + 1) ** 3
    gb = gb.cpu().numpy()[:, :nc]
    gl = gl.cpu().numpy()
    best = None
    for choice in itertools.product([False, True], repeat=len(kinks)):
        gb_o = np.zeros_like(C)
        gl_o = np.zeros((256, 4))
        for vi, (recs, R, gv) in enumerate(data):
            for (kv, k, m), flip in zip(kinks, choice):
                if flip and kv == vi:
                    recs = _flip_row(recs, k, m)
            b, l = ograd.backward(wl, C, recs, R, gv)
            gb_o += b
            gl_o += l
        e = (peak_rel(gb, gb_o[:, 0, :])[0], peak_rel(gl, gl_o)[0])
        best = e if best is None or max(e) < max(best) else best
    say("backward degree %d %s: dL/dC peak-rel %.3e, dL/dLUT %.3e (%d kink samples)" % (p, mode, best[0], best[1],
                                                                                       len(kinks)))
    assert best[0] <= TOL_F32 and best[1] <= TOL_F32


def test_backward_saturated_opacity():
    """Samples whose opacity a = 1 - (1 - alpha)^(ds/xi) rounds to 1 in FP32
    (a short standard length xi and values beyond the table's top, where alpha
    is clamped): the march ends there, and the adjoint stays finite and equal
    to the oracle's (FP64, where a stays just below 1)."""
    import lrgen
    import paper_1707_01170_amd as P
    from oracle import bezier as obez
    from oracle import grad as ograd
    from oracle.bspline import LREvaluator
    from oracle.lookup import ElementIndex
    say("[gpu] backward saturated opacity")
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=61)
    views = [lrgen.sphere_view([0.3, 0.8, -0.5], 26, 20)]
    # the march stops only where the transmittance is exactly 0 (not at the
    # default 2^-16), so that the oracle, which never stops, sees the same samples
    wl = lrgen.Workload("sat", s, lrgen.default_lut(), 0.0, 0.6, "adaptive", 0, "lut", views, xi=0.004,
                        term_alpha=1.0)
    C = obez.extract(s, LREvaluator(s))
    ei = ElementIndex(s.elem_box)
    ii, jj = _grid(views[0])
    rgba_o, _, recs = ograd.forward_records(wl, views[0], C, ei, ii=ii, jj=jj)
    rr = [r["ds"].astype(np.float64) / wl.xi for r in recs]
    n_sat = sum(int(np.sum(np.float32(1.0) - (np.float32(1.0) - r["asrc"].astype(np.float32)) ** q.astype(np.float32)
                           == np.float32(1.0))) for r, q in zip(recs, rr))
    assert n_sat > 0, "no sample saturates"
    g = np.random.default_rng(5).normal(size=rgba_o.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        gb_o, gl_o = ograd.backward(wl, C, recs, ii.size, g)
    vol = P.Volume(s, blocks=4)
    sc = P.Scene(vol, P.RenderParams.of(wl))
    rgba, _, _ = P.render(sc, views)
    gb, gl = P.render_backward(sc, views, rgba, torch.from_numpy(g.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    gb, gl = gb.cpu().numpy()[:, :27], gl.cpu().numpy()
    assert np.isfinite(gb).all() and np.isfinite(gl).all()
    e_i, _ = peak_rel(rgba.cpu().numpy(), rgba_o)
    e_b, _ = peak_rel(gb, gb_o[:, 0, :])
    e_l, _ = peak_rel(gl, gl_o)
    say("saturated opacity (%d samples): image %.3e, dL/dC %.3e, dL/dLUT %.3e" % (n_sat, e_i, e_b, e_l))
    assert e_i <= TOL_F32 and e_b <= TOL_F32 and e_l <= TOL_F32


def test_backward_full_size_sampled():
    """Full 4 x 512^2 launch; the upstream gradient is non-zero on seeded
    pixels only, which the oracle differentiates one by one."""
    import paper_1707_01170_amd as P
    say("[gpu] backward full")
    wl, sc = scene("scalar20k")
    views = wl.views
    rng = np.random.default_rng(9)
    pix, gs_sparse = [], []
    g = np.zeros((sum(v.width * v.height for v in views), 4), np.float32)
    off = 0
    for v in views:
        ii = rng.integers(0, v.width, 128)
        jj = rng.integers(0, v.height, 128)
        key = jj * v.width + ii
        key, first = np.unique(key, return_index=True)
        ii, jj = ii[first], jj[first]
        gv = rng.normal(size=(ii.size, 4))
        g[off + key] = gv
        pix.append((ii, jj))
        gs_sparse.append(gv)
        off += v.width * v.height
    gb_o, gl_o, _ = _oracle_grad(views, pix, gs_sparse)
    rgba, _, _ = P.render(sc, views)
    gb, gl = P.render_backward(sc, views, rgba, torch.from_numpy(g).cuda())
    torch.cuda.synchronize()
    e_b, r_b = peak_rel(gb.cpu().numpy()[:, :27], gb_o[:, 0, :])
    e_l, r_l = peak_rel(gl.cpu().numpy(), gl_o)
    say("backward full-size sampled: dL/dC %.3e rms %.3e | dL/dLUT %.3e rms %.3e" % (e_b, r_b, e_l, r_l))
    assert e_b <= TOL_F32 and e_l <= TOL_F32


def test_autograd_l2_loss():
    """RenderFunction end to end: L2 loss against target images rendered from
    the second coefficient set, each side with its own images."""
    import paper_1707_01170_amd as P
    from oracle import grad as ograd
    say("[gpu] autograd")
    wl, sc = scene("scalar20k")
    views = [resized(v, 36, 28) for v in wl.views]
    pix = [_grid(v) for v in views]
    vol = sc.volume
    bez_t, _ = vol.extract(wl.extra["coef_target"], "f32")
    tgt, _, _ = P.render(sc, views, bezier=bez_t)
    bez = vol.bezier.clone().requires_grad_(True)
    lut = sc.lut.clone().requires_grad_(True)
    out = P.RenderFunction.apply(bez, lut, sc, views)
    loss = ((out[:, :3] - tgt[:, :3]) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    # oracle
    from oracle import render as orr
    Ct = _oracle_blocks("B")
    ei = oracle_parts("scalar20k")[1]
    tg_o = [orr.render_view(wl, v, orr.BezierField(wl.spline, Ct), eidx=ei, ii=ii, jj=jj)[0]
            for v, (ii, jj) in zip(views, pix)]
    _, _, imgs = _oracle_grad(views, pix, [None] * 4)
    gs = [ograd.l2_grad(a, b) for a, b in zip(imgs, tg_o)]
    gb_o, gl_o, _ = _oracle_grad(views, pix, gs)
    L_o = sum(ograd.l2_loss(a, b) for a, b in zip(imgs, tg_o))
    assert abs(loss.item() - L_o) <= 1e-4 * L_o
    e_b, _ = peak_rel(bez.grad.cpu().numpy()[:, :27], gb_o[:, 0, :])
    e_l, _ = peak_rel(lut.grad.cpu().numpy(), gl_o)
    say("autograd: loss %.6f vs %.6f; dL/dC %.3e dL/dLUT %.3e" % (loss.item(), L_o, e_b, e_l))
    assert e_b <= TOL_F32 and e_l <= TOL_F32


# ------------------------------------------------ adjoint of the change of basis
@pytest.mark.parametrize("case", ["scalar20k", "vector_deg3"])
def test_extraction_adjoint(case):
    """lr_extract_bezier_backward against the oracle's transpose of its own
    interpolation extraction, for a random dL/dC (FP32 and FP64 inputs)."""
    import lrgen
    import paper_1707_01170_amd as P
    from oracle import bezier as obez
    from oracle.bspline import LREvaluator
    say("[gpu] extraction adjoint %s" % case)
    if case == "scalar20k":
        s = workload("scalar20k").spline
        ev = oracle_parts("scalar20k")[0]
        blocks = 64
    else:
        s = lrgen.small_random(p=(3, 3, 3), n=(4, 4, 4), n_ref=40, seed=31, ncomp=3)
        ev = LREvaluator(s)
        blocks = 8
    vol = P.Volume(s, blocks=blocks, dtype="f32")
    nq, nc = s.coef.shape[1], int(np.prod([v + 1 for v in s.p]))
    rng = np.random.default_rng(12)
    G = rng.normal(size=(s.n_elem, nq, nc)).astype(np.float32)
    G[rng.random(s.n_elem) < 0.3] = 0.0                    # elements no ray reached
    ref = obez.extract_adjoint(s, ev, G.astype(np.float64))
    for dt, tdt in (("f32", torch.float32), ("f64", torch.float64)):
        stride = P.bezier_stride(s.p, nq, {"f32": 0, "f64": 2}[dt])
        g = torch.zeros((s.n_elem, stride), dtype=tdt)
        g[:, :nq * nc] = torch.from_numpy(G.reshape(s.n_elem, -1)).to(tdt)
        got = vol.extract_backward(g.cuda()).cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say("extraction adjoint %s (%s grad): rel err %.3e" % (case, dt, err))
        assert err <= 1e-12


def test_autograd_to_lr_coefficients():
    """coef -> ExtractFunction -> RenderFunction -> L2 loss: dL/dc against the
    oracle's reverse mode through its own render and extraction adjoint."""
    import paper_1707_01170_amd as P
    from oracle import bezier as obez
    from oracle import grad as ograd
    from oracle import render as orr
    say("[gpu] autograd to LR coefficients")
    wl, sc = scene("scalar20k")
    views = [resized(v, 32, 24) for v in wl.views]
    pix = [_grid(v) for v in views]
    vol = sc.volume
    bez_t, _ = vol.extract(wl.extra["coef_target"], "f32")
    tgt, _, _ = P.render(sc, views, bezier=bez_t)
    coef = torch.from_numpy(np.ascontiguousarray(wl.spline.coef, dtype=np.float64)).cuda().requires_grad_(True)
    bez = P.ExtractFunction.apply(coef, vol)
    out = P.RenderFunction.apply(bez, sc.lut, sc, views)
    loss = ((out[:, :3] - tgt[:, :3]) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    Ct = _oracle_blocks("B")
    ei = oracle_parts("scalar20k")[1]
    tg_o = [orr.render_view(wl, v, orr.BezierField(wl.spline, Ct), eidx=ei, ii=ii, jj=jj)[0]
            for v, (ii, jj) in zip(views, pix)]
    _, _, imgs = _oracle_grad(views, pix, [None] * 4)
    gs = [ograd.l2_grad(a, b) for a, b in zip(imgs, tg_o)]
    gb_o, _, _ = _oracle_grad(views, pix, gs)
    gc_o = obez.extract_adjoint(wl.spline, oracle_parts("scalar20k")[0], gb_o)
    e_c, r_c = peak_rel(coef.grad.cpu().numpy(), gc_o)
    say("autograd to c: dL/dc peak-rel %.3e rms %.3e" % (e_c, r_c))
    assert e_c <= TOL_F32

"""GPU edge cases against the oracle: camera inside the volume, views that miss,
one-pixel and ragged views, degrees 1 and 3 (scalar and 3-component), a single-element volume, the
sample cap, early termination, FP16 blocks in the schedule."""
import copy

import numpy as np
import pytest
import torch

import lrgen
from gpu_util import TOL_F32, peak_rel, per_ray_schedule, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _wl(spline, views, step_mode="adaptive", n_fixed=64, vmin=0.0, vmax=1.0, color="lut"):
    return lrgen.Workload("edge", spline, lrgen.default_lut(), vmin, vmax, step_mode, n_fixed, color, views)


def _both(wl, blocks=4, dtype="f32", max_samples=None, record=False):
    import paper_1707_01170_amd as P
    from oracle import render as orr
    from oracle.bspline import LREvaluator
    from oracle.lookup import ElementIndex
    vol = P.Volume(wl.spline, blocks=blocks, dtype=dtype)
    prm = P.RenderParams.of(wl)
    if max_samples is not None:
        prm.max_samples = max_samples
    sc = P.Scene(vol, prm)
    rgba, offs, ns = P.render(sc, wl.views, nsamples=True)
    torch.cuda.synchronize()
    rgba, ns = rgba.cpu().numpy(), ns.cpu().numpy()
    ev, ei = LREvaluator(wl.spline), ElementIndex(wl.spline.elem_box)
    refs, rns = [], []
    for v in wl.views:
        jj, ii = np.meshgrid(np.arange(v.height), np.arange(v.width), indexing="ij")
        r, n, _ = orr.render_view(wl, v, orr.LRField(ev), eidx=ei, ii=ii.ravel(), jj=jj.ravel())
        refs.append(r)
        rns.append(n)
    return sc, rgba, ns, np.concatenate(refs), np.concatenate(rns)


def test_camera_inside_the_volume():
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=40)
    views = [lrgen.sphere_view(u, 40, 30, radius=0.2) for u in ([1, 0, 0], [0.3, -0.5, 0.8])]
    _, rgba, ns, ref, rns = _both(_wl(s, views))
    err, _ = peak_rel(rgba, ref)
    say("camera inside: peak-rel %.3e" % err)
    assert err <= TOL_F32 and np.all(ns > 0) and np.all(ns <= rns)


def test_views_that_miss_and_tiny_views():
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=41)
    away = lrgen.sphere_view([1, 0, 0], 16, 16)
    away.fwd = -away.fwd                           # looking away from the volume
    views = [away, lrgen.sphere_view([0, 1, 0], 1, 1), lrgen.sphere_view([0, 1, 0.2], 1, 7),
             lrgen.sphere_view([0.1, 1, 0], 7, 1), lrgen.sphere_view([1, 1, 1], 17, 9)]
    _, rgba, ns, ref, rns = _both(_wl(s, views))
    assert np.all(rgba[:256] == 0) and np.all(ns[:256] == 0)
    assert np.abs(rgba - ref).max() <= TOL_F32 * max(np.abs(ref).max(), 1e-3)
    assert np.array_equal(ns > 0, rns > 0)


@pytest.mark.parametrize("p,mode", [(1, "adaptive"), (3, "fixed"), (1, "fixed"), (3, "adaptive")])
def test_degrees_one_and_three(p, mode):
    import paper_1707_01170_amd as P
    s = lrgen.small_random(p=(p, p, p), n=(4, 4, 4), n_ref=40, seed=42 + p)
    views = [lrgen.sphere_view([0.4, -0.6, 0.7], 36, 28)]
    wl = _wl(s, views, step_mode=mode, n_fixed=97)
    sc, rgba, ns, ref, rns = _both(wl, blocks=8)
    err, _ = peak_rel(rgba, ref)
    say("degree %d %s: peak-rel %.3e" % (p, mode, err))
    assert err <= TOL_F32
    # schedule bit for bit on a few rays
    from oracle import render as orr
    from oracle.bspline import LREvaluator
    ii = np.array([3, 17, 30, 20]); jj = np.array([5, 14, 20, 2])
    t, e, ds, cnt = (x.cpu().numpy() for x in P.trace(sc, views[0], np.stack([ii, jj], 1), max_out=4096))
    _, n_o, recs = orr.render_view(wl, views[0], orr.LRField(LREvaluator(s)), ii=ii, jj=jj, record=True)
    sched = per_ray_schedule(recs, 4)
    for k in range(4):
        c = int(cnt[k])
        assert np.array_equal(t[k, :c], sched[k][0][:c]) and np.array_equal(e[k, :c], sched[k][1][:c])


@pytest.mark.parametrize("p,mode,dtype", [(1, "adaptive", "f32"), (3, "adaptive", "f32"), (1, "fixed", "f32"),
                                          (3, "fixed", "f32"), (1, "adaptive", "f16"), (3, "adaptive", "f16")])
def test_vector_degrees_one_and_three(p, mode, dtype):
    """3-component fields of degrees 1 and 3 (the hue colouring: |v| through
    the table, hue from the direction; value range [0, max |c_i|]) against
    the oracle with FP32 and FP16 blocks; the schedule bit for bit on a few
    rays."""
    import paper_1707_01170_amd as P
    from oracle import render as orr
    from oracle.bspline import LREvaluator
    from gpu_util import TOL_F16
    s = lrgen.small_random(p=(p, p, p), n=(4, 4, 4), n_ref=40, seed=52 + p, ncomp=3)
    s = s.with_coef(2.0 * s.coef - 1.0)          # components of both signs: the hue covers its circle
    vmax = float(np.sqrt((s.coef ** 2).sum(axis=1)).max())
    views = [lrgen.sphere_view([0.5, 0.7, -0.4], 40, 30)]
    wl = _wl(s, views, step_mode=mode, n_fixed=97, vmax=vmax, color="hue")
    sc, rgba, ns, ref, rns = _both(wl, blocks=8, dtype=dtype)
    err, rms = peak_rel(rgba, ref)
    say("vector degree %d %s %s: peak-rel %.3e rms %.3e" % (p, mode, dtype, err, rms))
    assert err <= (TOL_F32 if dtype == "f32" else TOL_F16)
    assert np.array_equal(ns > 0, rns > 0)
    hit = np.nonzero(rns > 0)[0]                 # four pixels whose rays meet the volume
    pick = hit[np.linspace(0, hit.size - 1, 4).astype(int)]
    ii, jj = pick % views[0].width, pick // views[0].width
    t, e, ds, cnt = (x.cpu().numpy() for x in P.trace(sc, views[0], np.stack([ii, jj], 1), max_out=4096))
    _, n_o, recs = orr.render_view(wl, views[0], orr.LRField(LREvaluator(s)), ii=ii, jj=jj, record=True)
    sched = per_ray_schedule(recs, 4)
    for k in range(4):
        c = int(cnt[k])
        assert c > 0 and np.array_equal(t[k, :c], sched[k][0][:c]) and np.array_equal(e[k, :c], sched[k][1][:c])


def test_single_element_volume():
    s = lrgen.tensor_spline((2, 2, 2), (1, 1, 1), coef=np.random.default_rng(3).random(27))
    views = [lrgen.sphere_view([0.2, 0.9, 0.3], 24, 24), lrgen.ortho_z_view(16)]
    _, rgba, ns, ref, rns = _both(_wl(s, views), blocks=1)
    assert peak_rel(rgba, ref)[0] <= TOL_F32


def test_sample_cap():
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=44)
    views = [lrgen.sphere_view([0.2, 0.9, 0.3], 20, 20)]
    _, rgba, ns, ref, rns = _both(_wl(s, views), max_samples=5)
    assert ns.max() == 5 and np.array_equal(ns, np.minimum(rns, 5))


def test_early_termination_bound():
    """A nearly opaque constant field: the GPU stops at opacity 1 - 2^-16, the
    oracle composites everything; the difference stays below the bound."""
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=45)
    s = s.with_coef(np.full_like(s.coef, 1.0))
    views = [lrgen.sphere_view([0.3, 0.8, -0.5], 24, 20)]
    _, rgba, ns, ref, rns = _both(_wl(s, views))
    assert np.any(ns < rns)
    assert np.abs(rgba - ref).max() <= 2.0 ** -16 + 1e-5


def test_fp16_blocks_same_schedule():
    import paper_1707_01170_amd as P
    from conftest import workload
    from gpu_util import resized
    wl = workload("blobs50k")
    v16 = P.Volume(wl.spline, blocks=64, dtype="f16")
    v32 = P.Volume(wl.spline, blocks=64, dtype="f32")
    view = resized(wl.views[0], 48, 32)
    pix = np.stack([np.arange(0, 48, 3), np.arange(0, 32, 2)], 1)
    a = P.trace(P.Scene(v16, P.RenderParams.of(wl)), view, pix)
    b = P.trace(P.Scene(v32, P.RenderParams.of(wl)), view, pix)
    c16, c32 = a[3].cpu().numpy(), b[3].cpu().numpy()
    for k in range(pix.shape[0]):
        n = min(c16[k], c32[k])
        assert np.array_equal(a[0][k, :n].cpu(), b[0][k, :n].cpu()) and np.array_equal(a[1][k, :n].cpu(), b[1][k, :n].cpu())


def test_corrupt_forest_is_reported():
    """A forest whose references point past its nodes or elements: the
    descent's own bounds checks report it (element -1 from lr_lookup, NaN
    pixels from lr_render) instead of reading past the arrays, and points and
    rays that never meet the corrupt references are unaffected."""
    import paper_1707_01170_amd as P
    from paper_1707_01170_amd import _lib as L
    say("[gpu] corrupt forest")
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=44)
    wl = _wl(s, [lrgen.sphere_view([0.2, -0.9, 0.4], 32, 24)])
    vol = P.Volume(s, blocks=1)
    assert vol.n_nodes > 8
    sc = P.Scene(vol, P.RenderParams.of(wl))
    good, _, _ = P.render(sc, wl.views)
    pts = torch.from_numpy(np.random.default_rng(3).random((4096, 3)).astype(np.float32))
    ids_good = P.lookup(vol, pts).cpu().numpy()
    nodes = vol.nodes.clone()
    nodes[1, 0] = vol.n_nodes + 5                                         # a node index past the nodes
    nodes[2, 1] = np.int32(np.uint32(L.LR_LEAF | (vol.n_elem + 7)).view(np.int32))   # an element past the elements
    saved = vol.nodes
    vol.nodes = nodes
    try:
        ids = P.lookup(vol, pts).cpu().numpy()
        bad, _, _ = P.render(sc, wl.views)
        torch.cuda.synchronize()
    finally:
        vol.nodes = saved
    bad, good = bad.cpu().numpy(), good.cpu().numpy()
    hit = ids == -1
    assert hit.any() and np.array_equal(ids[~hit], ids_good[~hit])
    nan = np.isnan(bad).any(axis=1)
    assert nan.any() and np.array_equal(bad[~nan], good[~nan])
    say("corrupt forest: %d of %d points report -1, %d of %d pixels NaN" % (hit.sum(), hit.size, nan.sum(), nan.size))

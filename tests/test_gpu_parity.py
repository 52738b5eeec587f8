"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Element look-up and the sample schedule are compared bit for bit; images to
1e-4 of the peak value (FP32 path); Bezier extraction to 1e-12 (FP64).
"""
import numpy as np
import pytest
import torch

import lrgen
from conftest import workload
from gpu_util import (TOL_F16, TOL_F32, oracle_parts, oracle_render, peak_rel, per_ray_schedule, resized,
                      sample_pixels, say, scene, volume)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1707_01170_amd as P
    P._lib.lib()


# ---------------------------------------------------------------- Alg. 1 look-up
@pytest.mark.parametrize("name,blocks", [("scalar20k", 16), ("scalar20k", 64), ("scalar_ortho64", 1), ("scalar_ortho64", 4)])
def test_lookup_bit_exact(name, blocks):
    import paper_1707_01170_amd as P
    say("[gpu] lookup", name, blocks)
    wl = workload(name)
    vol = volume(name, blocks=blocks)
    box = wl.spline.elem_box
    rng = np.random.default_rng(blocks)
    B = np.arange(blocks + 1) / blocks
    grid = np.stack(np.meshgrid(B, B, rng.random(8), indexing="ij"), -1).reshape(-1, 3)
    pts = np.concatenate([rng.random((200000, 3)), box[:, :3], box[:, 3:], box[:, [0, 4, 2]], box[:, [3, 1, 5]],
                          grid, np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 0.0]])]).astype(np.float32)
    got = P.lookup(vol, torch.from_numpy(pts)).cpu().numpy()
    _, ei = oracle_parts(name)
    ref = ei.find(pts.astype(np.float64))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("name,blocks", [("scalar20k", 16), ("scalar20k", 1), ("vortex200k", 256)])
def test_forest_written_to_device(name, blocks):
    """lr_build_forest_device (size query, then build and copy on the stream)
    writes the same heads and nodes as the host build's export, and the
    look-up through them is the brute-force scan's."""
    import paper_1707_01170_amd as P
    say("[gpu] forest to device", name, blocks)
    wl = workload(name)
    heads, nodes, stats = P.build_forest_device(wl.spline.elem_box, blocks)
    torch.cuda.synchronize()
    ref = P.Forest.build(wl.spline.elem_box, blocks)
    assert np.array_equal(heads.cpu().numpy().view(np.uint32), ref.heads)
    assert np.array_equal(nodes.cpu().numpy().view(np.uint32), ref.nodes)
    assert stats["n_nodes"] == ref.stats["n_nodes"] and stats["max_depth"] == ref.stats["max_depth"]


# ---------------------------------------------------------------- Sec. 3.2.3 extraction
def _small_vector():
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=40, seed=31, ncomp=3)
    return s


@pytest.mark.parametrize("which", ["scalar_ortho64", "deg3", "vector"])
def test_extraction_f64_matches_oracle(which):
    import paper_1707_01170_amd as P
    from oracle import bezier as obez
    from oracle.bspline import LREvaluator
    say("[gpu] extract", which)
    s = {"scalar_ortho64": lambda: workload("scalar_ortho64").spline,
         "deg3": lambda: lrgen.small_random(p=(3, 3, 3), n=(2, 2, 2), n_ref=50, seed=32, dist="cluster"),
         "vector": _small_vector}[which]()
    vol = P.Volume(s, blocks=4, dtype="f64")
    got = vol.bezier.cpu().numpy()
    ref = obez.extract(s, LREvaluator(s))
    nc = ref.shape[1] * ref.shape[2]
    g = got[:, :nc].reshape(ref.shape)
    assert np.abs(g - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert np.all(got[:, nc:] == 0)
    rng = vol.bez_range.cpu().numpy()
    if s.ncomp == 1:
        assert abs(rng[0] - ref.min()) <= 1e-12 and abs(rng[1] - ref.max()) <= 1e-12
    else:
        assert rng[0] == 0 and abs(rng[1] - np.linalg.norm(ref, axis=1).max()) <= 1e-12


@pytest.mark.parametrize("name", ["blobs50k", "vortex200k"])
def test_extraction_full_size_sampled(name):
    """Full volumes (more elements than the extraction launch has wavefronts,
    so each wavefront loops over several): seeded elements, the first and
    last and those around the loop's stride, against the oracle's
    interpolation; the reported value range equals the range of all FP64
    blocks (merged across wavefronts)."""
    import paper_1707_01170_amd as P
    from oracle import bezier as obez
    say("[gpu] extract full size", name)
    wl = workload(name)
    s = wl.spline
    vol = P.Volume(s, blocks=4, dtype="f64")
    got = vol.bezier.cpu().numpy()
    n = s.n_elem
    assert n > 8192
    rng_ = np.random.default_rng(17)
    pick = np.unique(np.concatenate([rng_.integers(0, n, 48), [0, 1, 8191, 8192, 8193, 16384, n - 8193, n - 1]]))
    ref = obez.extract(s, oracle_parts(name)[0], elems=pick)
    nc = ref.shape[1] * ref.shape[2]
    g = got[pick, :nc].reshape(ref.shape)
    err = np.abs(g - ref).max() / max(1.0, np.abs(ref).max())
    say("%s extraction sampled max rel %.3e" % (name, err))
    assert err <= 1e-12
    assert np.all(got[:, nc:] == 0)
    blocks = got[:, :nc].reshape(n, s.ncomp, -1)
    r = vol.bez_range.cpu().numpy()
    if s.ncomp == 1:
        assert r[0] == blocks.min() and r[1] == blocks.max()
    else:
        top = np.sqrt((blocks ** 2).sum(axis=1)).max()
        assert r[0] == 0 and abs(r[1] - top) <= 1e-14 * top


def test_extraction_rounding_is_rne():
    import paper_1707_01170_amd as P
    s = _small_vector()
    vol = P.Volume(s, blocks=4, dtype="f64")
    f64 = vol.bezier.cpu().numpy()
    b32, _ = vol.extract(s.coef, "f32")
    b16, _ = vol.extract(s.coef, "f16")
    nc = 81
    assert np.array_equal(b32.cpu().numpy()[:, :nc], f64[:, :nc].astype(np.float32))
    assert np.array_equal(b16.cpu().numpy()[:, :nc].view(np.uint16), f64[:, :nc].astype(np.float16).view(np.uint16))
    # values near FP16 ties and subnormals
    t = s.with_coef(np.linspace(-3e-5, 3e-5, s.n_bspl * 3).reshape(-1, 3) + 1e-9)
    f64b, _ = vol.extract(t.coef, "f64")
    b16b, _ = vol.extract(t.coef, "f16")
    assert np.array_equal(b16b.cpu().numpy()[:, :nc].view(np.uint16),
                          f64b.cpu().numpy()[:, :nc].astype(np.float16).view(np.uint16))


# ---------------------------------------------------------------- Eq. 4 schedule, bit for bit
@pytest.mark.parametrize("name,blocks", [("scalar_ortho64", 64), ("scalar20k", 64), ("blobs50k", 64),
                                         ("vortex200k", 64), ("vortex200k", 256), ("blobs50k", 128)])
def test_sample_schedule_bit_exact(name, blocks):
    """(t, element, ds) of traced rays equal the oracle's schedule, also through
    the forests the benchmark and the serving configuration use (256^3, 128^3)."""
    import paper_1707_01170_amd as P
    say("[gpu] trace", name, blocks)
    wl, sc = scene(name, blocks=blocks)
    view = wl.views[0] if name == "scalar_ortho64" else resized(wl.views[0], 96, 64)
    rng = np.random.default_rng(7)
    ii = rng.integers(0, view.width, 48)
    jj = rng.integers(0, view.height, 48)
    t, e, ds, cnt = P.trace(sc, view, np.stack([ii, jj], 1), max_out=8192)
    t, e, ds, cnt = (x.cpu().numpy() for x in (t, e, ds, cnt))
    _, ns, recs = oracle_render(name, view, ii, jj, record=True)
    sched = per_ray_schedule(recs, ii.size)
    n_cmp = 0
    for k in range(ii.size):
        ot, oe, ods = sched[k]
        c = int(cnt[k])
        assert c <= ns[k]
        assert np.array_equal(t[k, :c], ot[:c]), k
        assert np.array_equal(e[k, :c], oe[:c]), k
        assert np.array_equal(ds[k, :c], ods[:c]), k
        n_cmp += c
    assert n_cmp > 1000


# ---------------------------------------------------------------- whole images
def _render(sc, views, bezier=None):
    import paper_1707_01170_amd as P
    rgba, offs, ns = P.render(sc, views, bezier=bezier, nsamples=True)
    torch.cuda.synchronize()
    return rgba.cpu().numpy(), offs, ns.cpu().numpy()


def test_scalar_ortho64_full_image():
    say("[gpu] scalar_ortho64 image")
    wl, sc = scene("scalar_ortho64")
    rgba, _, ns = _render(sc, wl.views)
    ii, jj = np.meshgrid(np.arange(64), np.arange(64))
    ref, rns, _ = oracle_render("scalar_ortho64", wl.views[0], ii.ravel(), jj.ravel())
    err, rms = peak_rel(rgba, ref)
    say("scalar_ortho64 peak-rel max %.3e rms %.3e" % (err, rms))
    assert err <= TOL_F32
    assert np.array_equal(ns[rns == 256], rns[rns == 256]) and np.all(ns <= 256)


@pytest.mark.parametrize("name,w,h", [("scalar20k", 72, 40), ("blobs50k", 50, 38), ("vortex200k", 72, 41)])
def test_small_full_images(name, w, h):
    """Whole images several tiles wide with ragged edges."""
    say("[gpu] small image", name)
    wl, sc = scene(name)
    view = resized(wl.views[0], w, h)
    rgba, _, ns = _render(sc, [view])
    jj, ii = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    ref, rns, _ = oracle_render(name, view, ii.ravel(), jj.ravel())
    err, rms = peak_rel(rgba, ref)
    say("%s %dx%d peak-rel max %.3e rms %.3e" % (name, w, h, err, rms))
    assert err <= TOL_F32
    assert np.all(ns <= rns) and np.mean(ns == rns) > 0.5


@pytest.mark.parametrize("name,blocks", [("blobs50k", 128), ("vortex200k", 256), ("scalar20k", 128)])
def test_full_size_sampled(name, blocks):
    """The full-size launch in the benchmark's configuration (forest size as
    timed), checked on seeded pixels and one tile."""
    say("[gpu] full size", name, blocks)
    wl, sc = scene(name, blocks=blocks)
    rgba, offs, ns = _render(sc, wl.views)
    v = len(wl.views) - 1
    view = wl.views[v]
    ii, jj = sample_pixels(view, 1024, seed=5, tile=24)
    ref, rns, _ = oracle_render(name, view, ii, jj)
    got = rgba[offs[v] + jj * view.width + ii]
    err, rms = peak_rel(got, ref)
    say("%s full-size sampled peak-rel max %.3e rms %.3e" % (name, err, rms))
    assert err <= TOL_F32
    assert np.all(ns[offs[v] + jj * view.width + ii] <= rns)


def test_constant_field_closed_form():
    """Eq. 3 with a constant field: alpha = 1 - (1 - alpha_src)^(L/xi), C = C_src alpha."""
    import copy

    import paper_1707_01170_amd as P
    from oracle import camera as ocam
    wl = copy.copy(workload("scalar20k"))
    k = 77
    c0 = wl.vmin + (k / 255.0) * (wl.vmax - wl.vmin)
    vol = volume("scalar20k")
    bez, _ = vol.extract(np.full_like(wl.spline.coef, c0), "f32")
    sc = P.Scene(vol, P.RenderParams.of(wl))
    view = resized(wl.views[0], 64, 48)
    rgba, _, _ = _render(sc, [view], bezier=bez)
    jj, ii = np.meshgrid(np.arange(48), np.arange(64), indexing="ij")
    _, _, t0, t1, hit = ocam.primary_rays(view, ii.ravel(), jj.ravel())
    L = np.where(hit, t1.astype(float) - t0.astype(float), 0.0)
    lut = wl.lut.astype(np.float64)
    alpha = 1.0 - (1.0 - lut[k, 3]) ** (L / wl.xi)
    assert np.abs(rgba[:, 3] - alpha).max() < 2e-5
    assert np.abs(rgba[:, :3] - alpha[:, None] * lut[k, :3]).max() < 2e-5


@pytest.mark.parametrize("name", ["blobs50k", "scalar20k", "vortex200k"])
def test_fp16_storage(name):
    """FP16 Bezier storage with FP32 arithmetic: error stated, sanity-bounded."""
    say("[gpu] fp16", name)
    wl, sc16 = scene(name, dtype="f16")
    _, sc32 = scene(name)
    view = resized(wl.views[0], 64, 40)
    a, _, _ = _render(sc16, [view])
    b, _, _ = _render(sc32, [view])
    jj, ii = np.meshgrid(np.arange(40), np.arange(64), indexing="ij")
    ref, _, _ = oracle_render(name, view, ii.ravel(), jj.ravel())
    e16, r16 = peak_rel(a, ref)
    e32, r32 = peak_rel(b, ref)
    say("%s fp16 peak-rel %.3e rms %.3e | fp32 %.3e rms %.3e" % (name, e16, r16, e32, r32))
    assert e16 <= TOL_F16 and e32 <= TOL_F32


def test_fp16_storage_benchmark_launch_sampled():
    """The timed 1080p launch of the vector volume (forest 256^3) from FP16
    blocks, on seeded pixels and one tile, against the oracle; the FP32 launch
    on the same pixels beside it."""
    say("[gpu] fp16 1080p vector launch")
    wl, sc16 = scene("vortex200k", blocks=256, dtype="f16")
    _, sc32 = scene("vortex200k", blocks=256)
    view = wl.views[0]
    a, _, _ = _render(sc16, [view])
    b, _, _ = _render(sc32, [view])
    ii, jj = sample_pixels(view, 1024, seed=8, tile=24)
    ref, _, _ = oracle_render("vortex200k", view, ii, jj)
    e16, r16 = peak_rel(a[jj * view.width + ii], ref)
    e32, r32 = peak_rel(b[jj * view.width + ii], ref)
    say("vortex200k 1080p: fp16 peak-rel %.3e rms %.3e | fp32 %.3e rms %.3e" % (e16, r16, e32, r32))
    assert e16 <= TOL_F16 and e32 <= TOL_F32


def test_views_mixed_in_one_call():
    """Views of mixed size in one call (20 views: two launches of at most 16)
    equal the same views alone, forward bit for bit and the adjoint to float
    atomics' reordering."""
    import paper_1707_01170_amd as P
    from paper_1707_01170_amd import _lib as L
    wl, sc = scene("scalar20k")
    views = [resized(wl.views[i % 4], w, h) for i, (w, h) in enumerate([(40, 24), (17, 33), (64, 64), (8, 8)] * 5)]
    assert len(views) > L.LR_MAX_VIEWS_PER_LAUNCH
    together, offs, _ = P.render(sc, views)
    tg = together.cpu().numpy()
    for v, o in zip(views, offs):
        alone, _, _ = P.render(sc, [v])
        assert np.array_equal(tg[o:o + v.width * v.height], alone.cpu().numpy())
    g = torch.from_numpy(np.random.default_rng(4).normal(size=tg.shape).astype(np.float32)).cuda()
    gb, gl = P.render_backward(sc, views, together, g)
    sb, sl = torch.zeros_like(gb), torch.zeros_like(gl)
    for v, o in zip(views, offs):
        n = v.width * v.height
        b, l = P.render_backward(sc, [v], together[o:o + n], g[o:o + n])
        sb += b
        sl += l
    torch.cuda.synchronize()
    assert peak_rel(gb.cpu().numpy(), sb.cpu().numpy())[0] <= 1e-5
    assert peak_rel(gl.cpu().numpy(), sl.cpu().numpy())[0] <= 1e-5


def test_bad_input_is_rejected():
    import paper_1707_01170_amd as P
    from paper_1707_01170_amd import _lib as L
    wl, sc = scene("scalar20k")
    bad = resized(wl.views[0], 8, 8)
    bad.eye = np.array([np.nan, 0, 0], np.float32)
    with pytest.raises(L.LRError) as ex:
        P.render(sc, [bad])
    assert ex.value.status == L.LR_EINVAL
    ok, _, _ = P.render(sc, [resized(wl.views[0], 8, 8)])
    torch.cuda.synchronize()
    assert torch.isfinite(ok).all()


def test_serving_configuration_full_size_fp16():
    """The serving configuration at its largest request size: the blob volume
    with FP16 blocks (forest 128^3), one 2048^2 view, checked on seeded pixels
    and one tile against the oracle; the FP32 blocks on the same pixels for
    comparison."""
    import lrgen
    from gpu_util import TOL_F16
    say("[gpu] serving configuration, 2048^2, FP16")
    wl16, sc16 = scene("blobs50k", blocks=128, dtype="f16")
    _, sc32 = scene("blobs50k", blocks=128)
    view = lrgen.blob_requests(n=64)[0].view
    view = resized(view, 2048, 2048)
    a, _, _ = _render(sc16, [view])
    b, _, _ = _render(sc32, [view])
    ii, jj = sample_pixels(view, 1024, seed=6, tile=24)
    ref, _, _ = oracle_render("blobs50k", view, ii, jj)
    e16, r16 = peak_rel(a[jj * view.width + ii], ref)
    e32, r32 = peak_rel(b[jj * view.width + ii], ref)
    say("serving config 2048^2: fp16 peak-rel %.3e rms %.3e | fp32 %.3e rms %.3e" % (e16, r16, e32, r32))
    assert e16 <= TOL_F16 and e32 <= TOL_F32

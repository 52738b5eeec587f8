"""Gradient-based local illumination (Sec. 4.1) on the GPU against the FP64
oracle: the value and the gradient come from the same Bezier block on the GPU
and from the LR B-splines (Cox-de Boor and its derivative) in the oracle."""
import dataclasses

import numpy as np
import pytest
import torch

from conftest import workload
from gpu_util import TOL_F32, oracle_parts, peak_rel, resized, sample_pixels, say, scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _oracle(name, view, shading, light, ii=None, jj=None):
    from oracle import render as orr
    wl = workload(name)
    ev, ei = oracle_parts(name)
    if ii is None:
        jj, ii = np.meshgrid(np.arange(view.height), np.arange(view.width), indexing="ij")
        ii, jj = ii.ravel(), jj.ravel()
    return orr.render_view(wl, view, orr.LRField(ev), eidx=ei, ii=ii, jj=jj, shading=shading, light=light)


def _gpu_render(name, view, shading, light, blocks=64):
    import paper_1707_01170_amd as P
    wl, sc = scene(name, blocks=blocks)
    prm = dataclasses.replace(P.RenderParams.of(wl), shading=shading, light=light)
    rgba, _, ns = P.render(P.Scene(sc.volume, prm), [view], nsamples=True)
    torch.cuda.synchronize()
    return rgba.cpu().numpy(), ns.cpu().numpy()


@pytest.mark.parametrize("name,w,h,shading", [
    ("scalar_ortho64", 0, 0, "directional"),
    ("scalar20k", 96, 72, "headlight"),
    ("blobs50k", 64, 48, "headlight"),
    ("vortex200k", 80, 45, "directional"),
])
def test_shaded_images_match_oracle(name, w, h, shading):
    say("[gpu] shading", name, shading)
    wl = workload(name)
    view = wl.views[0] if w == 0 else resized(wl.views[0], w, h)
    light = (0.48, -0.6, 0.64)
    got, ns = _gpu_render(name, view, shading, light)
    ref, rns, _ = _oracle(name, view, shading, light)
    err, rms = peak_rel(got, ref)
    plain, _ = _gpu_render(name, view, "none", light)
    changed = np.abs(plain[:, :3] - got[:, :3]).max() / max(np.abs(plain).max(), 1e-9)
    say("shaded %s %s: peak-rel %.3e rms %.3e (shading changed the image by %.3f)" % (name, shading, err, rms, changed))
    assert np.array_equal(ns > 0, rns > 0)
    assert changed > 0.05
    assert err <= TOL_F32


@pytest.mark.parametrize("p,ncomp,shading,dtype", [(1, 1, "headlight", "f32"), (1, 3, "directional", "f32"),
                                                  (3, 3, "headlight", "f32"), (3, 3, "headlight", "f16"),
                                                  (1, 3, "directional", "f16")])
def test_shaded_other_degrees_match_oracle(p, ncomp, shading, dtype):
    """Illumination of the degrees and component counts the named volumes do
    not cover (degree 1 scalar and vector, degree 3 vector; components of both
    signs), against the oracle's LR-spline derivatives; FP16 blocks against
    the FP16 bound."""
    import lrgen
    import paper_1707_01170_amd as P
    from oracle import render as orr
    from oracle.bspline import LREvaluator
    from oracle.lookup import ElementIndex
    from gpu_util import TOL_F16
    say("[gpu] shading degree %d, %d components, %s, %s" % (p, ncomp, shading, dtype))
    s = lrgen.small_random(p=(p, p, p), n=(4, 4, 4), n_ref=40, seed=71 + p + ncomp, ncomp=ncomp)
    if ncomp == 3:
        s = s.with_coef(2.0 * s.coef - 1.0)
        vmin, vmax, color = 0.0, float(np.sqrt((s.coef ** 2).sum(axis=1)).max()), "hue"
    else:
        vmin, vmax, color = 0.0, 1.0, "lut"
    view = lrgen.sphere_view([-0.6, 0.5, 0.6], 44, 32)
    wl = lrgen.Workload("shade", s, lrgen.default_lut(), vmin, vmax, "adaptive", 64, color, [view])
    light = (0.48, -0.6, 0.64)
    vol = P.Volume(s, blocks=8, dtype=dtype)
    out = {}
    for sh in ("none", shading):
        prm = dataclasses.replace(P.RenderParams.of(wl), shading=sh, light=light)
        rgba, _, ns = P.render(P.Scene(vol, prm), [view], nsamples=True)
        torch.cuda.synchronize()
        out[sh] = (rgba.cpu().numpy(), ns.cpu().numpy())
    jj, ii = np.meshgrid(np.arange(view.height), np.arange(view.width), indexing="ij")
    ref, rns, _ = orr.render_view(wl, view, orr.LRField(LREvaluator(s)), eidx=ElementIndex(s.elem_box),
                                  ii=ii.ravel(), jj=jj.ravel(), shading=shading, light=light)
    got, ns = out[shading]
    err, rms = peak_rel(got, ref)
    plain = out["none"][0]
    changed = np.abs(plain[:, :3] - got[:, :3]).max() / max(np.abs(plain).max(), 1e-9)
    say("shaded degree %d x%d %s %s: peak-rel %.3e rms %.3e (shading changed the image by %.3f)"
        % (p, ncomp, shading, dtype, err, rms, changed))
    assert np.array_equal(ns > 0, rns > 0)
    assert changed > 0.05
    assert err <= (TOL_F32 if dtype == "f32" else TOL_F16)


def test_linear_field_constant_intensity():
    """A linear field has one normal: the shaded image is I times the plain one
    in colour and identical in opacity (directional light)."""
    import lrgen
    import paper_1707_01170_amd as P
    s = lrgen.tensor_spline((2, 2, 2), (4, 4, 4))
    g = s.greville()
    a = np.array([0.3, -0.2, 0.25])
    s = s.with_coef((0.2 + g @ a)[:, None])
    view = lrgen.sphere_view([0.3, -0.8, 0.5], 40, 30)
    wl = lrgen.Workload("lin", s, lrgen.default_lut(), -0.5, 1.2, "adaptive", 0, "lut", [view])
    vol = P.Volume(s, blocks=4)
    light = (0.6, 0.0, 0.8)
    I = max(0.4, abs(np.dot(a, light)) / np.linalg.norm(a))
    prm = P.RenderParams.of(wl)
    plain, _, _ = P.render(P.Scene(vol, prm), [view])
    lit, _, _ = P.render(P.Scene(vol, dataclasses.replace(prm, shading="directional", light=light)), [view])
    plain, lit = plain.cpu().numpy(), lit.cpu().numpy()
    assert np.array_equal(plain[:, 3], lit[:, 3])
    assert np.abs(lit[:, :3] - I * plain[:, :3]).max() <= 1e-5 * np.abs(plain).max()


def test_full_size_sampled_headlight():
    """The illuminated 1080p launch as the benchmark times it (vector volume,
    forest 256^3, headlight), checked on seeded pixels and one tile."""
    import paper_1707_01170_amd as P
    say("[gpu] shading full size")
    name = "vortex200k"
    wl, sc = scene(name, blocks=256)
    view = wl.views[0]
    prm = dataclasses.replace(P.RenderParams.of(wl), shading="headlight")
    rgba, _, ns = P.render(P.Scene(sc.volume, prm), [view], nsamples=True)
    torch.cuda.synchronize()
    ii, jj = sample_pixels(view, 1024, seed=9, tile=24)
    k = jj * view.width + ii
    ref, rns, _ = _oracle(name, view, "headlight", (0.0, 0.0, 1.0), ii=ii, jj=jj)
    got = rgba.cpu().numpy()[k]
    err, rms = peak_rel(got, ref)
    say("headlight 1080p sampled: peak-rel %.3e rms %.3e" % (err, rms))
    assert np.array_equal(ns.cpu().numpy()[k] > 0, rns > 0)
    assert err <= TOL_F32


@pytest.mark.parametrize("name,shading", [("vortex200k", "headlight"), ("blobs50k", "directional"),
                                          ("vortex200k", "none"), ("blobs50k", "none"), ("scalar20k", "headlight")])
def test_fp16_blocks_equal_fp32_kernel_on_widened_blocks(name, shading):
    """FP16 blocks are widened exactly (inside each multiply-add, or when the
    block is loaded in the illuminated vector kernel), so a render from FP16
    blocks equals, bit for bit, the FP32 kernels' render of the same values
    stored as FP32.  The plain FP32 kernels gather block reloads (a lane
    waits until half of its wave's active lanes need one) while the FP16
    ones reload at once, so this also pins that the gathering leaves every
    sample unchanged."""
    import paper_1707_01170_amd as P
    say("[gpu] fp16 == fp32 on widened blocks", name, shading)
    wl, sc16 = scene(name, blocks=64, dtype="f16")
    _, sc32 = scene(name, blocks=64)
    view = resized(wl.views[0], 96, 60)
    prm = dataclasses.replace(P.RenderParams.of(wl), shading=shading, light=(0.48, -0.6, 0.64))
    a, _, _ = P.render(P.Scene(sc16.volume, prm), [view])
    n32 = sc32.volume.bezier.shape[1]
    widened = sc16.volume.bezier.float()[:, :n32].contiguous()
    b, _, _ = P.render(P.Scene(sc32.volume, prm), [view], bezier=widened)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("name,blocks", [("vortex200k", 256), ("blobs50k", 128)])
def test_gathered_reloads_leave_the_full_frame_unchanged(name, blocks):
    """The benchmark's frame (vortex200k at 1920x1080 through the 256^3
    forest) and the serving volume's view, rendered by the FP32 kernel, which
    gathers block reloads, and by the FP16 kernel (which reloads at once for
    the vector frame and, for the one blob view, gathers as well), from the
    same block values: identical bit for bit."""
    import paper_1707_01170_amd as P
    say("[gpu] gathered reloads, full frame", name, blocks)
    wl, sc16 = scene(name, blocks=blocks, dtype="f16")
    _, sc32 = scene(name, blocks=blocks)
    view = wl.views[0]
    prm = P.RenderParams.of(wl)
    a, _, na = P.render(P.Scene(sc16.volume, prm), [view], nsamples=True)
    widened = sc16.volume.bezier.float()[:, :sc32.volume.bezier.shape[1]].contiguous()
    b, _, nb = P.render(P.Scene(sc32.volume, prm), [view], bezier=widened, nsamples=True)
    torch.cuda.synchronize()
    say("%s %dx%d: %d samples" % (name, view.width, view.height, int(nb.sum())))
    assert torch.equal(na, nb) and torch.equal(a, b)


@pytest.mark.parametrize("lookup", ["forest", "octree"])
def test_small_fp16_degree3_launch_equals_large(lookup):
    """Degree-3 scalar FP16 launches of at most 28 672 workgroups gather
    block reloads (one 1024^2 view: 16 384); a launch of four copies of the
    view (65 536) reloads at once: every copy equals the single view bit for
    bit, sample counts included."""
    import paper_1707_01170_amd as P
    say("[gpu] small and large FP16 degree-3 launches", lookup)
    wl = workload("blobs50k")
    vol = P.Volume(wl.spline, blocks=128, dtype="f16", lookup=lookup)
    sc = P.Scene(vol, P.RenderParams.of(wl))
    view = wl.views[0]
    assert (view.width, view.height) == (1024, 1024)
    a, _, na = P.render(sc, [view], nsamples=True, schedule=False)
    b, _, nb = P.render(sc, [view] * 4, nsamples=True, schedule=False)
    torch.cuda.synchronize()
    n = view.width * view.height
    for k in range(4):
        assert torch.equal(b[k * n:(k + 1) * n], a) and torch.equal(nb[k * n:(k + 1) * n], na), k


@pytest.mark.parametrize("name", ["blobs50k", "scalar20k"])
def test_fp16_blocks_with_octree_equal_fp32_on_widened_blocks(name):
    """The octree look-up with FP16 blocks: bit-identical to the FP32 octree
    kernel on the widened blocks, and to the forest's FP16 render."""
    import paper_1707_01170_amd as P
    say("[gpu] fp16 octree", name)
    wl = workload(name)
    v16 = P.Volume(wl.spline, lookup="octree", dtype="f16")
    v32 = P.Volume(wl.spline, lookup="octree")
    view = resized(wl.views[0], 80, 48)
    prm = P.RenderParams.of(wl)
    a, _, _ = P.render(P.Scene(v16, prm), [view])
    widened = v16.bezier.float()[:, :v32.bezier.shape[1]].contiguous()
    b, _, _ = P.render(P.Scene(v32, prm), [view], bezier=widened)
    _, sc16 = scene(name, blocks=64, dtype="f16")
    c, _, _ = P.render(P.Scene(sc16.volume, prm), [view])
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)

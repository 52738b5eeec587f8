"""Cost-ordered dispatch (lr_render_scheduled): the order in which blocks of
tiles are dealt changes no pixel, so every render equals lr_render's bit for
bit, including the per-pixel sample counts, for single and multi-launch view
sets, both look-up structures, fixed and adaptive steps, FP16 blocks and
shading; a too-small, null or misaligned workspace is an error.  The
persistent form (lr_render_persistent: workgroups taking tiles from one or
eight atomic counters, in either order, with the GPU-filling grid or a small
one) renders the same bits too."""
import ctypes
import dataclasses

import pytest
import torch

import lrgen
from conftest import workload
from gpu_util import resized, say, scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(sc, views, **kw):
    import paper_1707_01170_amd as P
    total = sum(v.width * v.height for v in views)
    outs = []
    for schedule in (False, True):
        out = torch.full((total, 4), -7.0, device="cuda:0")   # a pixel left unwritten would keep -7
        _, _, ns = P.render(sc, views, out=out, nsamples=True, schedule=schedule, **kw)
        outs.append((out, ns))
    torch.cuda.synchronize()
    (a, na), (b, nb) = outs
    return a, b, na, nb


@pytest.mark.parametrize("name,blocks,dtype,shading", [("vortex200k", 256, "f32", "none"),
                                                       ("vortex200k", 256, "f16", "headlight"),
                                                       ("blobs50k", 128, "f16", "none"),
                                                       ("scalar20k", 64, "f32", "none"),
                                                       ("scalar_ortho64", 16, "f32", "none")])
def test_scheduled_equals_ring_order(name, blocks, dtype, shading):
    import paper_1707_01170_amd as P
    say("[gpu] scheduled dispatch", name, blocks, dtype, shading)
    wl, sc = scene(name, blocks=blocks, dtype=dtype)
    if shading != "none":
        sc = P.Scene(sc.volume, dataclasses.replace(P.RenderParams.of(wl), shading=shading))
    a, b, na, nb = _both(sc, wl.views)
    say("%s: %d views, %d samples" % (name, len(wl.views), int(nb.sum())))
    assert bool((a != -7.0).all())
    assert torch.equal(a, b) and torch.equal(na, nb)


def test_scheduled_octree_and_many_views():
    """The octree look-up; 20 views of mixed sizes, so two launches reuse one workspace."""
    import paper_1707_01170_amd as P
    say("[gpu] scheduled dispatch, octree, 20 views")
    wl = workload("blobs50k")
    vol = P.Volume(wl.spline, lookup="octree", device="cuda:0")
    sc = P.Scene(vol, P.RenderParams.of(wl))
    import numpy as np
    rng = np.random.default_rng(5)
    dirs = lrgen.random_directions(rng, 20)
    sizes = [(40, 28), (96, 96), (200, 64), (17, 33), (128, 200)]
    views = [lrgen.sphere_view(dirs[k], *sizes[k % len(sizes)]) for k in range(20)]
    a, b, na, nb = _both(sc, views)
    assert bool((a != -7.0).all())
    assert torch.equal(a, b) and torch.equal(na, nb)


def _r256(b):
    return (b + 255) // 256 * 256


@pytest.mark.parametrize("name", ["vortex200k", "blobs50k"])
def test_dealing_order_in_workspace(name):
    """The dealing order the scheduled render leaves in its workspace, read
    back and checked against its definition: per view, every 16x16-pixel
    block in exactly one slot (the others -1); slot s on XCD s mod 8 (the
    hardware deals workgroups round-robin to the XCDs); the four blocks of a
    2x2 group on the XCD its group was dealt to (the XCD map); groups dealt
    evenly (counts per XCD differ by at most one); and each XCD's blocks in
    slots x, x + 8, ... by non-increasing estimate on the 64 levels of the
    view's largest estimate, without gaps.  Layout of the workspace: FP32
    estimates per block, one XCD byte per group, then int32 slots, each part
    256-byte aligned."""
    import numpy as np
    import paper_1707_01170_amd as P
    say("[gpu] dealing order in the workspace", name)
    wl, sc = scene(name, blocks=256 if name == "vortex200k" else 128)
    rng = np.random.default_rng(11)
    dirs = lrgen.random_directions(rng, 3)
    views = [wl.views[0], lrgen.sphere_view(dirs[0], 200, 120), lrgen.sphere_view(dirs[1], 33, 47),
             lrgen.sphere_view(dirs[2], 512, 512)]
    ws = P.render_workspace(views, "cuda:0")
    P.render(sc, views, workspace=ws)
    torch.cuda.synchronize()
    raw = ws.cpu().numpy()
    qdims = [((v.width + 15) // 16, (v.height + 15) // 16) for v in views]
    groups = [((qw + 1) // 2) * ((qh + 1) // 2) for qw, qh in qdims]
    nslots = [32 * ((g + 7) // 8) for g in groups]
    nq = sum(qw * qh for qw, qh in qdims)
    off_x = _r256(4 * nq)
    off_o = off_x + _r256(sum(nslots) // 4)
    assert raw.size == off_o + _r256(4 * sum(nslots))
    cost = raw[:4 * nq].view(np.float32)
    xmap = raw[off_x:off_x + sum(nslots) // 4].view(np.int8)
    order = raw[off_o:off_o + 4 * sum(nslots)].view(np.int32)
    qb = sb = 0
    for (qw, qh), ng, ns in zip(qdims, groups, nslots):
        c = cost[qb:qb + qw * qh]
        xm = xmap[sb // 4:sb // 4 + ng].astype(np.int64)
        sl = order[sb:sb + ns]
        assert np.all(c >= 0.0) and np.all((xm >= 0) & (xm < 8))
        blocks = sl[sl >= 0]
        assert np.array_equal(np.sort(blocks), np.arange(qw * qh)) and np.all(sl >= -1)
        gpx = np.bincount(xm, minlength=8)
        assert gpx.max() - gpx.min() <= 1, gpx
        mx = np.float32(c.max())
        scale = np.float32(63.0) / mx if mx > 0 else np.float32(0.0)
        level = 63 - np.clip((c * scale).astype(np.int32), 0, 63)
        for x in range(8):
            col = sl[x::8]
            k = int(np.sum(col >= 0))
            assert np.all(col[:k] >= 0) and np.all(col[k:] == -1), x
            b = col[:k]
            g = (b // qw // 2) * ((qw + 1) // 2) + (b % qw) // 2
            assert np.all(xm[g] == x), x
            assert np.all(np.diff(level[b]) >= 0), x
        qb += qw * qh
        sb += ns
    say("%s: %d views, %d blocks in %d slots" % (name, len(views), nq, sum(nslots)))


def test_workspace_errors():
    import paper_1707_01170_amd as P
    from paper_1707_01170_amd import _lib as L
    from paper_1707_01170_amd.api import _ptr, _stream, view_array
    say("[gpu] scheduled dispatch, workspace errors")
    wl, sc = scene("scalar20k")
    views = [resized(wl.views[0], 64, 48)]
    ws = P.render_workspace(views, "cuda:0")
    arr, _ = view_array(views)
    out = torch.empty((64 * 48, 4), device="cuda:0")
    s = sc.struct()
    lib = L.lib()
    n = ws.numel()
    assert lib.lr_render_scheduled(ctypes.byref(s), arr, 1, _ptr(out), None, _ptr(ws), n - 1, _stream()) == L.LR_ECAPACITY
    assert lib.lr_render_scheduled(ctypes.byref(s), arr, 1, _ptr(out), None, None, n, _stream()) == L.LR_EINVAL
    big = torch.empty(n + 512, dtype=torch.uint8, device="cuda:0")
    base = big[(-big.data_ptr()) % 256:]
    assert lib.lr_render_scheduled(ctypes.byref(s), arr, 1, _ptr(out), None, base.data_ptr() + 4, n, _stream()) == L.LR_EINVAL
    assert lib.lr_render_scheduled(ctypes.byref(s), arr, 1, _ptr(out), None, _ptr(ws), n, _stream()) == L.LR_OK
    torch.cuda.synchronize()


@pytest.mark.parametrize("name,blocks,dtype", [("vortex200k", 256, "f32"), ("blobs50k", 128, "f16"),
                                               ("scalar20k", 64, "f32"), ("scalar_ortho64", 16, "f32")])
def test_persistent_equals_hardware_dispatch(name, blocks, dtype):
    import paper_1707_01170_amd as P
    say("[gpu] persistent dispatch", name, blocks, dtype)
    wl, sc = scene(name, blocks=blocks, dtype=dtype)
    total = sum(v.width * v.height for v in wl.views)
    ref = torch.full((total, 4), -7.0, device="cuda:0")
    _, _, nref = P.render(sc, wl.views, out=ref, nsamples=True, schedule=False)
    torch.cuda.synchronize()
    assert bool((ref != -7.0).all())
    for queues in (1, 8):
        for order in (False, True):
            for wg in (0, 13):
                out = torch.full((total, 4), -7.0, device="cuda:0")
                _, _, ns = P.render(sc, wl.views, out=out, nsamples=True, schedule=order, queues=queues,
                                    workgroups=wg)
                torch.cuda.synchronize()
                assert torch.equal(out, ref) and torch.equal(ns, nref), (queues, order, wg)
    say("%s: %d views, identical in 8 persistent forms" % (name, len(wl.views)))


def test_persistent_many_views():
    """20 views of mixed sizes: two launches reuse the counters in one workspace."""
    import numpy as np

    import paper_1707_01170_amd as P
    say("[gpu] persistent dispatch, 20 views")
    wl, sc = scene("blobs50k", blocks=64, dtype="f32")
    rng = np.random.default_rng(7)
    dirs = lrgen.random_directions(rng, 20)
    sizes = [(40, 28), (96, 96), (200, 64), (17, 33), (128, 200)]
    views = [lrgen.sphere_view(dirs[k], *sizes[k % len(sizes)]) for k in range(20)]
    total = sum(v.width * v.height for v in views)
    ref, _, nref = P.render(sc, views, nsamples=True, schedule=False)
    for queues, order, wg in ((1, True, 0), (8, False, 8), (8, True, 24)):
        out = torch.full((total, 4), -7.0, device="cuda:0")
        _, _, ns = P.render(sc, views, out=out, nsamples=True, schedule=order, queues=queues, workgroups=wg)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(ns, nref), (queues, order, wg)


def test_persistent_errors():
    import paper_1707_01170_amd as P
    from paper_1707_01170_amd import _lib as L
    from paper_1707_01170_amd.api import _ptr, _stream, view_array
    say("[gpu] persistent dispatch, errors")
    wl, sc = scene("blobs50k", blocks=64, dtype="f32")
    views = [resized(wl.views[0], 64, 48)]
    ws = P.render_workspace(views, "cuda:0")
    arr, _ = view_array(views)
    out = torch.empty((64 * 48, 4), device="cuda:0")
    lib = L.lib()
    n = ws.numel()

    def call(s, queues=8, order=1, wg=0, w=ws.data_ptr(), nb=n):
        return lib.lr_render_persistent(ctypes.byref(s), arr, 1, _ptr(out), None, queues, order, wg, w, nb, _stream())

    s = sc.struct()
    assert call(s) == L.LR_OK
    assert call(s, nb=n - 1) == L.LR_ECAPACITY
    assert call(s, w=None) == L.LR_EINVAL
    assert call(s, queues=2) == L.LR_EINVAL
    assert call(s, order=2) == L.LR_EINVAL
    assert call(s, wg=-1) == L.LR_EINVAL
    oct_sc = P.Scene(P.Volume(wl.spline, lookup="octree", device="cuda:0"), P.RenderParams.of(wl))
    assert call(oct_sc.struct()) == L.LR_EINVAL
    lit = P.Scene(sc.volume, dataclasses.replace(P.RenderParams.of(wl), shading="headlight"))
    assert call(lit.struct()) == L.LR_EINVAL
    torch.cuda.synchronize()

"""lr_render_scheduled_noalloc, the allocation-free form of
lr_render_scheduled (its dispatch-order scratch is an array the library holds
on the GPU): called through the C ABI twice in a row, the second time with a
smaller input, it equals lr_render_scheduled's images and sample counts bit
for bit; a request beyond its scratch is rejected without rendering."""
import ctypes

import numpy as np
import pytest
import torch

import lrgen
from gpu_util import resized, say, scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _noalloc(sc, views):
    from paper_1707_01170_amd import _lib as L
    from paper_1707_01170_amd.api import _ptr, _stream, view_array
    arr, _ = view_array(views)
    total = sum(v.width * v.height for v in views)
    out = torch.full((total, 4), -7.0, device="cuda:0")
    ns = torch.zeros(total, dtype=torch.int32, device="cuda:0")
    s = sc.struct()
    st = L.lib().lr_render_scheduled_noalloc(ctypes.byref(s), arr, len(views), _ptr(out), _ptr(ns), _stream())
    assert st == L.LR_OK, L.lib().lr_last_error()
    return out, ns


def test_noalloc_equals_scheduled_twice_second_smaller():
    import paper_1707_01170_amd as P
    say("[gpu] no-alloc scheduled render")
    wl, sc = scene("vortex200k", blocks=256)
    big = [wl.views[0]]                                   # 1920 x 1080: 8 160 blocks
    small = [resized(wl.views[0], 320, 200), resized(wl.views[0], 64, 40)]
    for views in (big, small):
        out, ns = _noalloc(sc, views)
        ref, _, rns = P.render(sc, views, nsamples=True, schedule=True)
        torch.cuda.synchronize()
        say("no-alloc %d views, %d pixels" % (len(views), out.shape[0]))
        assert bool((out != -7.0).all())
        assert torch.equal(out, ref) and torch.equal(ns, rns)


def test_noalloc_rejects_beyond_its_scratch():
    from paper_1707_01170_amd import _lib as L
    from paper_1707_01170_amd.api import view_array
    say("[gpu] no-alloc scheduled render, too large")
    wl, sc = scene("scalar20k")
    rng = np.random.default_rng(1)
    views = [lrgen.sphere_view(d, 4096, 4096) for d in lrgen.random_directions(rng, 5)]   # 5 x 65 536 blocks
    arr, _ = view_array(views)
    s = sc.struct()
    st = L.lib().lr_render_scheduled_noalloc(ctypes.byref(s), arr, len(views), ctypes.c_void_p(1), None, None)
    assert st == L.LR_ECAPACITY
    assert b"scratch" in L.lib().lr_last_error()

"""The documented Python API end to end on the GPU (the usage shown in the
README): render, illumination, octree volumes, streamlines, and the autograd
chain from LR coefficients to the image, which must equal the two adjoint
entry points called by hand."""
import numpy as np
import pytest
import torch

from conftest import workload
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_documented_usage():
    import paper_1707_01170_amd as P
    say("[gpu] api usage")
    wl = workload("scalar20k")
    vol = P.Volume(wl.spline, blocks=128)
    views = list(wl.views)
    sc = P.Scene(vol, P.RenderParams.of(wl))
    rgba, offs, ns = P.render(sc, views, nsamples=True)
    imgs = P.unpack(rgba, views, offs)
    assert len(imgs) == 4 and imgs[0].shape == (512, 512, 4) and int(ns.sum()) > 0
    lit = P.Scene(vol, P.RenderParams.of(wl))
    lit.params.shading = "headlight"
    rl, _, _ = P.render(lit, views)
    assert torch.equal(rl[:, 3], rgba[:, 3]) and not torch.equal(rl[:, :3], rgba[:, :3])
    ov = P.Volume(wl.spline, lookup="octree")
    ro, _, _ = P.render(P.Scene(ov, P.RenderParams.of(wl)), views)
    assert torch.equal(ro, rgba)
    # autograd: coefficients -> blocks -> image
    coef = torch.tensor(wl.spline.coef, device="cuda", requires_grad=True)
    out = P.RenderFunction.apply(P.ExtractFunction.apply(coef, vol), sc.lut, sc, views)
    (out[:, :3] ** 2).sum().backward()
    gb, _ = P.render_backward(sc, views, out.detach(), torch.cat([2 * out.detach()[:, :3],
                                                               torch.zeros_like(out[:, 3:])], 1))
    gc = vol.extract_backward(gb)
    torch.cuda.synchronize()
    rel = float((coef.grad - gc).abs().max() / gc.abs().max())
    say("autograd chain vs explicit adjoints: %.3e" % rel)
    assert rel < 1e-5          # float atomics: summation order differs between the two runs


def test_streamlines_usage():
    import paper_1707_01170_amd as P
    wl = workload("vortex200k")
    vol = P.Volume(wl.spline, blocks=256)
    sc = P.Scene(vol, P.RenderParams.of(wl))
    pts, times, count = P.streamlines(sc, seeds=[[0.5, 0.6, 0.3], [0.45, 0.5, 0.5]], method="rk4",
                                      step="heuristic", precision="mixed", t_end=1.0)
    torch.cuda.synchronize()
    assert pts.shape == (2, 256, 4) and times.shape == (2, 256) and count.shape == (2,)
    c = count.cpu().numpy()
    assert np.all(c > 10) and torch.all(pts[0, : c[0], 3] == 1.0)

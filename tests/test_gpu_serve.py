"""Serving: continuous batching of mixed-resolution views (GPU)."""
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


class Req:
    def __init__(self, t, view):
        self.arrival_s = t
        self.view = view


def _stream(n, seed, sizes=(40, 64, 96, 128, 200)):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(0.002, n))
    dirs = lrgen.random_directions(rng, n)
    return [Req(float(t[k]), lrgen.sphere_view(dirs[k], int(rng.choice(sizes)), int(rng.choice(sizes))))
            for k in range(n)]


@pytest.mark.parametrize("dtype,time_scale,schedule", [("f32", 1.0, False), ("f16", 1.0, False), ("f32", 0.0, False),
                                                       ("f16", 0.05, False), ("f16", 0.0, True)])
def test_results_identical_alone_and_in_the_mix(dtype, time_scale, schedule):
    """Each request's image is the same bits alone and batched with others;
    time_scale compresses the arrivals (0: all at once), so that requests
    queue and launches carry several views; schedule: launches dealt by cost
    estimate (lr_render_scheduled, one workspace per stream)."""
    from paper_1707_01170_amd.serve import Server, render_alone
    say("[gpu] serve mix", dtype, time_scale, schedule)
    _, sc = scene("blobs50k", dtype=dtype)
    reqs = _stream(60, 1)
    srv = Server(sc, budget_bytes=16 * 200 * 200 * 6, n_streams=3, schedule=schedule)
    st = srv.run(reqs, keep_images=True, time_scale=time_scale)
    assert st.n == 60 and st.launches < 60 and st.max_inflight >= 1
    if time_scale == 0.0:
        assert st.mean_views_per_launch > 2.0
    for r in st.results:
        alone = render_alone(sc, reqs[r.index].view)
        assert torch.equal(r.image, alone), r.index
        assert r.latency_ms > 0
    say("serve mix %s: p50 %.2f ms p99 %.2f ms, %d launches, %.1f views/launch, max in flight %d"
        % (dtype, st.p50_ms, st.p99_ms, st.launches, st.mean_views_per_launch, st.max_inflight))


def test_scheduled_workspace_grows():
    """Cost-ordered serving sized up front for small launches: thin and large
    requests need more dealing-order workspace than that, the stream's
    workspace grows before such a launch, and every image is still the same
    bits as the request rendered alone."""
    from paper_1707_01170_amd.serve import Server, render_alone
    say("[gpu] serve, scheduled workspace growth")
    _, sc = scene("blobs50k", dtype="f16")
    rng = np.random.default_rng(4)
    dirs = lrgen.random_directions(rng, 24)
    shapes = [(1, 900), (700, 3), (16, 16), (300, 260), (5, 517), (64, 1000)]
    reqs = [Req(0.0, lrgen.sphere_view(dirs[k], *shapes[k % len(shapes)])) for k in range(24)]
    srv = Server(sc, budget_bytes=16 * 900 * 600, n_streams=2, max_pixels_per_launch=64 * 64, schedule=True)
    small = min(w.numel() for w in srv.workspaces)
    st = srv.run(reqs, keep_images=True, time_scale=0.0)
    assert st.n == 24 and max(w.numel() for w in srv.workspaces) > small
    for r in st.results:
        assert torch.equal(r.image, render_alone(sc, reqs[r.index].view)), r.index


def test_tight_budget_queues_instead_of_failing():
    from paper_1707_01170_amd.serve import Server
    _, sc = scene("scalar20k")
    reqs = _stream(30, 2, sizes=(128, 200))
    srv = Server(sc, budget_bytes=16 * 200 * 200 + 16, n_streams=2)   # one large request at a time
    st = srv.run(reqs)
    assert st.n == 30 and st.mean_views_per_launch <= 2.0
    with pytest.raises(ValueError):
        Server(sc, budget_bytes=16 * 64 * 64).run([Req(0.0, lrgen.sphere_view([1, 0, 0], 128, 128))])

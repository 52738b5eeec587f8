"""Streamlines on the GPU (Sec. 5) against the FP64 oracle on the vortex-tube
vector volume: constant steps point by point for all nine methods, the Eq. 4
heuristic step sequence, embedded error control and single vs mixed
precision through the error metric Eq. 7, look-up structures, stopping rules."""
import numpy as np
import pytest
import torch

from conftest import workload
from gpu_util import oracle_parts, say, scene

pytestmark = pytest.mark.gpu

NAME = "vortex200k"
METHODS = ["rk1", "rk2", "rk3", "rk4", "rk4_38", "rkf5", "he", "bs", "rkf45"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _seeds(n, seed=5):
    rng = np.random.default_rng(seed)
    r = 0.03 + 0.12 * rng.random(n)
    a = 2 * np.pi * rng.random(n)
    return np.stack([0.5 + r * np.cos(a), 0.5 + r * np.sin(a), 0.25 + 0.4 * rng.random(n)], 1)


def _field():
    ev = oracle_parts(NAME)[0]
    return lambda x: ev.evaluate(x)


def _gpu_lines(seeds, **kw):
    import paper_1707_01170_amd as P
    _, sc = scene(NAME, blocks=256)
    pts, tim, cnt = P.streamlines(sc, seeds, **kw)
    torch.cuda.synchronize()
    return pts.cpu().numpy(), tim.cpu().numpy(), cnt.cpu().numpy()


def _check_tail(j, k, pts, tim, cnt, base, t_end, max_samples, method="rk4", p_max=2):
    """A line that left the oracle's step sequence at point k must still be a
    valid line of the method from there: each later step h equals base times
    the Eq. 4 distance of the element at the GPU's own FP32 position (the last
    one shortened to land on t_end), each next point is the oracle's RK step
    of that h from the GPU's point (within the FP32 evaluation of the field
    and the FP32 rounding of the stored point), and the line ends at t_end, at
    max_samples, or where the next step would leave [0,1]^3.  Returns the
    largest position difference."""
    from oracle import streamline as ost
    wl = workload(NAME)
    f = _field()
    worst = 0.0
    n = int(cnt[j])
    for i in range(max(k - 1, 0), n - 1):
        x = pts[j, i, :3].astype(np.float64)
        h_exp = min(base * float(ost.heuristic_ds(wl.spline.elem_box, oracle_parts(NAME)[1], x[None], p_max)[0]),
                    t_end - tim[j, i])
        h_gpu = tim[j, i + 1] - tim[j, i]
        assert abs(h_gpu - h_exp) <= 4e-16 * max(1.0, t_end), (j, i, h_gpu, h_exp)
        x1, _, _ = ost.rk_step(f, x[None], np.array([h_gpu]), ost.TABLEAUS[method])
        d = float(np.abs(x1[0] - pts[j, i + 1, :3]).max())
        worst = max(worst, d)
        assert d <= 2e-6, (j, i, d)
    if n < max_samples and t_end - tim[j, n - 1] > 1e-12:
        x = pts[j, n - 1, :3].astype(np.float64)
        h = min(base * float(ost.heuristic_ds(wl.spline.elem_box, oracle_parts(NAME)[1], x[None], p_max)[0]),
                t_end - tim[j, n - 1])
        x1, _, _ = ost.rk_step(f, x[None], np.array([h]), ost.TABLEAUS[method])
        assert np.any((x1[0] < 1e-6) | (x1[0] > 1.0 - 1e-6)), (j, x1)
    return worst


@pytest.mark.parametrize("method", METHODS)
def test_constant_step_matches_oracle(method):
    """Same method, same constant step: the lines agree point by point to the
    FP32 evaluation of the field (FP64 outer loop on both sides)."""
    from oracle import streamline as ost
    say("[gpu] streamline constant", method)
    seeds = _seeds(24)
    kw = dict(method=method, step="constant", base=2.0 ** -7, t_end=0.125, max_samples=64)
    pts, tim, cnt = _gpu_lines(seeds, **kw)
    X, T, c = ost.integrate(_field(), seeds, method, "constant", kw["base"], kw["t_end"], kw["max_samples"])
    assert np.array_equal(cnt, c) and np.all(c == 17)
    for j in range(seeds.shape[0]):
        n = c[j]
        assert np.array_equal(tim[j, :n], T[j, :n])
        assert np.abs(pts[j, :n, :3] - X[j, :n]).max() <= 2e-6
        assert np.all(pts[j, :n, 3] == 1.0) and np.all(pts[j, n:] == 0.0)


def test_heuristic_steps_match_oracle():
    """Eq. 4 steps: the step sequence is decided on FP32 positions on both
    sides; lines whose positions stay clear of element faces follow the same
    sequence exactly (FP32 round-off can legitimately move a point across a
    face, after which the two sides take different but valid steps)."""
    from oracle import streamline as ost
    from oracle.lookup import ElementIndex
    say("[gpu] streamline heuristic")
    wl = workload(NAME)
    seeds = _seeds(48, 6)
    kw = dict(method="rk4", step="heuristic", base=1.0, t_end=0.25, max_samples=512)
    pts, tim, cnt = _gpu_lines(seeds, **kw)
    X, T, c = ost.integrate(_field(), seeds, "rk4", "heuristic", 1.0, 0.25, 512,
                            elem_box=wl.spline.elem_box, eidx=oracle_parts(NAME)[1], p_max=2)
    same = 0
    worst = 0.0
    for j in range(seeds.shape[0]):
        n = min(cnt[j], c[j])
        k = int(np.argmax(tim[j, :n] != T[j, :n])) if np.any(tim[j, :n] != T[j, :n]) else n
        assert k >= 2
        assert np.abs(pts[j, :k, :3] - X[j, :k]).max() <= 1e-5
        same += (k == n and cnt[j] == c[j])
        if not (k == n and cnt[j] == c[j]):
            worst = max(worst, _check_tail(j, k, pts, tim, cnt, 1.0, 0.25, 512))
    say("heuristic: %d of %d lines identical in their step sequence, %d..%d points; the others valid from "
        "where they part (largest step difference %.2e)" % (same, seeds.shape[0], cnt.min(), cnt.max(), worst))
    assert same >= 0.9 * seeds.shape[0]
    assert cnt.max() > 60


@pytest.mark.parametrize("method", ["he", "bs", "rkf45"])
def test_embedded_error_matches_oracle(method):
    """Embedded error control: both sides reach the same global error (Eq. 7
    against a small-step RKF5 reference) within a factor 2."""
    from oracle import streamline as ost
    say("[gpu] streamline embedded", method)
    wl = workload(NAME)
    seeds = _seeds(12, 7)
    f = _field()
    tol = 1e-6
    pts, tim, cnt = _gpu_lines(seeds, method=method, step="embedded", base=1.0, t_end=0.25, tol=tol,
                               max_samples=4096)
    X, T, c = ost.integrate(f, seeds, method, "embedded", 1.0, 0.25, 4096, elem_box=wl.spline.elem_box,
                            eidx=oracle_parts(NAME)[1], p_max=2, tol=tol)
    ref = ost.reference(f, seeds, 0.25, 2.0 ** -10)
    e_gpu = ost.error_metric(ref, pts[:, :, :3].astype(np.float64), tim, cnt)
    e_orc = ost.error_metric(ref, X, T, c)
    say("embedded %s: E gpu %.3e oracle %.3e, points gpu %d oracle %d" % (method, e_gpu, e_orc, cnt.sum(), c.sum()))
    # Lines with the same number of accepted steps, point by point.  The step
    # factors come from error estimates of FP32 (GPU) and FP64 (oracle) field
    # values, so the accepted times drift apart slightly; a point then differs
    # from the oracle's by the distance travelled in that time difference
    # (speed |f| times |dt|) plus the FP32 evaluation.
    equal = np.nonzero(cnt == c)[0]
    dx = dt = excess = 0.0
    for j in equal:
        n = c[j]
        d = np.abs(pts[j, :n, :3] - X[j, :n]).max(axis=1)
        tdiff = np.abs(tim[j, :n] - T[j, :n])
        speed = np.sqrt((f(np.clip(X[j, :n], 0.0, 1.0)) ** 2).sum(axis=1))
        dx, dt = max(dx, float(d.max())), max(dt, float(tdiff.max()))
        excess = max(excess, float((d - 1.5 * speed * tdiff).max()))
    say("embedded %s: %d of 12 lines with equal counts; point by point |dx| <= %.2e, |dt| <= %.2e, |dx| beyond "
        "the time difference <= %.2e" % (method, equal.size, dx, dt, excess))
    assert equal.size >= 9 and dt <= 1e-3 and excess <= 2e-6
    assert np.all(np.abs(T[np.arange(12), c - 1] - 0.25) < 1e-12)
    assert np.all(np.abs(tim[np.arange(12), cnt - 1] - 0.25) < 1e-12)
    assert e_gpu <= 2 * e_orc + 1e-7 and e_orc <= 2 * e_gpu + 1e-7


def test_mixed_precision_converges_where_single_stalls():
    """Sec. 5.6: with a small base step the FP32 outer loop stops converging;
    the FP64 outer loop with FP32 field evaluation keeps converging."""
    from oracle import streamline as ost
    say("[gpu] streamline precision")
    seeds = _seeds(8, 8)
    f = _field()
    ref = ost.reference(f, seeds, 0.125, 2.0 ** -12)
    errs = {}
    for prec in ("mixed", "single"):
        for base in (2.0 ** -7, 2.0 ** -11):
            pts, tim, cnt = _gpu_lines(seeds, method="rk4", step="constant", precision=prec, base=base, t_end=0.125,
                                       max_samples=4096)
            errs[prec, base] = ost.error_metric(ref, pts[:, :, :3].astype(np.float64), tim, cnt)
    say("precision: " + ", ".join("%s h=2^%d: %.3e" % (p, int(np.log2(b)), e) for (p, b), e in errs.items()))
    assert errs["mixed", 2.0 ** -11] < errs["single", 2.0 ** -11] / 4


def test_octree_lines_identical_to_forest():
    import paper_1707_01170_amd as P
    say("[gpu] streamline octree")
    wl = workload(NAME)
    vol = P.Volume(wl.spline, lookup="octree")
    sc = P.Scene(vol, P.RenderParams.of(wl))
    seeds = _seeds(64, 9)
    a = P.streamlines(sc, seeds, method="rk4", base=1.0, t_end=0.5, max_samples=512)
    b = _gpu_lines(seeds, method="rk4", base=1.0, t_end=0.5, max_samples=512)
    torch.cuda.synchronize()
    assert np.array_equal(a[0].cpu().numpy(), b[0]) and np.array_equal(a[2].cpu().numpy(), b[2])


def test_stopping_rules_on_the_gpu():
    """Time limit landed on, sample cap, domain exit (points stay in [0,1]^3),
    inactive entries after the end."""
    say("[gpu] streamline stopping")
    seeds = np.concatenate([_seeds(8, 10), [[0.5, 0.5, 0.97], [0.02, 0.5, 0.5]]])
    pts, tim, cnt = _gpu_lines(seeds, method="rk2", base=1.0, t_end=3.0, max_samples=2048)
    for j in range(seeds.shape[0]):
        n = cnt[j]
        assert np.all((pts[j, :n, :3] >= 0) & (pts[j, :n, :3] <= 1)) and np.all(pts[j, n:] == 0)
    assert cnt[8] < 2048 and tim[8, cnt[8] - 1] < 3.0       # leaves through z = 1
    pts, tim, cnt = _gpu_lines(seeds, method="rk2", base=1.0, t_end=0.01, max_samples=2048)
    assert np.all(np.abs(tim[np.arange(10), cnt - 1] - 0.01) <= 1e-17)
    pts, tim, cnt = _gpu_lines(seeds, method="rk2", base=1.0, t_end=3.0, max_samples=5)
    assert np.all(cnt == 5)


def test_bench_configuration_sampled():
    """The launch the benchmark times (16 384 seeds, RK4 with the Eq. 4
    step, mixed precision, t_end 1, at most 2048 points), checked on a
    spread of its lines against the oracle as in the heuristic test."""
    import os
    import sys
    from oracle import streamline as ost
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    say("[gpu] streamline bench configuration")
    wl = workload(NAME)
    seeds = bench._stream_seeds(16384)
    kw = dict(method="rk4", step="heuristic", precision="mixed", base=1.0, t_end=1.0, max_samples=2048)
    pts, tim, cnt = _gpu_lines(seeds, **kw)
    pick = np.linspace(0, len(seeds) - 1, 16).astype(np.int64)
    X, T, c = ost.integrate(_field(), seeds[pick], "rk4", "heuristic", 1.0, 1.0, 2048,
                            elem_box=wl.spline.elem_box, eidx=oracle_parts(NAME)[1], p_max=2)
    same = 0
    worst = 0.0
    for n_, j in enumerate(pick):
        n = min(cnt[j], c[n_])
        d = tim[j, :n] != T[n_, :n]
        k = int(np.argmax(d)) if np.any(d) else n
        assert k >= 2
        assert np.abs(pts[j, :k, :3] - X[n_, :k]).max() <= 1e-5
        same += (k == n and cnt[j] == c[n_])
        if not (k == n and cnt[j] == c[n_]):
            worst = max(worst, _check_tail(j, k, pts, tim, cnt, 1.0, 1.0, 2048))
    say("bench configuration: %d of %d sampled lines identical, %d..%d points over all lines; the others "
        "valid from where they part (largest step difference %.2e)" % (same, len(pick), cnt.min(), cnt.max(), worst))
    assert same >= 0.75 * len(pick)
    assert np.all(cnt >= 2) and cnt.max() <= 2048


@pytest.mark.parametrize("p", [1, 3])
def test_other_degrees_match_oracle(p):
    """Vector fields of degree 1 and 3: each lane of a seed's group loads its
    component from a different offset of the block row (16-byte aligned for
    these degrees, with the window clipped at the row's end); constant RK4
    steps point by point against the oracle, mixed and single precision."""
    import lrgen
    import paper_1707_01170_amd as P
    from oracle import streamline as ost
    from oracle.bspline import LREvaluator
    say("[gpu] streamline degree", p)
    s = lrgen.small_random(p=(p, p, p), n=(4, 4, 4), n_ref=30, seed=60 + p, ncomp=3)
    s = s.with_coef(s.coef - 0.5)                   # centred components: lines wander, few leave early
    wl = lrgen.Workload("deg", s, lrgen.default_lut(), 0.0, 1.0, "adaptive", 64, "hue",
                        [lrgen.sphere_view([0.3, -0.8, 0.5], 8, 8)])
    sc = P.Scene(P.Volume(s, blocks=8), P.RenderParams.of(wl))
    seeds = _seeds(40, 9)
    ev = LREvaluator(s)
    for prec, tol in (("mixed", 2e-6), ("single", 2e-5)):
        kw = dict(method="rk4", step="constant", precision=prec, base=2.0 ** -7, t_end=0.125, max_samples=64)
        pts, tim, cnt = P.streamlines(sc, seeds, **kw)
        torch.cuda.synchronize()
        pts, tim, cnt = pts.cpu().numpy(), tim.cpu().numpy(), cnt.cpu().numpy()
        X, T, c = ost.integrate(lambda x: ev.evaluate(x), seeds, "rk4", "constant", kw["base"], kw["t_end"], 64)
        assert np.array_equal(cnt, c) and c.max() == 17 and c.min() >= 2
        for j in range(seeds.shape[0]):
            n = c[j]
            assert np.abs(pts[j, :n, :3] - X[j, :n]).max() <= tol, (prec, j)
            assert np.all(pts[j, :n, 3] == 1.0) and np.all(pts[j, n:] == 0.0)

"""Host-side streamline error metric (Eq. 7) of the package: cubic Lagrange
reading of a reference grid and the weighted sum, against closed forms."""
import numpy as np

from paper_1707_01170_amd import metrics


def _curve(t):
    return np.stack([0.1 + 0.3 * t - 0.2 * t ** 2 + 0.05 * t ** 3, 0.5 + 0.1 * t ** 3, 0.2 + 0.4 * t], -1)


def test_cubic_reference_is_read_exactly():
    h = 1.0 / 64
    grid = np.arange(0, 65) * h
    ref = (h, _curve(grid)[None], np.array([65]))
    t = np.random.default_rng(0).random(200)
    assert np.abs(metrics._at(ref, 0, t) - _curve(t)).max() < 1e-14


def test_metric_of_offset_lines():
    h = 1.0 / 64
    grid = np.arange(0, 65) * h
    ref = (h, np.stack([_curve(grid), _curve(grid)]), np.array([65, 65]))
    t = np.linspace(0, 1, 33)
    pts = np.stack([_curve(t), _curve(t) + np.array([0.0, 3e-3, 4e-3])])
    times = np.stack([t, t])
    assert abs(metrics.error_metric(ref, pts, times, np.array([33, 33])) - 5e-3) < 1e-13
    # points past the end of a shorter reference are left out
    ref2 = (h, ref[1], np.array([65, 33]))
    assert abs(metrics.error_metric(ref2, pts, times, np.array([33, 33])) - 5e-3 * 0.5) < 1e-13

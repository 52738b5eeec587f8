"""Host logic of the serving loop: the output-memory arena (no device)."""
import numpy as np
import pytest
import torch

from paper_1707_01170_amd.serve import Arena


def test_arena_first_fit_and_merge():
    a = Arena(100, "cpu")
    x = a.alloc(40)
    y = a.alloc(40)
    assert (x, y) == (0, 40)
    assert a.alloc(30) is None                  # only 20 left
    a.release(x, 40)
    assert a.alloc(30) == 0                     # reuses the freed hole
    a.release(0, 30)
    a.release(y, 40)
    assert a.free == [(0, 100)]                 # everything merged back


def test_arena_random_never_overlaps():
    rng = np.random.default_rng(0)
    a = Arena(1000, "cpu")
    live = {}
    for step in range(2000):
        if live and rng.random() < 0.5:
            k = list(live)[rng.integers(len(live))]
            a.release(k, live.pop(k))
        else:
            n = int(rng.integers(1, 200))
            s = a.alloc(n)
            if s is not None:
                for t, m in live.items():
                    assert s + n <= t or t + m <= s
                assert 0 <= s and s + n <= 1000
                live[s] = n
        assert sum(l for _, l in a.free) + sum(live.values()) == 1000

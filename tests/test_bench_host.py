"""Host-side pieces of the benchmark: the algorithmic operation count it
prices the render kernel with, the code digest that keeps the committed HBM
counters attached to the kernel code they were taken on, and the refusal of
multi-GPU runs."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_flops_per_sample_counts():
    # the hot-path scope table's per-sample totals: 133 (degree-2 scalar),
    # 238 (degree-3 scalar), 325 (degree-2 3-vector)
    assert bench.flops_per_sample(2, 1) == 15 + 2 * (27 + 9 + 3) + 40 == 133
    assert bench.flops_per_sample(3, 1) == 30 + 2 * (64 + 16 + 4) + 40 == 238
    assert bench.flops_per_sample(2, 3) == 15 + 2 * (27 + 9 + 3) * 3 + 40 + 36 == 325
    # the adjoint's scatter of dv/dC_j = B_j(u): 2 (p+1)^3 + 2 (p+1)^2
    for p in (1, 2, 3):
        assert bench.ADJOINT_EXTRA_FLOPS[p] == 70 + 2 * (p + 1) ** 3 + 2 * (p + 1) ** 2


def test_accuracy_is_peak_relative():
    import numpy as np
    import torch

    class V:
        width, height = 4, 3
    ref = np.zeros((3, 4), np.float64)
    ref[:, 3] = 0.5
    ii, jj = np.array([0, 3, 2]), np.array([0, 1, 2])
    frame = torch.zeros((12, 4))
    frame[jj * 4 + ii] = torch.from_numpy(ref).float()
    frame[1 * 4 + 3, 3] = 0.51
    a = bench.accuracy(frame, V, (ii, jj, ref))
    assert abs(a["max"] - 0.01 / 0.5) < 1e-6
    assert abs(a["rms"] - np.sqrt(0.01 ** 2 / 12) / 0.5) < 1e-6


def _copy_sources(dst):
    d = os.path.join(dst, "paper_1707_01170_amd", "csrc")
    os.makedirs(d)
    for name in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1707_01170_amd", "csrc", name)) as f, \
                open(os.path.join(d, name), "w") as g:
            g.write(f.read())
    return d


def test_kernel_digest_ignores_comments_not_code(tmp_path, monkeypatch):
    d = _copy_sources(str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_digest()
    p = os.path.join(d, "render.hip")
    src = open(p).read()
    open(p, "w").write("// a new comment\n/* and a\n block one */\n" + src.replace("\n", "\n\n", 3))
    assert bench.kernel_digest() == base
    open(p, "w").write(src.replace("kQuad = 2", "kQuad = 4", 1))
    assert bench.kernel_digest() != base
    open(p, "w").write(src)
    q = os.path.join(d, "eval.h")
    ev = open(q).read()
    open(q, "w").write(ev + "\nconstexpr int kUnused = 1;\n")
    assert bench.kernel_digest() != base


def test_measured_traffic_tracks_the_code(tmp_path, monkeypatch):
    import shutil
    d = _copy_sources(str(tmp_path))
    os.makedirs(os.path.join(str(tmp_path), "profiles"))
    shutil.copy(os.path.join(ROOT, "profiles", "render_kernel_vector1080p_traffic.json"),
                os.path.join(str(tmp_path), "profiles"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    t = bench.measured_traffic(256)
    if t is None:
        pytest.skip("the render kernel changed since its counters were taken")
    assert t > 0 and bench.measured_traffic(128) is None
    p = os.path.join(d, "render.hip")
    open(p, "a").write("\nstatic int changed_code;\n")
    assert bench.measured_traffic(256) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_per_config_workloads():
    """The other workloads of the bench line: each names a cached workload
    with views, the serving entry picks the stream's first 2048^2 request,
    and the forest and storage are ones the library builds."""
    for name, label, blocks, dtype, which in bench.PER_CONFIG:
        wl, views = bench.per_config_views(name, which)
        assert views and label and dtype in ("f32", "f16")
        assert blocks in (16, 64, 128, 256)
        if which == "serve2048":
            assert (views[0].width, views[0].height) == (2048, 2048)
        else:
            assert views == list(wl.views)
    names = [c[0] for c in bench.PER_CONFIG]
    assert names == ["scalar_ortho64", "blobs50k", "blobs50k", "scalar20k"]

"""The host builders of the C ABI (support CSR, k-d forest, octree) compiled
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer from the
library's host sources only, and driven over generated meshes: memory and
undefined-behaviour errors abort the driver, and every element centre must
descend to its element."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import lrgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_01170_amd", "csrc")
SOURCES = ["capi.cpp", "forest.cpp", "octree.cpp", "support.cpp"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")] + [os.path.join(CSRC, s) for s in SOURCES] + \
          ["-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def _write(path, spline, dyadic):
    p = np.asarray(spline.p, dtype=np.int32)
    kn = np.ascontiguousarray(spline.knots, dtype=np.float64)
    eb = np.ascontiguousarray(spline.elem_box, dtype=np.float64)
    with open(path, "wb") as f:
        f.write(p.tobytes())
        f.write(np.int64(kn.shape[0]).tobytes())
        f.write(np.int32(kn.shape[2]).tobytes())
        f.write(kn.tobytes())
        f.write(np.int64(eb.shape[0]).tobytes())
        f.write(eb.tobytes())
        f.write(np.int32(1 if dyadic else 0).tobytes())


@pytest.mark.parametrize("case", ["deg2", "deg3_cluster", "deg1", "tensor", "scalar20k"])
def test_host_builders_under_sanitizers(driver, tmp_path, case):
    if case == "scalar20k":
        s = lrgen.cached("scalar20k").spline
    else:
        s = {"deg2": lambda: lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=60, seed=3),
             "deg3_cluster": lambda: lrgen.small_random(p=(3, 3, 3), n=(2, 2, 2), n_ref=50, seed=4, dist="cluster"),
             "deg1": lambda: lrgen.small_random(p=(1, 1, 1), n=(4, 8, 2), n_ref=40, seed=5),
             "tensor": lambda: lrgen.tensor_spline((2, 2, 2), (2, 4, 8))}[case]()
    dyadic = bool(np.all(np.ldexp(s.elem_box, 24) == np.round(np.ldexp(s.elem_box, 24))))
    path = str(tmp_path / "mesh.bin")
    _write(path, s, dyadic)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, path], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "ALL OK" in r.stdout, (r.stdout[-3000:], r.stderr[-3000:])

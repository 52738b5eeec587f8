"""C ABI: the library loads, exports what include/lrvr.h declares, rejects bad
input with the documented status, and its host builders (k-d forest, element /
B-spline incidence) agree with brute force.  No device calls."""
import ctypes
import os
import re

import numpy as np
import pytest

import lrgen
from conftest import ROOT, workload
from oracle.bspline import LREvaluator
from oracle.lookup import ElementIndex, find_element_scan

P = pytest.importorskip("paper_1707_01170_amd")
from paper_1707_01170_amd import _lib as L  # noqa: E402


def _declared():
    src = open(os.path.join(ROOT, "include", "lrvr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lr_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared()
    assert {"lr_build_forest", "lr_extract_bezier", "lr_render", "lr_render_backward"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.SIGNATURES), "binding and header disagree"
    assert lib.lr_version() >= 100


def test_struct_sizes():
    assert ctypes.sizeof(L.ViewC) == 80 and ctypes.sizeof(L.SceneC) == 128
    assert P.bezier_stride((2, 2, 2), 1, L.LR_F32) == 28
    assert P.bezier_stride((3, 3, 3), 1, L.LR_F32) == 64
    assert P.bezier_stride((2, 2, 2), 3, L.LR_F32) == 84
    assert P.bezier_stride((2, 2, 2), 3, L.LR_F16) == 88
    assert P.bezier_stride((4, 2, 2), 1, L.LR_F32) == -1


def _forest_status(box, blocks):
    lib = L.lib()
    eb = np.ascontiguousarray(box, dtype=np.float64)
    b = np.asarray(blocks, dtype=np.int32)
    h = ctypes.c_void_p()
    st = lib.lr_build_forest(eb.ctypes.data, eb.shape[0], b.ctypes.data, ctypes.byref(h), None)
    if st == 0:
        lib.lr_forest_free(h)
    return st, lib.lr_last_error().decode()


def test_forest_errors():
    unit = np.array([[0, 0, 0, 1, 1, 1.0]])
    assert _forest_status(unit, (4, 4, 4))[0] == L.LR_OK
    assert _forest_status(unit, (3, 4, 4))[0] == L.LR_ENOTPOW2
    assert _forest_status(unit, (1024, 1, 1))[0] == L.LR_ENOTPOW2
    half = np.array([[0, 0, 0, 0.1, 1, 1.0], [0.1, 0, 0, 1, 1, 1.0]])
    st, msg = _forest_status(half, (2, 2, 2))
    assert st == L.LR_EKNOT and "FP32" in msg
    gap = np.array([[0, 0, 0, 0.5, 1, 1.0]])
    assert _forest_status(gap, (2, 2, 2))[0] == L.LR_EPARTITION
    overlap = np.array([[0, 0, 0, 0.75, 1, 1.0], [0.25, 0, 0, 1, 1, 1.0], [0.0, 0, 0, 0.0625, 0.0625, 0.0625]])
    assert _forest_status(overlap, (2, 2, 2))[0] == L.LR_EPARTITION
    with pytest.raises(L.LRError):
        P.Forest.build(gap, 2)


def descend(forest, p):
    """Alg. 1 over the exported arrays (test-side reimplementation)."""
    B = np.array(forest.blocks)
    pf = p.astype(np.float32)
    c = np.minimum((pf * B.astype(np.float32)).astype(np.int64), B - 1)
    out = np.empty(p.shape[0], dtype=np.int64)
    split = forest.nodes[:, 2].view(np.float32) if forest.nodes.shape[0] else None
    for k in range(p.shape[0]):
        r = int(forest.heads[(c[k, 2] * B[1] + c[k, 1]) * B[0] + c[k, 0]])
        while not r & L.LR_LEAF:
            n = forest.nodes[r]
            r = int(n[0] if pf[k, n[3]] < split[r] else n[1])
        out[k] = r & ~L.LR_LEAF
    return out


def _probe_points(box, n, seed):
    rng = np.random.default_rng(seed)
    faces = np.concatenate([box[:, [0, 1, 2]], box[:, [3, 4, 5]], box[:, [3, 1, 2]], box[:, [0, 4, 5]],
                            0.5 * (box[:, :3] + box[:, 3:])])
    return np.concatenate([rng.random((n, 3)).astype(np.float32).astype(np.float64), faces])


@pytest.mark.parametrize("blocks", [1, 2, (4, 2, 8), 16])
def test_forest_descent_equals_scan(blocks):
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=80, seed=21, dist="cluster")
    f = P.Forest.build(s.elem_box, blocks)
    x = _probe_points(s.elem_box, 3000, 1)
    assert np.array_equal(descend(f, x), ElementIndex(s.elem_box).find(x))
    assert np.array_equal(descend(f, x[:400]), find_element_scan(s.elem_box, x[:400]))
    assert f.stats["n_heads"] == np.prod(np.broadcast_to(blocks, 3))


def test_forest_matches_figure():
    """Golden: the paper's k-d forest figure (Sec. 3.2.1)."""
    names, boxes, trees = [], [], {}
    for line in open(os.path.join(ROOT, "tests", "golden", "kdforest_fig.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if ":" in line:
            k, v = line.split(":")
            trees[k] = v.split()
        else:
            tok = line.split()
            names.append(tok[0])
            boxes.append([float(t) for t in tok[1:]])
    f = P.Forest.build(np.array(boxes), 2)

    def preorder(r):
        if r & L.LR_LEAF:
            return [names[r & ~L.LR_LEAF]]
        n = f.nodes[r]
        s = float(np.float32(n[2:3].view(np.float32)[0]))
        return ["xyz"[n[3]] + "<" + repr(s)] + preorder(int(n[0])) + preorder(int(n[1]))

    def norm(tok):
        return [t if "<" not in t else t.split("<")[0] + "<" + repr(float(t.split("<")[1])) for t in tok]

    assert preorder(int(f.heads[0])) == norm(trees["P000"])
    assert preorder(int(f.heads[7])) == norm(trees["P111"])
    assert f.stats["max_depth"] == 3


def test_forest_depth_stats():
    s = workload("config1").spline
    f = P.Forest.build(s.elem_box, 4)
    st = f.stats
    assert st["min_depth"] == 0 and st["max_depth"] >= 1
    # single element per block at a fine forest: every head is direct
    t = lrgen.tensor_spline((2, 2, 2), (4, 4, 4))
    f2 = P.Forest.build(t.elem_box, 8)
    assert f2.stats["n_direct"] == 512 and f2.stats["max_depth"] == 0 and f2.stats["n_nodes"] == 0
    f1 = P.Forest.build(t.elem_box, 1)      # one k-d tree over 64 elements: balanced, depth 6
    assert f1.stats["max_depth"] == 6 and f1.stats["n_nodes"] == 63


def test_support_csr_matches_oracle():
    for s in (workload("config1").spline, lrgen.small_random(p=(3, 3, 3), n=(3, 3, 3), n_ref=40, seed=5)):
        ptr, idx = P.support_csr(s)
        ev = LREvaluator(s)
        for e in range(0, s.n_elem, max(1, s.n_elem // 60)):
            assert np.array_equal(idx[ptr[e]:ptr[e + 1]], ev.bsplines_on_element(s.elem_box[e]))
        assert np.all(np.diff(ptr) >= np.prod([q + 1 for q in s.p]))

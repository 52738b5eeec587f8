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


def test_build_id_matches_sources():
    """The loaded library was built from the sources in the tree."""
    from paper_1707_01170_amd import _build
    assert L.lib().lr_build_id().decode() == _build.source_digest()


def test_forest_device_size_query():
    """lr_build_forest_device, phase 1 (no device buffers): the sizes and
    statistics of the host build, and its argument checks; nothing touches a
    device."""
    lib = L.lib()
    s = lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=30, seed=3)
    eb = np.ascontiguousarray(s.elem_box, dtype=np.float32)
    for blocks in (1, 4):
        ref = P.Forest.build(s.elem_box, blocks)
        b = np.array([blocks] * 3, np.int32)
        nn = ctypes.c_int64(-1)
        st = L.ForestStats()
        assert lib.lr_build_forest_device(eb.ctypes.data, eb.shape[0], b.ctypes.data, None, None, 0,
                                          ctypes.byref(nn), ctypes.byref(st), None) == L.LR_OK
        assert nn.value == ref.stats["n_nodes"] == st.n_nodes and st.n_heads == blocks ** 3
        assert st.max_depth == ref.stats["max_depth"]
    f = ctypes.c_void_p(0x1000)
    b = np.array([4, 4, 4], np.int32)
    assert lib.lr_build_forest_device(eb.ctypes.data, eb.shape[0], b.ctypes.data, f, None, 5, None, None,
                                      None) == L.LR_EINVAL
    assert lib.lr_build_forest_device(eb.ctypes.data, eb.shape[0], b.ctypes.data, None, f, 5, None, None,
                                      None) == L.LR_EINVAL
    b = np.array([4, 3, 4], np.int32)
    assert lib.lr_build_forest_device(eb.ctypes.data, eb.shape[0], b.ctypes.data, None, None, 0, None, None,
                                      None) == L.LR_ENOTPOW2
    b = np.array([1, 1, 1], np.int32)
    small = ctypes.c_int64()
    lib.lr_build_forest_device(eb.ctypes.data, eb.shape[0], b.ctypes.data, None, None, 0, ctypes.byref(small),
                               None, None)
    assert small.value > 1
    assert lib.lr_build_forest_device(eb.ctypes.data, eb.shape[0], b.ctypes.data, f, f, small.value - 1, None, None,
                                      None) == L.LR_ECAPACITY


def test_struct_sizes():
    assert ctypes.sizeof(L.ViewC) == 80 and ctypes.sizeof(L.SceneC) == 144
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
    s = workload("scalar_ortho64").spline
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
    for s in (workload("scalar_ortho64").spline, lrgen.small_random(p=(3, 3, 3), n=(3, 3, 3), n_ref=40, seed=5)):
        ptr, idx = P.support_csr(s)
        ev = LREvaluator(s)
        for e in range(0, s.n_elem, max(1, s.n_elem // 60)):
            assert np.array_equal(idx[ptr[e]:ptr[e + 1]], ev.bsplines_on_element(s.elem_box[e]))
        assert np.all(np.diff(ptr) >= np.prod([q + 1 for q in s.p]))


def _scene_struct(**kw):
    s = L.SceneC()
    s.p[:] = kw.get("p", (2, 2, 2))
    s.ncomp = kw.get("ncomp", 1)
    s.n_elem = kw.get("n_elem", 10)
    fake = 0x1000                      # never dereferenced: validation fails first
    s.elem_box = s.bezier = s.heads = s.nodes = s.lut = fake
    s.bezier_dtype = kw.get("dtype", L.LR_F32)
    s.blocks[:] = kw.get("blocks", (4, 4, 4))
    s.n_nodes = 1
    s.vmin, s.vmax, s.xi = kw.get("vmin", 0.0), kw.get("vmax", 1.0), kw.get("xi", 1.0)
    s.alpha_clamp, s.term_alpha = kw.get("alpha_clamp", 0.99), 0.99
    s.step_mode = kw.get("step_mode", L.LR_STEP_ADAPTIVE)
    s.n_fixed_steps = kw.get("n_fixed_steps", 0)
    s.color_mode = kw.get("color_mode", L.LR_COLOR_LUT)
    s.max_samples = kw.get("max_samples", 100)
    s.lookup = kw.get("lookup", L.LR_LOOKUP_FOREST)
    s.shading = kw.get("shading", L.LR_SHADE_NONE)
    s.light[:] = kw.get("light", (0.0, 0.0, 1.0))
    return s


@pytest.mark.parametrize("kw,status", [
    ({"p": (2, 3, 2)}, L.LR_EINVAL),               # render kernels take equal degrees
    ({"p": (4, 4, 4)}, L.LR_EINVAL),
    ({"ncomp": 3}, L.LR_EINVAL),                   # 3 components need the hue colour mode
    ({"dtype": L.LR_F64}, L.LR_EINVAL),
    ({"blocks": (3, 4, 4)}, L.LR_ENOTPOW2),
    ({"vmax": 0.0}, L.LR_EINVAL),
    ({"xi": 0.0}, L.LR_EINVAL),
    ({"alpha_clamp": 1.0}, L.LR_EINVAL),
    ({"step_mode": L.LR_STEP_FIXED, "n_fixed_steps": 0}, L.LR_EINVAL),
    ({"max_samples": 0}, L.LR_EINVAL),
    ({"lookup": 2}, L.LR_EINVAL),
    ({"shading": 3}, L.LR_EINVAL),
    ({"shading": L.LR_SHADE_DIRECTIONAL, "light": (0.0, 0.0, 0.0)}, L.LR_EINVAL),
    ({"shading": L.LR_SHADE_HEADLIGHT, "lookup": L.LR_LOOKUP_OCTREE}, L.LR_EINVAL),
])
def test_render_rejects_bad_scene(kw, status):
    import lrgen
    lib = L.lib()
    s = _scene_struct(**kw)
    arr, _ = P.api.view_array([lrgen.sphere_view([1, 0, 0], 8, 8)])
    assert lib.lr_render(ctypes.byref(s), arr, 1, ctypes.c_void_p(0x1000), None, None) == status
    assert lib.lr_last_error()


def test_render_rejects_bad_views():
    import lrgen
    lib = L.lib()
    s = _scene_struct()
    v = lrgen.sphere_view([1, 0, 0], 8, 8)
    arr, _ = P.api.view_array([v])
    assert lib.lr_render(ctypes.byref(s), arr, 0, ctypes.c_void_p(0x1000), None, None) == L.LR_EINVAL
    assert lib.lr_render(ctypes.byref(s), arr, 1, None, None, None) == L.LR_EINVAL
    arr[0].width = 0
    assert lib.lr_render(ctypes.byref(s), arr, 1, ctypes.c_void_p(0x1000), None, None) == L.LR_EINVAL
    arr[0].width = 8
    arr[0].proj = 7
    assert lib.lr_render(ctypes.byref(s), arr, 1, ctypes.c_void_p(0x1000), None, None) == L.LR_EINVAL
    arr[0].proj = L.LR_PERSP
    arr[0].eye[0] = float("inf")
    assert lib.lr_render(ctypes.byref(s), arr, 1, ctypes.c_void_p(0x1000), None, None) == L.LR_EINVAL


def test_backward_rejects_vector_f16_and_shading():
    import lrgen
    lib = L.lib()
    arr, _ = P.api.view_array([lrgen.sphere_view([1, 0, 0], 8, 8)])
    f = ctypes.c_void_p(0x1000)
    s = _scene_struct(ncomp=3, color_mode=L.LR_COLOR_HUE)
    assert lib.lr_render_backward(ctypes.byref(s), arr, 1, f, f, f, f, None) == L.LR_EINVAL
    s = _scene_struct(dtype=L.LR_F16)
    assert lib.lr_render_backward(ctypes.byref(s), arr, 1, f, f, f, f, None) == L.LR_EINVAL
    s = _scene_struct(shading=L.LR_SHADE_HEADLIGHT)
    assert lib.lr_render_backward(ctypes.byref(s), arr, 1, f, f, f, f, None) == L.LR_EINVAL
    assert b"shading" in lib.lr_last_error()


def test_lookup_and_extract_validate_first():
    lib = L.lib()
    f = ctypes.c_void_p(0x1000)
    b = np.array([3, 4, 4], np.int32)
    assert lib.lr_lookup(f, f, 1, b.ctypes.data, 10, f, 5, f, None) == L.LR_ENOTPOW2
    b = np.array([4, 4, 4], np.int32)
    assert lib.lr_lookup(f, f, 1, b.ctypes.data, 10, f, 0, f, None) == L.LR_OK       # empty batch
    assert lib.lr_lookup(f, f, 1, b.ctypes.data, 0, f, 5, f, None) == L.LR_EINVAL
    # the grid of 256-point workgroups must fit 2^31 - 1 workgroups
    assert lib.lr_lookup(f, f, 1, b.ctypes.data, 10, f, 0x7fffffff * 256 + 1, f, None) == L.LR_EINVAL
    assert lib.lr_lookup_octree(f, f, 1, 10, f, 0x7fffffff * 256 + 1, f, None) == L.LR_EINVAL
    assert b"too many points" in lib.lr_last_error()
    s = L.LRSplineDev()
    s.p[:] = (2, 2, 2)
    s.ncomp, s.kstride, s.n_bspl, s.n_elem = 1, 4, 10, 5
    s.knots = s.coef = s.gamma = s.elem_box = s.csr_ptr = s.csr_idx = 0x1000
    assert lib.lr_extract_bezier(ctypes.byref(s), 7, f, None, None) == L.LR_EINVAL
    s.kstride = 3
    assert lib.lr_extract_bezier(ctypes.byref(s), L.LR_F32, f, None, None) == L.LR_EINVAL
    s.kstride, s.ncomp = 4, 5
    assert lib.lr_extract_bezier(ctypes.byref(s), L.LR_F32, f, None, None) == L.LR_EINVAL
    # adjoint of the extraction: same checks, plus its own dtype and pointers
    s.ncomp = 1
    assert lib.lr_extract_bezier_backward(ctypes.byref(s), L.LR_F16, f, f, None) == L.LR_EINVAL
    assert lib.lr_extract_bezier_backward(ctypes.byref(s), L.LR_F32, None, f, None) == L.LR_EINVAL
    assert lib.lr_extract_bezier_backward(ctypes.byref(s), L.LR_F32, f, None, None) == L.LR_EINVAL
    s.p[:] = (2, 4, 2)
    assert lib.lr_extract_bezier_backward(ctypes.byref(s), L.LR_F64, f, f, None) == L.LR_EINVAL
    assert b"degree" in lib.lr_last_error()
    s.p[:] = (2, 2, 2)
    s.coef = 0                                   # the adjoint does not read coef
    s.gamma = 0
    assert lib.lr_extract_bezier_backward(ctypes.byref(s), L.LR_F64, f, f, None) == L.LR_EINVAL
    assert b"null array" in lib.lr_last_error()


# ---------------------------------------------------------------- octree
def descend_octree(oc, p):
    """The documented octree descent over the exported arrays (test side)."""
    pf = p.astype(np.float32)
    out = np.empty(p.shape[0], dtype=np.int64)
    for k in range(p.shape[0]):
        r, level = oc.root, 0
        while not r & L.LR_LEAF:
            scale = np.float32(2.0 ** (level + 1))
            c = np.minimum((pf[k] * scale).astype(np.int64), 2 ** (level + 1) - 1) & 1
            r = int(oc.nodes[r, c[0] | (c[1] << 1) | (c[2] << 2)])
            level += 1
        out[k] = r & ~L.LR_LEAF
    return out


def _leaf_depths(oc):
    if oc.root & L.LR_LEAF:
        return [0]
    out, stack = [], [(oc.root, 0)]
    while stack:
        r, d = stack.pop()
        for c in oc.nodes[r]:
            c = int(c)
            if c & L.LR_LEAF:
                out.append(d + 1)
            else:
                stack.append((c, d + 1))
    return out


@pytest.mark.parametrize("make", [
    lambda: lrgen.small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=80, seed=21, dist="cluster"),
    lambda: workload("scalar_ortho64").spline,
    lambda: lrgen.small_random(p=(3, 1, 2), n=(2, 4, 8), n_ref=60, seed=22),
])
def test_octree_descent_equals_scan(make):
    s = make()
    oc = P.Octree.build(s.elem_box)
    x = _probe_points(s.elem_box, 2000, 2)
    assert np.array_equal(descend_octree(oc, x), ElementIndex(s.elem_box).find(x))
    d = np.array(_leaf_depths(oc))
    st = oc.stats
    assert st["n_heads"] == 1 and st["n_nodes"] == oc.nodes.shape[0]
    assert st["min_depth"] == d.min() and st["max_depth"] == d.max()
    assert abs(st["mean_depth"] - d.mean()) < 1e-12 and abs(st["var_depth"] - d.var()) < 1e-12


def test_octree_shapes_and_errors():
    t = P.Octree.build(lrgen.tensor_spline((2, 2, 2), (4, 4, 4)).elem_box)
    assert t.stats["n_nodes"] == 9 and t.stats["min_depth"] == 2 and t.stats["max_depth"] == 2
    one = P.Octree.build(np.array([[0, 0, 0, 1, 1, 1.0]]))
    assert one.root == L.LR_LEAF and one.stats["n_nodes"] == 0 and one.stats["n_direct"] == 1
    # an element with sides 1/2 x 1/8 x 1/8 spans 16 leaves
    a = lrgen.tensor_spline((1, 1, 1), (2, 8, 8)).elem_box
    oa = P.Octree.build(a)
    assert len(_leaf_depths(oa)) == 8 ** 3 and oa.stats["max_depth"] == 3
    lib = L.lib()

    def status(box):
        eb = np.ascontiguousarray(box, dtype=np.float64)
        h = ctypes.c_void_p()
        st = lib.lr_build_octree(eb.ctypes.data, eb.shape[0], ctypes.byref(h), None)
        if st == 0:
            lib.lr_octree_free(h)
        return st
    assert status(np.array([[0, 0, 0, 0.1, 1, 1.0], [0.1, 0, 0, 1, 1, 1.0]])) == L.LR_EKNOT
    assert status(np.array([[0, 0, 0, 0.5, 1, 1.0]])) == L.LR_EPARTITION
    assert status(np.array([[0, 0, 0, 0.75, 1, 1.0], [0.25, 0, 0, 1, 1, 1.0]])) == L.LR_EPARTITION
    assert status(np.array([[0, 0, 0, 2.0, 1, 1.0]])) == L.LR_EPARTITION
    f = ctypes.c_void_p(0x1000)
    assert lib.lr_lookup_octree(f, f, 1, 0, f, 5, f, None) == L.LR_EINVAL
    assert lib.lr_lookup_octree(f, f, 1, 10, f, 0, f, None) == L.LR_OK


def test_streamlines_validate_first():
    lib = L.lib()
    f = ctypes.c_void_p(0x1000)
    s = _scene_struct(ncomp=3, color_mode=L.LR_COLOR_HUE)

    def prm(**kw):
        p = L.StreamParams()
        p.method, p.step_mode, p.precision = kw.get("method", 3), kw.get("step", 0), kw.get("prec", 0)
        p.max_samples, p.base, p.t_end, p.tol = kw.get("max_samples", 16), kw.get("base", 1.0), 1.0, kw.get("tol", 0.0)
        return p

    def st(scene, p, n=4, seeds=f, pts=f):
        return lib.lr_streamlines(ctypes.byref(scene), ctypes.byref(p), seeds, n, pts, None, None, None)
    assert st(s, prm(), n=0) == L.LR_OK                             # no seeds: nothing launched
    assert st(s, prm(), seeds=None) == L.LR_EINVAL
    assert st(s, prm(), pts=None) == L.LR_EINVAL
    assert st(s, prm(method=9)) == L.LR_EINVAL
    assert st(s, prm(step=2)) == L.LR_EINVAL                        # RK4 has no embedded pair
    assert st(s, prm(method=8, step=2)) == L.LR_EINVAL              # embedded needs tol > 0
    assert st(s, prm(prec=2)) == L.LR_EINVAL
    assert st(s, prm(max_samples=0)) == L.LR_EINVAL
    assert st(s, prm(base=0.0)) == L.LR_EINVAL
    assert st(_scene_struct(), prm()) == L.LR_EINVAL                # scalar field
    assert b"3-component" in lib.lr_last_error()
    s16 = _scene_struct(ncomp=3, color_mode=L.LR_COLOR_HUE, dtype=L.LR_F16)
    assert st(s16, prm()) == L.LR_EINVAL
    sb = _scene_struct(ncomp=3, color_mode=L.LR_COLOR_HUE, blocks=(3, 4, 4))
    assert st(sb, prm()) == L.LR_ENOTPOW2


def test_header_is_plain_c(tmp_path):
    """include/lrvr.h compiles as C99 and its struct sizes and offsets match the binding's."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "h.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lrvr.h"\n'
                   'int main(void) { printf("%d %d %d %d %d %d %d %d\\n", (int)sizeof(lr_scene), (int)sizeof(lr_view), '
                   '(int)sizeof(lr_lrspline), (int)sizeof(lr_kdnode), (int)sizeof(lr_forest_stats), '
                   '(int)sizeof(lr_stream_params), (int)offsetof(lr_scene, shading), (int)offsetof(lr_scene, lookup));'
                   ' return 0; }\n')
    exe = tmp_path / "h"
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                           str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(L.SceneC), ctypes.sizeof(L.ViewC), ctypes.sizeof(L.LRSplineDev), ctypes.sizeof(L.KdNode),
            ctypes.sizeof(L.ForestStats), ctypes.sizeof(L.StreamParams), L.SceneC.shading.offset, L.SceneC.lookup.offset]
    assert got == want


def test_render_workspace_size():
    """Host-only query of lr_render_scheduled's workspace, for the largest
    launch (16 views per launch): 4 bytes per 16x16-pixel block, then for s
    dealing slots (32 per 8 groups of 2x2 blocks of a view, rounded up) s / 4
    bytes of group XCDs and 4 s bytes of order, each part rounded up to 256
    bytes; bad views are errors."""
    from paper_1707_01170_amd.api import view_array
    n = ctypes.c_int64(0)

    def size(views):
        arr, _ = view_array(views)
        st = L.lib().lr_render_workspace_size(arr, len(views), ctypes.byref(n))
        return st, n.value

    def expect(views):
        r256 = lambda b: (b + 255) // 256 * 256
        per_launch = []
        for k in range(0, len(views), 16):
            q = slots = 0
            for v in views[k:k + 16]:
                qw, qh = (v.width + 15) // 16, (v.height + 15) // 16
                q += qw * qh
                slots += 32 * ((((qw + 1) // 2) * ((qh + 1) // 2) + 7) // 8)
            per_launch.append(r256(4 * q) + r256(slots // 4) + r256(4 * slots))
        return max(per_launch)

    v = lrgen.sphere_view(np.array([1.0, 0.2, 0.3]), 1920, 1080)
    assert size([v]) == (L.LR_OK, 32768 + 2048 + 32768) == (L.LR_OK, expect([v]))
    rng = np.random.default_rng(2)
    views = [lrgen.sphere_view(lrgen.random_directions(rng, 1)[0], int(w), int(h))
             for w, h in rng.integers(1, 700, size=(21, 2))]
    assert size(views) == (L.LR_OK, expect(views))
    bad = lrgen.sphere_view(np.array([1.0, 0.0, 0.0]), 64, 64)
    bad.width = 0
    assert size([bad])[0] == L.LR_EINVAL
    assert L.lib().lr_render_workspace_size(None, 1, ctypes.byref(n)) == L.LR_EINVAL


def test_render_persistent_argument_checks():
    """lr_render_persistent refuses queue counts other than 1 and 8, orders
    other than 0 and 1 and grids outside [0, 2^20] before it reads anything
    else (host only, no GPU work)."""
    f = L.lib().lr_render_persistent
    for queues, order, wg in ((0, 0, 0), (2, 0, 0), (16, 1, 0), (1, 2, 0), (8, -1, 0), (8, 1, -1), (1, 0, (1 << 20) + 1)):
        assert f(None, None, 1, None, None, queues, order, wg, None, 0, None) == L.LR_EINVAL, (queues, order, wg)
    assert b"lr_render_persistent" in L.lib().lr_last_error()

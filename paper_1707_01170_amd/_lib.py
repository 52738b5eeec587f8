"""ctypes binding of the C ABI declared in include/lrvr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

from . import _build

LR_OK, LR_EINVAL, LR_ENOTPOW2, LR_EKNOT, LR_ECAPACITY, LR_EHIP, LR_EPARTITION = 0, -1, -2, -3, -4, -5, -6
LR_F32, LR_F16, LR_F64 = 0, 1, 2
LR_STEP_FIXED, LR_STEP_ADAPTIVE = 0, 1
LR_COLOR_LUT, LR_COLOR_HUE = 0, 1
LR_PERSP, LR_ORTHO = 0, 1
LR_LOOKUP_FOREST, LR_LOOKUP_OCTREE = 0, 1
LR_SHADE_NONE, LR_SHADE_DIRECTIONAL, LR_SHADE_HEADLIGHT = 0, 1, 2
RK_METHODS = {"rk1": 0, "rk2": 1, "rk3": 2, "rk4": 3, "rk4_38": 4, "rkf5": 5, "he": 6, "bs": 7, "rkf45": 8}
LR_STREAM_HEURISTIC, LR_STREAM_CONSTANT, LR_STREAM_EMBEDDED = 0, 1, 2
LR_PREC_MIXED, LR_PREC_SINGLE = 0, 1
LR_LEAF = 0x80000000
LR_MAX_VIEWS_PER_LAUNCH = 16

_c_i32, _c_i64, _c_f32, _c_f64, _c_u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_uint32
_vp = ctypes.c_void_p


class KdNode(ctypes.Structure):
    _fields_ = [("lo", _c_u32), ("hi", _c_u32), ("split", _c_f32), ("axis", _c_u32)]


class ForestStats(ctypes.Structure):
    _fields_ = [("n_heads", _c_i64), ("n_nodes", _c_i64), ("n_direct", _c_i64), ("min_depth", _c_i32),
                ("max_depth", _c_i32), ("mean_depth", _c_f64), ("var_depth", _c_f64)]


class LRSplineDev(ctypes.Structure):
    _fields_ = [("p", _c_i32 * 3), ("ncomp", _c_i32), ("kstride", _c_i32), ("pad", _c_i32),
                ("n_bspl", _c_i64), ("n_elem", _c_i64), ("knots", _vp), ("coef", _vp), ("gamma", _vp),
                ("elem_box", _vp), ("csr_ptr", _vp), ("csr_idx", _vp)]


class SceneC(ctypes.Structure):
    _fields_ = [("p", _c_i32 * 3), ("ncomp", _c_i32), ("n_elem", _c_i64), ("elem_box", _vp), ("bezier", _vp),
                ("bezier_dtype", _c_i32), ("blocks", _c_i32 * 3), ("heads", _vp), ("nodes", _vp),
                ("n_nodes", _c_i64), ("lut", _vp), ("vmin", _c_f32), ("vmax", _c_f32), ("xi", _c_f32),
                ("alpha_clamp", _c_f32), ("term_alpha", _c_f32), ("step_mode", _c_i32),
                ("n_fixed_steps", _c_i32), ("color_mode", _c_i32), ("max_samples", _c_i32), ("lookup", _c_i32),
                ("shading", _c_i32), ("light", _c_f32 * 3)]


class ViewC(ctypes.Structure):
    _fields_ = [("proj", _c_i32), ("width", _c_i32), ("height", _c_i32), ("pad", _c_i32),
                ("out_offset", _c_i64), ("eye", _c_f32 * 3), ("fwd", _c_f32 * 3), ("right", _c_f32 * 3),
                ("up", _c_f32 * 3), ("tx", _c_f32), ("ty", _c_f32)]


class StreamParams(ctypes.Structure):
    _fields_ = [("method", _c_i32), ("step_mode", _c_i32), ("precision", _c_i32), ("max_samples", _c_i32),
                ("base", _c_f64), ("t_end", _c_f64), ("tol", _c_f64)]


assert ctypes.sizeof(StreamParams) == 40
assert ctypes.sizeof(KdNode) == 16 and ctypes.sizeof(ViewC) == 80 and ctypes.sizeof(SceneC) == 144
assert ctypes.sizeof(ForestStats) == 48 and ctypes.sizeof(LRSplineDev) == 88

# name: (restype, argtypes)
SIGNATURES = {
    "lr_last_error": (ctypes.c_char_p, []),
    "lr_version": (_c_i32, []),
    "lr_build_forest": (_c_i32, [_vp, _c_i64, _vp, ctypes.POINTER(_vp), ctypes.POINTER(ForestStats)]),
    "lr_forest_export": (_c_i32, [_vp, _vp, _vp]),
    "lr_forest_free": (None, [_vp]),
    "lr_build_forest_device": (_c_i32, [_vp, _c_i64, _vp, _vp, _vp, _c_i64, ctypes.POINTER(_c_i64),
                                        ctypes.POINTER(ForestStats), _vp]),
    "lr_build_id": (ctypes.c_char_p, []),
    "lr_lookup": (_c_i32, [_vp, _vp, _c_i64, _vp, _c_i64, _vp, _c_i64, _vp, _vp]),
    "lr_build_octree": (_c_i32, [_vp, _c_i64, ctypes.POINTER(_vp), ctypes.POINTER(ForestStats)]),
    "lr_octree_export": (_c_i32, [_vp, _vp, _vp]),
    "lr_octree_free": (None, [_vp]),
    "lr_lookup_octree": (_c_i32, [_vp, _vp, _c_i64, _c_i64, _vp, _c_i64, _vp, _vp]),
    "lr_bezier_stride": (_c_i64, [_vp, _c_i32, _c_i32]),
    "lr_build_support": (_c_i32, [_vp, _c_i64, _c_i32, _vp, _vp, _c_i64, _vp, _vp, _c_i64,
                                  ctypes.POINTER(_c_i64)]),
    "lr_extract_bezier": (_c_i32, [ctypes.POINTER(LRSplineDev), _c_i32, _vp, _vp, _vp]),
    "lr_extract_bezier_backward": (_c_i32, [ctypes.POINTER(LRSplineDev), _c_i32, _vp, _vp, _vp]),
    "lr_render": (_c_i32, [ctypes.POINTER(SceneC), ctypes.POINTER(ViewC), _c_i32, _vp, _vp, _vp]),
    "lr_render_scheduled": (_c_i32, [ctypes.POINTER(SceneC), ctypes.POINTER(ViewC), _c_i32, _vp, _vp, _vp, _c_i64,
                                     _vp]),
    "lr_render_workspace_size": (_c_i32, [ctypes.POINTER(ViewC), _c_i32, ctypes.POINTER(_c_i64)]),
    "lr_render_scheduled_noalloc": (_c_i32, [ctypes.POINTER(SceneC), ctypes.POINTER(ViewC), _c_i32, _vp, _vp, _vp]),
    "lr_render_persistent": (_c_i32, [ctypes.POINTER(SceneC), ctypes.POINTER(ViewC), _c_i32, _vp, _vp, _c_i32, _c_i32,
                                      _c_i32, _vp, _c_i64, _vp]),
    "lr_render_backward": (_c_i32, [ctypes.POINTER(SceneC), ctypes.POINTER(ViewC), _c_i32, _vp, _vp, _vp, _vp, _vp]),
    "lr_streamlines": (_c_i32, [ctypes.POINTER(SceneC), ctypes.POINTER(StreamParams), _vp, _c_i64, _vp, _vp, _vp,
                                _vp]),
    "lr_trace_rays": (_c_i32, [ctypes.POINTER(SceneC), ctypes.POINTER(ViewC), _vp, _c_i64, _c_i32, _vp, _vp, _vp,
                               _vp, _vp]),
}

_lib = None


class LRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d)" % (msg, status))
        self.status = status


def _built_id(path):
    """The build id a library file reports (read in a child process, so that
    a stale binary is never loaded into this one)."""
    import subprocess
    import sys
    code = ("import ctypes,sys; L=ctypes.CDLL(sys.argv[1]); f=L.lr_build_id; f.restype=ctypes.c_char_p; "
            "print(f().decode())")
    r = subprocess.run([sys.executable, "-c", code, path], capture_output=True, text=True)
    return r.stdout.strip() if r.returncode == 0 else None


def lib():
    """The loaded HIP library.  Builds it in-tree if it was never built or was
    built from other sources than the ones in the tree (its lr_build_id differs
    from their digest); raises if that fails (there is no fallback
    implementation)."""
    global _lib
    if _lib is None:
        want = _build.source_digest()
        if not os.path.exists(_build.LIB) or _built_id(_build.LIB) != want:
            import sys
            print("[lrvr] building %s (sources changed since it was built)" % _build.LIB, file=sys.stderr, flush=True)
            _build.build()
        import torch  # noqa: F401  (loads the HIP runtime the library links against)
        L = ctypes.CDLL(_build.LIB)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        got = L.lr_build_id().decode()
        if got != want:
            raise RuntimeError("%s reports build %s, its sources are %s" % (_build.LIB, got, want))
        _lib = L
    return _lib


def check(status):
    if status != LR_OK:
        raise LRError(status, lib().lr_last_error().decode())
    return status

"""Seeded synthetic inputs for LR-spline volume rendering.

This module makes the inputs both the FP64 oracle and the GPU library consume:
LR-spline volumes (Eq. 2, Sec. 3.1), camera views, transfer-function tables and
request streams.  It holds none of the rendering method's arithmetic (no spline
evaluation, no change of basis, no element look-up, no compositing); the only
spline arithmetic here is the knot insertion that local refinement needs to
create an LR-spline, implemented in ``lrgen.cpp``.

The paper's data sets are not available; the five workloads below stand in for
them with the shapes the paper describes: tri-degree (2,2,2) or (3,3,3)
volumes, scalar or 3-vector fields, many levels of local refinement, dyadic
knots (exact in FP32), 1280x720..1920x1080 views.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_lrgen.so")
_SRC = os.path.join(_HERE, "lrgen.cpp")

SEED_BASE = 20170705
ALPHA_CLAMP = 1.0 - 2.0 ** -16       # opacity clamp and early-termination threshold
POINT_BATCH = 65536                   # seed points drawn per batch (fixes RNG consumption)


def build(force: bool = True) -> str:
    """Compile the refinement generator with g++ (host code only)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                               "-fvisibility=hidden", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        i32p = ctypes.POINTER(ctypes.c_int32)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.lrgen_create.argtypes = [i32p, i32p, ctypes.c_int32, ctypes.c_int32]
        lib.lrgen_create.restype = ctypes.c_void_p
        lib.lrgen_destroy.argtypes = [ctypes.c_void_p]
        lib.lrgen_set_coef.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64]
        lib.lrgen_set_coef.restype = ctypes.c_int32
        lib.lrgen_refine.argtypes = [ctypes.c_void_p, dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        lib.lrgen_refine.restype = ctypes.c_int64
        lib.lrgen_refine_plane.argtypes = [ctypes.c_void_p, dp, ctypes.c_int32, ctypes.c_double]
        lib.lrgen_refine_plane.restype = ctypes.c_int32
        lib.lrgen_counts.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]
        lib.lrgen_export.argtypes = [ctypes.c_void_p, dp, dp, dp, dp]
        lib.lrgen_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class LRSpline:
    """A trivariate LR-spline on [0,1]^3 (Eq. 2).

    p         tri-degree (p1, p2, p3)
    knots     [n_bspl, 3, max(p)+2] local knot vectors (axis d uses p[d]+2 entries)
    gamma     [n_bspl] partition-of-unity weights
    coef      [n_bspl, ncomp] coefficients
    elem_box  [n_elem, 6] element boxes (lo x,y,z, hi x,y,z); a box partition
    """
    p: tuple
    knots: np.ndarray
    gamma: np.ndarray
    coef: np.ndarray
    elem_box: np.ndarray

    @property
    def ncomp(self) -> int:
        return int(self.coef.shape[1])

    @property
    def n_bspl(self) -> int:
        return int(self.knots.shape[0])

    @property
    def n_elem(self) -> int:
        return int(self.elem_box.shape[0])

    def with_coef(self, coef: np.ndarray) -> "LRSpline":
        coef = np.ascontiguousarray(coef, dtype=np.float64).reshape(self.n_bspl, -1)
        return LRSpline(self.p, self.knots, self.gamma, coef, self.elem_box)

    def greville(self) -> np.ndarray:
        """Greville point of each B-spline: mean of its p interior knots per axis."""
        g = np.empty((self.n_bspl, 3))
        for d in range(3):
            pd = self.p[d]
            g[:, d] = self.knots[:, d, 1:pd + 1].mean(axis=1)
        return g


class Refiner:
    """Incremental LR refinement of an open tensor mesh (host C++)."""

    def __init__(self, p, n, ncomp=1, grid=None):
        lib = _load()
        if grid is None:
            grid = int(min(128, max(16, 1 << int(np.ceil(np.log2(2 * max(n)))))))
        pa = (ctypes.c_int32 * 3)(*p)
        na = (ctypes.c_int32 * 3)(*n)
        self._h = lib.lrgen_create(pa, na, int(ncomp), int(grid))
        if not self._h:
            raise ValueError(lib.lrgen_last_error().decode())
        self.p = tuple(int(x) for x in p)
        self.n = tuple(int(x) for x in n)
        self.ncomp = int(ncomp)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().lrgen_destroy(h)
            self._h = None

    def counts(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _load().lrgen_counts(self._h, ctypes.byref(a), ctypes.byref(b))
        return int(a.value), int(b.value)

    def set_initial_coef(self, c):
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(-1, self.ncomp)
        if _load().lrgen_set_coef(self._h, _dp(c), c.shape[0]) != 0:
            raise ValueError(_load().lrgen_last_error().decode())

    def refine(self, pts, target_elems=1 << 62, max_ref=1 << 62) -> int:
        pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        used = _load().lrgen_refine(self._h, _dp(pts), pts.shape[0], int(target_elems), int(max_ref))
        if used < 0:
            raise RuntimeError(_load().lrgen_last_error().decode())
        return int(used)

    def refine_plane(self, q, axis, value):
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(3)
        if _load().lrgen_refine_plane(self._h, _dp(q), int(axis), float(value)) != 0:
            raise RuntimeError(_load().lrgen_last_error().decode())

    def export(self) -> LRSpline:
        ne, nb = self.counts()
        ks = max(self.p) + 2
        eb = np.empty((ne, 6))
        kn = np.empty((nb, 3, ks))
        ga = np.empty(nb)
        co = np.empty((nb, self.ncomp))
        _load().lrgen_export(self._h, _dp(eb), _dp(kn), _dp(ga), _dp(co))
        return LRSpline(self.p, kn, ga, co, eb)


# --------------------------------------------------------------------------
# Transfer function and views
# --------------------------------------------------------------------------

def default_lut() -> np.ndarray:
    """256-entry RGBA table: opacity a linear ramp i/255, colour
    (u, 1-|2u-1|, 1-u) with u = i/255.  Returned as float32 [256, 4]."""
    u = np.arange(256, dtype=np.float64) / 255.0
    lut = np.stack([u, 1.0 - np.abs(2.0 * u - 1.0), 1.0 - u, u], axis=1)
    return lut.astype(np.float32)


@dataclass
class View:
    """One camera.  All vectors are float32 values (rounded once from FP64).

    proj   'persp' (rays from eye through pixel centres) or 'ortho' (rays along
           fwd from eye + sx*right + sy*up)
    tx, ty horizontal / vertical half-extent factors: tan(fov/2)*W/H and
           tan(fov/2) for perspective, half-width and half-height for ortho
    Pixel (i, j): column i, row j with row 0 at the top.
    """
    proj: str
    width: int
    height: int
    eye: np.ndarray
    fwd: np.ndarray
    right: np.ndarray
    up: np.ndarray
    tx: np.float32
    ty: np.float32


def ortho_z_view(res: int) -> View:
    """Orthographic view along +z covering [0,1]^2 at res x res pixels."""
    f = np.float32
    return View("ortho", res, res, np.array([0.5, 0.5, 0.0], f), np.array([0, 0, 1], f),
                np.array([1, 0, 0], f), np.array([0, 1, 0], f), f(0.5), f(0.5))


def sphere_view(u: np.ndarray, width: int, height: int, fov_deg: float = 45.0,
                radius: float = 2.0) -> View:
    """Perspective camera at c + radius*u looking at the volume centre c."""
    c = np.array([0.5, 0.5, 0.5])
    u = np.asarray(u, dtype=np.float64)
    u = u / np.linalg.norm(u)
    eye = c + radius * u
    fwd = (c - eye) / np.linalg.norm(c - eye)
    upv = np.array([0.0, 0.0, 1.0]) if abs(fwd[2]) <= 0.999 else np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, upv)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    t = np.tan(np.deg2rad(fov_deg) / 2.0)
    f = np.float32
    return View("persp", int(width), int(height), eye.astype(f), fwd.astype(f), right.astype(f),
                up.astype(f), f(t * width / height), f(t))


def random_directions(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    """A volume plus its rendering parameters."""
    name: str
    spline: LRSpline
    lut: np.ndarray
    vmin: float
    vmax: float
    step_mode: str            # 'fixed' or 'adaptive'
    n_fixed_steps: int
    color_mode: str           # 'lut' or 'hue'
    views: List[View]
    xi: float = 1.0
    alpha_clamp: float = ALPHA_CLAMP
    term_alpha: float = ALPHA_CLAMP
    extra: dict = field(default_factory=dict)


def _streams(offset: int):
    ss = np.random.SeedSequence(SEED_BASE + offset)
    mesh, coef, noise, camera, requests = ss.spawn(5)
    return mesh, coef, noise, camera, requests


def _refine_until(r: Refiner, draw, target=None, exact=None):
    """Feeds seed points from draw(batch) until the element target (or the
    exact refinement count) is reached."""
    done = 0
    while True:
        pts = draw(POINT_BATCH)
        if exact is not None:
            used = r.refine(pts, max_ref=exact - done)
            done += used
            if done >= exact:
                return
        else:
            r.refine(pts, target_elems=target)
            if r.counts()[0] >= target:
                return


def _value_range_scalar(c):
    return float(np.min(c)), float(np.max(c))


def _value_range_vector(c):
    return 0.0, float(np.max(np.linalg.norm(c, axis=1)))


def scalar_ortho64(n_views: int = 1) -> Workload:
    """(2,2,2) scalar; 4^3 mesh plus exactly 20 refinements at U[0,1]^3 points;
    c ~ U[0,1]; 64x64 orthographic view along z; fixed 256 steps per ray."""
    mesh, coef, noise, camera, _ = _streams(1)
    rm = np.random.default_rng(mesh)
    r = Refiner((2, 2, 2), (4, 4, 4))
    _refine_until(r, lambda n: rm.random((n, 3)), exact=20)
    s = r.export()
    s = s.with_coef(np.random.default_rng(coef).random((s.n_bspl, 1)))
    return Workload("scalar_ortho64", s, default_lut(), 0.0, 1.0, "fixed", 256, "lut", [ortho_z_view(64)])


def blobs50k(width: int = 1024, height: int = 1024, n_views: int = 1, target: int = 50000) -> Workload:
    """(3,3,3) scalar; 16^3 mesh refined toward 8 Gaussian blobs (centres
    U[0.2,0.8]^3, sigma 0.05) until n_elem >= 50k; c = blob sum at the Greville
    point + N(0, 0.01^2); 1024^2 perspective view, FOV 45, radius 2; adaptive step."""
    mesh, coef, noise, camera, _ = _streams(2)
    rm = np.random.default_rng(mesh)
    mu = rm.uniform(0.2, 0.8, size=(8, 3))

    def draw(n):
        b = rm.integers(0, 8, size=n)
        q = mu[b] + rm.normal(0.0, 0.05, size=(n, 3))
        return q[np.all((q >= 0.0) & (q <= 1.0), axis=1)]

    r = Refiner((3, 3, 3), (16, 16, 16))
    _refine_until(r, draw, target=target)
    s = r.export()
    g = s.greville()
    c = np.exp(-((g[:, None, :] - mu[None, :, :]) ** 2).sum(-1) / (2 * 0.05 ** 2)).sum(1)
    c = c + np.random.default_rng(noise).normal(0.0, 0.01, size=c.shape)
    s = s.with_coef(c[:, None])
    vmin, vmax = _value_range_scalar(s.coef)
    rc = np.random.default_rng(camera)
    views = [sphere_view(u, width, height) for u in random_directions(rc, n_views)]
    return Workload("blobs50k", s, default_lut(), vmin, vmax, "adaptive", 0, "lut", views,
                    extra={"blob_centres": mu})


def vortex(x: np.ndarray) -> np.ndarray:
    """v = (-(y-1/2), x-1/2, 0.2) * exp(-r^2/0.04), r^2 = (x-1/2)^2 + (y-1/2)^2."""
    dx, dy = x[:, 0] - 0.5, x[:, 1] - 0.5
    w = np.exp(-(dx * dx + dy * dy) / 0.04)
    return np.stack([-dy * w, dx * w, 0.2 * w], axis=1)


def vortex200k(width: int = 1920, height: int = 1080, n_views: int = 1, target: int = 200000) -> Workload:
    """(2,2,2) 3-vector; 32^3 mesh refined along the vortex tube x=y=1/2 (seed
    points (1/2+dx, 1/2+dy, z), d ~ N(0, 0.1^2 I), z ~ U[0,1]) until n_elem >=
    200k; c = vortex(Greville) + N(0, 0.01^2 I); |v| through the LUT opacity,
    hue from the direction; 1920x1080 perspective; adaptive step."""
    mesh, coef, noise, camera, _ = _streams(3)
    rm = np.random.default_rng(mesh)

    def draw(n):
        d = rm.normal(0.0, 0.1, size=(n, 2))
        z = rm.random(n)
        q = np.stack([0.5 + d[:, 0], 0.5 + d[:, 1], z], axis=1)
        return q[np.all((q >= 0.0) & (q <= 1.0), axis=1)]

    r = Refiner((2, 2, 2), (32, 32, 32), ncomp=3)
    _refine_until(r, draw, target=target)
    s = r.export()
    c = vortex(s.greville()) + np.random.default_rng(noise).normal(0.0, 0.01, size=(s.n_bspl, 3))
    s = s.with_coef(c)
    vmin, vmax = _value_range_vector(s.coef)
    rc = np.random.default_rng(camera)
    views = [sphere_view(u, width, height) for u in random_directions(rc, n_views)]
    return Workload("vortex200k", s, default_lut(), vmin, vmax, "adaptive", 0, "hue", views)


SERVING_RESOLUTIONS = (256, 512, 1024, 2048)


@dataclass
class Request:
    arrival_s: float
    view: View


def blob_requests(n: int = 1000, rate_hz: float = 200.0) -> List[Request]:
    """Poisson request stream on the blobs50k volume: inter-arrival times
    Exp(mean 1/rate), square resolutions drawn uniformly from 256..2048."""
    _, _, _, camera, requests = _streams(4)
    rq = np.random.default_rng(requests)
    gaps = rq.exponential(1.0 / rate_hz, size=n)
    res = rq.integers(0, len(SERVING_RESOLUTIONS), size=n)
    dirs = random_directions(np.random.default_rng(camera), n)
    t = np.cumsum(gaps)
    return [Request(float(t[k]), sphere_view(dirs[k], SERVING_RESOLUTIONS[res[k]], SERVING_RESOLUTIONS[res[k]]))
            for k in range(n)]


def scalar20k(width: int = 512, height: int = 512, n_views: int = 4, target: int = 20000) -> Workload:
    """(2,2,2) scalar; 16^3 mesh with U[0,1]^3 refinements until n_elem >= 20k;
    coefficient set A ~ U[0,1] (rendered, differentiated) and set B ~ U[0,1]
    (targets, in extra['coef_target']); 4 perspective views 512^2; adaptive."""
    mesh, coef, noise, camera, _ = _streams(5)
    rm = np.random.default_rng(mesh)
    r = Refiner((2, 2, 2), (16, 16, 16))
    _refine_until(r, lambda n: rm.random((n, 3)), target=target)
    s = r.export()
    ca, cb = coef.spawn(2)
    a = np.random.default_rng(ca).random((s.n_bspl, 1))
    b = np.random.default_rng(cb).random((s.n_bspl, 1))
    rc = np.random.default_rng(camera)
    views = [sphere_view(u, width, height) for u in random_directions(rc, n_views)]
    return Workload("scalar20k", s.with_coef(a), default_lut(), 0.0, 1.0, "adaptive", 0, "lut", views,
                    extra={"coef_target": b})


def tensor_spline(p, n, coef: Optional[np.ndarray] = None, ncomp: int = 1) -> LRSpline:
    """Unrefined open tensor-product spline (Eq. 1) as an LR-spline."""
    r = Refiner(p, n, ncomp=ncomp)
    if coef is not None:
        r.set_initial_coef(coef)
    return r.export()


def small_random(p=(2, 2, 2), n=(4, 4, 4), n_ref=40, seed=0, ncomp=1, dist="uniform") -> LRSpline:
    """Small seeded LR-spline for tests: n_ref refinements at random points."""
    rng = np.random.default_rng(seed)
    r = Refiner(p, n, ncomp=ncomp)
    if dist == "uniform":
        pts = rng.random((n_ref, 3))
    else:  # clustered near one corner to get several refinement levels
        pts = np.clip(0.3 + 0.08 * rng.normal(size=(n_ref, 3)), 0.0, 1.0)
    r.refine(pts)
    s = r.export()
    return s.with_coef(rng.random((s.n_bspl, ncomp)))


WORKLOADS = {"scalar_ortho64": scalar_ortho64, "blobs50k": blobs50k, "vortex200k": vortex200k, "scalar20k": scalar20k}


# --------------------------------------------------------------------------
# On-disk cache of generated workloads (generation is deterministic; the
# cache only saves time).  Keyed by the generator's sources and arguments.
# --------------------------------------------------------------------------
_CACHE_DIR = os.path.join(os.path.dirname(_HERE), ".lrcache")
_MEM = {}


def _source_key(name, kw):
    import hashlib
    import json
    h = hashlib.sha1()
    for f in (_SRC, os.path.abspath(__file__)):
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(json.dumps([name, sorted(kw.items())]).encode())
    return h.hexdigest()[:20]


def _save(path, wl: Workload):
    import json
    s = wl.spline
    views = [dict(proj=v.proj, width=v.width, height=v.height, eye=v.eye.tolist(), fwd=v.fwd.tolist(),
                  right=v.right.tolist(), up=v.up.tolist(), tx=float(v.tx), ty=float(v.ty)) for v in wl.views]
    meta = dict(name=wl.name, p=list(s.p), vmin=wl.vmin, vmax=wl.vmax, step_mode=wl.step_mode,
                n_fixed_steps=wl.n_fixed_steps, color_mode=wl.color_mode, views=views, xi=wl.xi,
                alpha_clamp=wl.alpha_clamp, term_alpha=wl.term_alpha, extra=sorted(wl.extra))
    arrays = dict(knots=s.knots, gamma=s.gamma, coef=s.coef, elem_box=s.elem_box, lut=wl.lut,
                  meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))
    for k, v in wl.extra.items():
        arrays["extra_" + k] = np.asarray(v)
    tmp = path + ".tmp%d.npz" % os.getpid()
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def _load_file(path) -> Workload:
    import json
    z = np.load(path)
    meta = json.loads(bytes(z["meta"]).decode())
    s = LRSpline(tuple(meta["p"]), z["knots"], z["gamma"], z["coef"], z["elem_box"])
    f = np.float32
    views = [View(v["proj"], v["width"], v["height"], np.array(v["eye"], f), np.array(v["fwd"], f),
                  np.array(v["right"], f), np.array(v["up"], f), f(v["tx"]), f(v["ty"])) for v in meta["views"]]
    extra = {k: z["extra_" + k] for k in meta["extra"]}
    return Workload(meta["name"], s, z["lut"], meta["vmin"], meta["vmax"], meta["step_mode"], meta["n_fixed_steps"],
                    meta["color_mode"], views, meta["xi"], meta["alpha_clamp"], meta["term_alpha"], extra)


def cached(name: str, **kw) -> Workload:
    """getattr(lrgen, name)(**kw), memoised in memory and under .lrcache/."""
    key = _source_key(name, kw)
    if key in _MEM:
        return _MEM[key]
    path = os.path.join(_CACHE_DIR, "%s-%s.npz" % (name, key))
    wl = None
    if os.path.exists(path):
        try:
            wl = _load_file(path)
        except Exception:
            wl = None
    if wl is None:
        wl = globals()[name](**kw)
        try:
            os.makedirs(_CACHE_DIR, exist_ok=True)
            _save(path, wl)
        except OSError:
            pass
    _MEM[key] = wl
    return wl

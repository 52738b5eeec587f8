"""Python API over the C ABI: device-resident volumes, rendering, adjoint.

PyTorch provides device memory and streams; every computation runs in the
library's HIP kernels (or, for the look-up structure and the element/B-spline
incidence, in its host C++ builders, as the paper precomputes them on the CPU).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


# ---------------------------------------------------------------- host builders
@dataclass
class Forest:
    """k-d forest built on the host (Sec. 3.2.1)."""
    blocks: tuple
    heads: np.ndarray          # uint32 [bz*by*bx]
    nodes: np.ndarray          # uint32 [n_nodes, 4]: lo, hi, split bits, axis
    stats: dict

    @staticmethod
    def build(elem_box: np.ndarray, blocks) -> "Forest":
        lib = L.lib()
        eb = np.ascontiguousarray(elem_box, dtype=np.float64)
        if isinstance(blocks, int):
            blocks = (blocks, blocks, blocks)
        b = np.asarray(blocks, dtype=np.int32)
        h = ctypes.c_void_p()
        st = L.ForestStats()
        L.check(lib.lr_build_forest(_np_ptr(eb), eb.shape[0], _np_ptr(b), ctypes.byref(h), ctypes.byref(st)))
        try:
            heads = np.empty(st.n_heads, dtype=np.uint32)
            nodes = np.empty((max(st.n_nodes, 0), 4), dtype=np.uint32)
            L.check(lib.lr_forest_export(h, _np_ptr(heads), _np_ptr(nodes) if st.n_nodes else None))
        finally:
            lib.lr_forest_free(h)
        stats = {k: getattr(st, k) for k, _ in L.ForestStats._fields_}
        return Forest(tuple(int(x) for x in b), heads, nodes, stats)


def build_forest_device(elem_box: np.ndarray, blocks, device=None):
    """The k-d forest built on the host and written into device tensors by
    lr_build_forest_device (size query, then build and copy on the current
    stream).  Returns (heads int32 [n_heads], nodes int32 [n_nodes, 4], stats)."""
    lib = L.lib()
    dev = torch.device(device if device is not None else "cuda")
    eb = np.ascontiguousarray(elem_box, dtype=np.float32)
    b = np.asarray((blocks,) * 3 if isinstance(blocks, int) else blocks, dtype=np.int32)
    n_nodes = ctypes.c_int64()
    st = L.ForestStats()
    L.check(lib.lr_build_forest_device(_np_ptr(eb), eb.shape[0], _np_ptr(b), None, None, 0, ctypes.byref(n_nodes),
                                       ctypes.byref(st), None))
    heads = torch.empty(st.n_heads, dtype=torch.int32, device=dev)
    nodes = torch.empty((max(n_nodes.value, 1), 4), dtype=torch.int32, device=dev)
    L.check(lib.lr_build_forest_device(_np_ptr(eb), eb.shape[0], _np_ptr(b), _ptr(heads), _ptr(nodes),
                                       nodes.shape[0], ctypes.byref(n_nodes), ctypes.byref(st), _stream(dev)))
    return heads, nodes[:n_nodes.value], {k: getattr(st, k) for k, _ in L.ForestStats._fields_}


@dataclass
class Octree:
    """Element octree of a dyadic mesh, built on the host (Sec. 3.2)."""
    root: int
    nodes: np.ndarray          # uint32 [n_nodes, 8]
    stats: dict

    @staticmethod
    def build(elem_box: np.ndarray) -> "Octree":
        lib = L.lib()
        eb = np.ascontiguousarray(elem_box, dtype=np.float64)
        h = ctypes.c_void_p()
        st = L.ForestStats()
        L.check(lib.lr_build_octree(_np_ptr(eb), eb.shape[0], ctypes.byref(h), ctypes.byref(st)))
        try:
            root = np.zeros(1, dtype=np.uint32)
            nodes = np.empty((max(st.n_nodes, 0), 8), dtype=np.uint32)
            L.check(lib.lr_octree_export(h, _np_ptr(root), _np_ptr(nodes) if st.n_nodes else None))
        finally:
            lib.lr_octree_free(h)
        stats = {k: getattr(st, k) for k, _ in L.ForestStats._fields_}
        return Octree(int(root[0]), nodes, stats)


def support_csr(spline):
    """Element -> B-spline incidence (CSR, host C++)."""
    lib = L.lib()
    kn = np.ascontiguousarray(spline.knots, dtype=np.float64)
    eb = np.ascontiguousarray(spline.elem_box, dtype=np.float64)
    p = np.asarray(spline.p, dtype=np.int32)
    ne = eb.shape[0]
    ptr = np.empty(ne + 1, dtype=np.int64)
    nnz = ctypes.c_int64()
    L.check(lib.lr_build_support(_np_ptr(kn), kn.shape[0], kn.shape[2], _np_ptr(p), _np_ptr(eb), ne,
                                 _np_ptr(ptr), None, 0, ctypes.byref(nnz)))
    idx = np.empty(nnz.value, dtype=np.int32)
    L.check(lib.lr_build_support(_np_ptr(kn), kn.shape[0], kn.shape[2], _np_ptr(p), _np_ptr(eb), ne,
                                 _np_ptr(ptr), _np_ptr(idx), idx.shape[0], ctypes.byref(nnz)))
    return ptr, idx


def bezier_stride(p, ncomp, dtype) -> int:
    pa = np.asarray(p, dtype=np.int32)
    return int(L.lib().lr_bezier_stride(_np_ptr(pa), int(ncomp), int(dtype)))


_DT = {"f32": (L.LR_F32, torch.float32), "f16": (L.LR_F16, torch.float16), "f64": (L.LR_F64, torch.float64)}


class Volume:
    """An LR-spline volume resident on one GPU: element boxes, look-up
    structure (k-d forest, or an octree for dyadic meshes) and Bezier blocks.
    `spline` needs p, knots [n_bspl,3,k], gamma, coef [n_bspl,ncomp] and
    elem_box [n_elem,6] (numpy, FP64)."""

    def __init__(self, spline, blocks=64, dtype="f32", device=None, lookup="forest"):
        self.device = torch.device(device if device is not None else "cuda")
        self.p = tuple(int(v) for v in spline.p)
        self.ncomp = int(spline.coef.shape[1])
        self.n_elem = int(spline.elem_box.shape[0])
        self.spline = spline
        self.lookup = lookup
        dev = self.device
        if lookup == "octree":
            self.forest = None
            self.octree = Octree.build(spline.elem_box)
            self.look_stats = self.octree.stats
            self.heads = torch.from_numpy(np.array([self.octree.root], np.uint32).view(np.int32)).to(dev)
            nodes = self.octree.nodes if self.octree.nodes.shape[0] else np.zeros((1, 8), np.uint32)
            self.n_nodes = int(self.octree.nodes.shape[0])
        elif lookup == "forest":
            self.octree = None
            self.forest = Forest.build(spline.elem_box, blocks)
            self.look_stats = self.forest.stats
            self.heads = torch.from_numpy(self.forest.heads.view(np.int32)).to(dev)
            nodes = self.forest.nodes if self.forest.nodes.shape[0] else np.zeros((1, 4), np.uint32)
            self.n_nodes = int(self.forest.nodes.shape[0])
        else:
            raise ValueError("lookup must be 'forest' or 'octree'")
        self.elem_box = torch.from_numpy(np.ascontiguousarray(spline.elem_box, dtype=np.float32)).to(dev)
        self.nodes = torch.from_numpy(np.ascontiguousarray(nodes).view(np.int32)).to(dev)
        ptr, idx = support_csr(spline)
        self.csr_ptr = torch.from_numpy(ptr).to(dev)
        self.csr_idx = torch.from_numpy(idx).to(dev)
        self.knots = torch.from_numpy(np.ascontiguousarray(spline.knots, dtype=np.float64)).to(dev)
        self.gamma = torch.from_numpy(np.ascontiguousarray(spline.gamma, dtype=np.float64)).to(dev)
        self.elem_box64 = torch.from_numpy(np.ascontiguousarray(spline.elem_box, dtype=np.float64)).to(dev)
        self.bezier, self.bez_range = self.extract(spline.coef, dtype)
        self.bezier_dtype = dtype

    def _spline(self, coef_t, ncomp) -> L.LRSplineDev:
        s = L.LRSplineDev()
        s.p[:] = self.p
        s.ncomp = ncomp
        s.kstride = self.knots.shape[2]
        s.n_bspl = self.knots.shape[0]
        s.n_elem = self.n_elem
        s.knots, s.gamma = self.knots.data_ptr(), self.gamma.data_ptr()
        s.coef = 0 if coef_t is None else coef_t.data_ptr()
        s.elem_box, s.csr_ptr, s.csr_idx = self.elem_box64.data_ptr(), self.csr_ptr.data_ptr(), self.csr_idx.data_ptr()
        return s

    def extract(self, coef, dtype="f32"):
        """Bezier blocks of this mesh for a coefficient set [n_bspl, ncomp]
        (numpy or a device tensor; FP64 change of basis on the GPU).
        Returns (blocks, range[2])."""
        code, tdt = _DT[dtype]
        if isinstance(coef, torch.Tensor):
            coef_t = coef.detach().to(self.device, torch.float64).reshape(self.knots.shape[0], -1).contiguous()
        else:
            coef_t = torch.from_numpy(np.ascontiguousarray(coef, dtype=np.float64).reshape(self.knots.shape[0], -1)).to(self.device)
        ncomp = coef_t.shape[1]
        stride = bezier_stride(self.p, ncomp, code)
        out = torch.empty((self.n_elem, stride), dtype=tdt, device=self.device)
        rng = torch.empty(2, dtype=torch.float64, device=self.device)
        s = self._spline(coef_t, ncomp)
        L.check(L.lib().lr_extract_bezier(ctypes.byref(s), code, _ptr(out), _ptr(rng), _stream(self.device)))
        return out, rng

    def extract_backward(self, grad_bezier: torch.Tensor) -> torch.Tensor:
        """dL/dc [n_bspl, ncomp] (FP64) from dL/d(blocks) in the block layout
        (float32 or float64; adjoint of the change of basis on the GPU)."""
        code = {torch.float32: L.LR_F32, torch.float64: L.LR_F64}[grad_bezier.dtype]
        g = grad_bezier.contiguous()
        ncomp = self.ncomp
        assert g.shape == (self.n_elem, bezier_stride(self.p, ncomp, code)), g.shape
        out = torch.zeros((self.knots.shape[0], ncomp), dtype=torch.float64, device=self.device)
        s = self._spline(None, ncomp)
        L.check(L.lib().lr_extract_bezier_backward(ctypes.byref(s), code, _ptr(g), _ptr(out), _stream(self.device)))
        return out


class ExtractFunction(torch.autograd.Function):
    """Differentiable change of basis: LR coefficients (FP64 [n_bspl, ncomp])
    -> float32 Bezier blocks of `volume`'s mesh."""

    @staticmethod
    def forward(ctx, coef, volume):
        out, _ = volume.extract(coef, "f32")
        ctx.volume = volume
        return out

    @staticmethod
    def backward(ctx, grad):
        return ctx.volume.extract_backward(grad.float()).to(grad.device), None


@dataclass
class RenderParams:
    lut: np.ndarray
    vmin: float
    vmax: float
    step_mode: str = "adaptive"
    n_fixed_steps: int = 256
    color_mode: str = "lut"
    xi: float = 1.0
    alpha_clamp: float = 1.0 - 2.0 ** -16
    term_alpha: float = 1.0 - 2.0 ** -16
    max_samples: int = 1 << 16
    shading: str = "none"             # 'none', 'directional' or 'headlight' (Sec. 4.1 illumination)
    light: tuple = (0.0, 0.0, 1.0)    # towards the light, for 'directional'

    @staticmethod
    def of(wl) -> "RenderParams":
        return RenderParams(np.asarray(wl.lut, dtype=np.float32), float(wl.vmin), float(wl.vmax), wl.step_mode,
                            int(wl.n_fixed_steps), wl.color_mode, float(wl.xi), float(wl.alpha_clamp),
                            float(wl.term_alpha))


def view_struct(v, out_offset: int) -> L.ViewC:
    c = L.ViewC()
    c.proj = L.LR_PERSP if v.proj == "persp" else L.LR_ORTHO
    c.width, c.height = int(v.width), int(v.height)
    c.out_offset = int(out_offset)
    c.eye[:] = [float(x) for x in np.asarray(v.eye, np.float32)]
    c.fwd[:] = [float(x) for x in np.asarray(v.fwd, np.float32)]
    c.right[:] = [float(x) for x in np.asarray(v.right, np.float32)]
    c.up[:] = [float(x) for x in np.asarray(v.up, np.float32)]
    c.tx, c.ty = float(np.float32(v.tx)), float(np.float32(v.ty))
    return c


def view_array(views: Sequence, offsets: Optional[Sequence[int]] = None):
    if offsets is None:
        offsets = np.concatenate([[0], np.cumsum([v.width * v.height for v in views])[:-1]]).astype(np.int64)
    arr = (L.ViewC * len(views))(*[view_struct(v, int(o)) for v, o in zip(views, offsets)])
    return arr, [int(o) for o in offsets]


class Scene:
    """What lr_render needs: a volume, render parameters, and (optionally) a
    replacement Bezier block tensor / LUT tensor (e.g. when differentiating)."""

    def __init__(self, volume: Volume, params: RenderParams):
        self.volume = volume
        self.params = params
        self.lut = torch.from_numpy(np.ascontiguousarray(params.lut, dtype=np.float32)).to(volume.device)

    def struct(self, bezier=None, lut=None) -> L.SceneC:
        v, pr = self.volume, self.params
        bez = v.bezier if bezier is None else bezier
        lut = self.lut if lut is None else lut
        assert bez.is_contiguous() and lut.is_contiguous() and lut.shape == (256, 4)
        s = L.SceneC()
        s.p[:] = v.p
        s.ncomp = v.ncomp
        s.n_elem = v.n_elem
        s.elem_box = v.elem_box.data_ptr()
        s.bezier = bez.data_ptr()
        s.bezier_dtype = {torch.float32: L.LR_F32, torch.float16: L.LR_F16}[bez.dtype]
        s.blocks[:] = v.forest.blocks if v.forest is not None else (1, 1, 1)
        s.lookup = L.LR_LOOKUP_OCTREE if v.lookup == "octree" else L.LR_LOOKUP_FOREST
        s.heads = v.heads.data_ptr()
        s.nodes = v.nodes.data_ptr()
        s.n_nodes = v.n_nodes
        s.lut = lut.data_ptr()
        s.vmin, s.vmax, s.xi = pr.vmin, pr.vmax, pr.xi
        s.alpha_clamp, s.term_alpha = pr.alpha_clamp, pr.term_alpha
        s.step_mode = L.LR_STEP_FIXED if pr.step_mode == "fixed" else L.LR_STEP_ADAPTIVE
        s.n_fixed_steps = int(pr.n_fixed_steps)
        s.color_mode = L.LR_COLOR_HUE if pr.color_mode == "hue" else L.LR_COLOR_LUT
        s.max_samples = int(pr.max_samples)
        s.shading = {"none": L.LR_SHADE_NONE, "directional": L.LR_SHADE_DIRECTIONAL,
                     "headlight": L.LR_SHADE_HEADLIGHT}[pr.shading]
        s.light[:] = [float(x) for x in pr.light]
        return s


def render_workspace(views: Sequence, device) -> torch.Tensor:
    """Device workspace for lr_render_scheduled over these views (256-byte aligned)."""
    arr, _ = view_array(views)
    n = ctypes.c_int64(0)
    L.check(L.lib().lr_render_workspace_size(arr, len(views), ctypes.byref(n)))
    ws = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + n.value]


def render(scene: Scene, views: Sequence, bezier=None, lut=None, out=None, nsamples: bool = False,
           schedule: bool = True, workspace: Optional[torch.Tensor] = None, queues: int = 0,
           workgroups: int = 0):
    """Render views into one packed RGBA tensor [sum W*H, 4] (float32).
    Returns (rgba, offsets, nsamples or None).  schedule: deal the work
    longest first from a per-launch cost estimate (lr_render_scheduled, in a
    workspace from render_workspace or allocated here); otherwise from the
    middle of each view outwards (lr_render).  queues 1 or 8: persistent
    workgroups take the tiles from that many atomic counters instead of the
    hardware's dispatch (lr_render_persistent, `workgroups` of them, 0 for as
    many as the GPU holds).  The images are the same."""
    dev = scene.volume.device
    arr, offs = view_array(views)
    total = sum(v.width * v.height for v in views)
    if out is None:
        out = torch.empty((total, 4), dtype=torch.float32, device=dev)
    ns = torch.empty(total, dtype=torch.int32, device=dev) if nsamples else None
    s = scene.struct(bezier, lut)
    if queues:
        ws = render_workspace(views, dev) if workspace is None else workspace
        L.check(L.lib().lr_render_persistent(ctypes.byref(s), arr, len(views), _ptr(out), _ptr(ns), queues,
                                             int(schedule), workgroups, _ptr(ws), ws.numel() * ws.element_size(),
                                             _stream(dev)))
    elif schedule:
        ws = render_workspace(views, dev) if workspace is None else workspace
        L.check(L.lib().lr_render_scheduled(ctypes.byref(s), arr, len(views), _ptr(out), _ptr(ns), _ptr(ws),
                                            ws.numel() * ws.element_size(), _stream(dev)))
    else:
        L.check(L.lib().lr_render(ctypes.byref(s), arr, len(views), _ptr(out), _ptr(ns), _stream(dev)))
    return out, offs, ns


def render_backward(scene: Scene, views: Sequence, rgba_fwd, grad_rgba, bezier=None, lut=None):
    dev = scene.volume.device
    arr, _ = view_array(views)
    bez = scene.volume.bezier if bezier is None else bezier
    lut_t = scene.lut if lut is None else lut
    gb = torch.zeros(bez.shape, dtype=torch.float32, device=dev)
    gl = torch.zeros((256, 4), dtype=torch.float32, device=dev)
    s = scene.struct(bez, lut_t)
    L.check(L.lib().lr_render_backward(ctypes.byref(s), arr, len(views), _ptr(rgba_fwd.contiguous()),
                                       _ptr(grad_rgba.contiguous()), _ptr(gb), _ptr(gl), _stream(dev)))
    return gb, gl


class RenderFunction(torch.autograd.Function):
    """Differentiable render: inputs (bezier f32 [n_elem, stride], lut f32
    [256, 4]); output packed RGBA.  The backward re-marches the rays in the
    adjoint kernel."""

    @staticmethod
    def forward(ctx, bezier, lut, scene, views):
        rgba, _, _ = render(scene, views, bezier=bezier.contiguous(), lut=lut.contiguous())
        ctx.scene, ctx.views = scene, views
        ctx.save_for_backward(bezier, lut, rgba)
        return rgba

    @staticmethod
    def backward(ctx, grad):
        bezier, lut, rgba = ctx.saved_tensors
        gb, gl = render_backward(ctx.scene, ctx.views, rgba, grad, bezier=bezier.contiguous(), lut=lut.contiguous())
        return gb, gl, None, None


def trace(scene: Scene, view, pixels: np.ndarray, max_out: int = 4096, bezier=None):
    """(t, element, ds, count) of the first max_out samples of each pixel's ray."""
    dev = scene.volume.device
    pix = torch.from_numpy(np.ascontiguousarray(pixels, dtype=np.int32).reshape(-1, 2)).to(dev)
    n = pix.shape[0]
    t = torch.zeros((n, max_out), dtype=torch.float32, device=dev)
    e = torch.full((n, max_out), -1, dtype=torch.int32, device=dev)
    ds = torch.zeros((n, max_out), dtype=torch.float32, device=dev)
    cnt = torch.zeros(n, dtype=torch.int32, device=dev)
    v = view_struct(view, 0)
    s = scene.struct(bezier)
    L.check(L.lib().lr_trace_rays(ctypes.byref(s), ctypes.byref(v), _ptr(pix), n, int(max_out), _ptr(t), _ptr(e),
                                  _ptr(ds), _ptr(cnt), _stream(dev)))
    return t, e, ds, cnt


def lookup(volume: Volume, points) -> torch.Tensor:
    """Element ids of points [n, 3] (Alg. 1, or the octree descent, on the GPU)."""
    pts = torch.as_tensor(points, dtype=torch.float32).to(volume.device).contiguous()
    out = torch.empty(pts.shape[0], dtype=torch.int32, device=volume.device)
    if volume.lookup == "octree":
        L.check(L.lib().lr_lookup_octree(_ptr(volume.heads), _ptr(volume.nodes), volume.n_nodes, volume.n_elem,
                                         _ptr(pts), pts.shape[0], _ptr(out), _stream(volume.device)))
        return out
    b = np.asarray(volume.forest.blocks, dtype=np.int32)
    L.check(L.lib().lr_lookup(_ptr(volume.heads), _ptr(volume.nodes), volume.n_nodes, _np_ptr(b),
                              volume.n_elem, _ptr(pts), pts.shape[0], _ptr(out), _stream(volume.device)))
    return out


def streamlines(scene: Scene, seeds, method: str = "rk4", step: str = "heuristic", precision: str = "mixed",
                base: float = 1.0, t_end: float = 1.0, tol: float = 1e-6, max_samples: int = 256):
    """Streamlines of the scene's 3-component field from seeds [n, 3] (Sec. 5).
    Returns (points [n, max_samples, 4] float32 (x, y, z, active),
    times [n, max_samples] float64, count [n] int32)."""
    dev = scene.volume.device
    sd = torch.as_tensor(np.asarray(seeds, dtype=np.float64).reshape(-1, 3)).to(dev).contiguous()
    n = sd.shape[0]
    pts = torch.empty((n, max_samples, 4), dtype=torch.float32, device=dev)
    tim = torch.empty((n, max_samples), dtype=torch.float64, device=dev)
    cnt = torch.empty(n, dtype=torch.int32, device=dev)
    prm = L.StreamParams()
    prm.method = L.RK_METHODS[method]
    prm.step_mode = {"heuristic": L.LR_STREAM_HEURISTIC, "constant": L.LR_STREAM_CONSTANT,
                     "embedded": L.LR_STREAM_EMBEDDED}[step]
    prm.precision = {"mixed": L.LR_PREC_MIXED, "single": L.LR_PREC_SINGLE}[precision]
    prm.max_samples = int(max_samples)
    prm.base, prm.t_end, prm.tol = float(base), float(t_end), float(tol)
    s = scene.struct()
    L.check(L.lib().lr_streamlines(ctypes.byref(s), ctypes.byref(prm), _ptr(sd), n, _ptr(pts), _ptr(tim), _ptr(cnt),
                                   _stream(dev)))
    return pts, tim, cnt


def unpack(rgba: torch.Tensor, views: Sequence, offsets: Sequence[int]) -> List[torch.Tensor]:
    """Split a packed RGBA tensor into per-view [H, W, 4] images."""
    return [rgba[o:o + v.width * v.height].view(v.height, v.width, 4) for v, o in zip(views, offsets)]

"""Emission-absorption ray casting of an LR-spline volume, FP64 (Sec. 4).

The accumulated radiance along a ray is the volume rendering integral Eq. 3;
it is discretised into segments of length ds_i and composited front to back
(Alg. 2):
    T      <- (1 - alpha_src)^(ds_i / xi)
    C_dst  <- C_dst + (1 - T)(1 - alpha_dst) C_src
    alpha_dst <- alpha_dst + (1 - T)(1 - alpha_dst)
with C_src, alpha_src from a transfer function of the field value (Sec. 4.1)
and xi a standard length.  Output per pixel: (C_r, C_g, C_b, alpha_dst) over a
black background.  This oracle composites every sample (no early stop).

Sampling schedules
  'fixed'    N segments of length (t_exit - t_entry)/N, sampled at midpoints
  'adaptive' Eq. 4 (Sec. 4.2): at t, sample p(t), find its element e, step
             ds = 2^-d * min side(e) with d the degree (max over axes); the
             segment composited is min(ds, t_exit - t); t <- t + ds; stop at
             t >= t_exit.  t, ds and t_exit - t are FP32 (replayed), so the
             element sequence matches a GPU that does the same FP32 operations.
  'fine'     fixed fine step 2^-12 (midpoints, last segment clipped), all FP64:
             the reference for the discretisation error of the schedules above.

Local illumination (Sec. 4.1, optional): C_src is multiplied by the diffuse
intensity I = max(0.4, |l . n|), n the unit normal of the isosurface through
the sample (the normalised gradient of the scalar field; for vector fields the
gradient of |f|, which is parallel to sum_c f_c grad f_c); I = 0.4 where the
gradient vanishes.  l is a fixed unit vector ('directional') or the unit
vector from the sample back along the ray towards the eye ('headlight').

Transfer function: value range [vmin, vmax] maps to s = clamp((v-vmin)/(vmax-vmin),
0, 1) * 255; RGBA = (1-w) LUT[i0] + w LUT[i1], i0 = floor(s), i1 = min(i0+1, 255),
w = s - i0; alpha_src <- min(alpha_src, 1 - 2^-16).  'hue' colour mode (vector
fields): v = |f|, alpha from the LUT, RGB = hsv(h, 1, 1) with
h = atan2(f_y, f_x) / 2pi mod 1 (h = 0 when f_x = f_y = 0).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import bezier as obez
from .camera import f32, positions, primary_rays
from .lookup import ElementIndex

MAX_SAMPLES = 1 << 16      # per-ray sample cap of the adaptive schedule
FINE_STEP = 2.0 ** -12


def transfer(v: np.ndarray, lut: np.ndarray, vmin: float, vmax: float):
    """LUT lookup with linear interpolation.  Returns rgba [m,4] and the
    interpolation state (s, i0, i1, w, inside) used by the derivative."""
    x = (np.asarray(v, dtype=np.float64) - vmin) / (vmax - vmin)
    inside = (x > 0.0) & (x < 1.0)
    s = np.clip(x, 0.0, 1.0) * 255.0
    i0 = np.minimum(np.floor(s).astype(np.int64), 255)
    i1 = np.minimum(i0 + 1, 255)
    w = s - i0
    lut = np.asarray(lut, dtype=np.float64)
    rgba = (1.0 - w)[:, None] * lut[i0] + w[:, None] * lut[i1]
    return rgba, (s, i0, i1, w, inside)


def hsv_full(h: np.ndarray) -> np.ndarray:
    """RGB of hue h in [0,1) at full saturation and value (hexcone model)."""
    h6 = np.asarray(h, dtype=np.float64) * 6.0
    k = np.floor(h6)
    f = h6 - k
    k = k.astype(np.int64) % 6
    one, zero = np.ones_like(f), np.zeros_like(f)
    table = [(one, f, zero), (1 - f, one, zero), (zero, one, f),
             (zero, 1 - f, one), (f, zero, one), (one, zero, 1 - f)]
    out = np.zeros(h6.shape + (3,))
    for s, (r, g, b) in enumerate(table):
        m = k == s
        out[m, 0], out[m, 1], out[m, 2] = r[m], g[m], b[m]
    return out


def hue(fx: np.ndarray, fy: np.ndarray) -> np.ndarray:
    zero = (fx == 0) & (fy == 0)
    h = np.mod(np.arctan2(fy, fx) / (2.0 * np.pi), 1.0)
    h = np.where(zero | (h >= 1.0), 0.0, h)
    return h


def source_terms(f: np.ndarray, sc):
    """C_src [m,3], alpha_src [m] (clamped), alpha before the clamp, and the
    transfer state, for field values f [m, ncomp]."""
    if sc.color_mode == "hue":
        v = np.sqrt((f * f).sum(axis=1))
        rgba, st = transfer(v, sc.lut, sc.vmin, sc.vmax)
        csrc = hsv_full(hue(f[:, 0], f[:, 1]))
    else:
        v = f[:, 0]
        rgba, st = transfer(v, sc.lut, sc.vmin, sc.vmax)
        csrc = rgba[:, :3]
    a_raw = rgba[:, 3]
    return csrc, np.minimum(a_raw, sc.alpha_clamp), a_raw, v, st


def illumination(f: np.ndarray, grad: np.ndarray, ldir: np.ndarray) -> np.ndarray:
    """I = max(0.4, |l . n|) for field values f [m, ncomp], gradients
    grad [m, ncomp, 3] and unit light vectors ldir [m, 3]."""
    if f.shape[1] == 1:
        n = grad[:, 0, :]
    else:
        n = (f[:, :, None] * grad).sum(axis=1)
    nn = np.sqrt((n * n).sum(axis=1))
    cos = np.divide(np.abs((n * ldir).sum(axis=1)), nn, out=np.zeros(nn.shape), where=nn > 0)
    return np.maximum(0.4, cos)


def composite(C, A, csrc, asrc, ds, xi):
    """One step of Alg. 2 for a batch of rays, in place (FP64)."""
    T = (1.0 - asrc) ** (ds / xi)
    C += ((1.0 - T) * (1.0 - A))[:, None] * csrc
    A += (1.0 - T) * (1.0 - A)
    return T


@dataclass
class Scene:
    p: tuple
    lut: np.ndarray
    vmin: float
    vmax: float
    xi: float
    alpha_clamp: float
    color_mode: str
    step_mode: str
    n_fixed_steps: int
    shading: str = "none"          # 'none', 'directional' or 'headlight'
    light: tuple = (0.0, 0.0, 1.0)

    @staticmethod
    def of(wl, shading="none", light=(0.0, 0.0, 1.0)):
        return Scene(tuple(int(v) for v in wl.spline.p), np.asarray(wl.lut, dtype=np.float64),
                     float(wl.vmin), float(wl.vmax), float(wl.xi), float(wl.alpha_clamp),
                     wl.color_mode, wl.step_mode, int(wl.n_fixed_steps), shading, tuple(light))

    def light_dirs(self, d: np.ndarray) -> np.ndarray:
        """Unit light vectors [m, 3] for rays of direction d [m, 3]."""
        if self.shading == "headlight":
            d = -np.asarray(d, dtype=np.float64)
            return d / np.sqrt((d * d).sum(axis=1))[:, None]
        l = np.asarray(self.light, dtype=np.float64)
        return np.broadcast_to(l / np.sqrt((l * l).sum()), (np.asarray(d).shape[0], 3))

    def shaded(self, field, x, e, f, csrc, d):
        """C_src times the local illumination (unchanged without shading)."""
        if self.shading == "none":
            return csrc
        return csrc * illumination(f, field.grad(x, e), self.light_dirs(d))[:, None]


class LRField:
    """f from the LR B-splines (Cox-de Boor), Eq. 2."""

    def __init__(self, evaluator):
        self.ev = evaluator

    def __call__(self, x, e):
        return self.ev.evaluate(x)

    def grad(self, x, e):
        return self.ev.gradient(x)


class BezierField:
    """f from per-element Bezier blocks C [n_elem, ncomp, nc] (Sec. 3.2.3)."""

    def __init__(self, spline, C):
        self.p = tuple(int(v) for v in spline.p)
        self.box = spline.elem_box
        self.C = C

    def __call__(self, x, e):
        return obez.evaluate(self.p, self.C[e], self.box[e], x)


def fixed_sample_t(t0: np.ndarray, dsf: np.ndarray, k: int) -> np.ndarray:
    """Parameter of the k-th fixed-step sample: the midpoint of segment k of
    N equal segments of length dsf starting at the entry t0 (FP32, R9)."""
    return t0 + f32(k + 0.5) * dsf


def render_rays(sc: Scene, elem_box, eidx: ElementIndex, field, o, d, t0, t1, hit,
                mode: str = "S", record: bool = False):
    """Composite the rays (o, d) over [t0, t1).  mode 'S' follows the scene's
    schedule (fixed or adaptive), 'F' the fine fixed step.  Returns
    (rgba [R,4], nsamples [R], records)."""
    R = o.shape[0]
    C = np.zeros((R, 3))
    A = np.zeros(R)
    ns = np.zeros(R, dtype=np.int64)
    recs = []
    dmax = max(sc.p)
    if mode == "F":
        o64, d64 = o.astype(np.float64), d.astype(np.float64)
        L = (t1.astype(np.float64) - t0.astype(np.float64))
        nseg = np.where(hit, np.ceil(L / FINE_STEP), 0).astype(np.int64)
        for k in range(int(nseg.max(initial=0))):
            idx = np.nonzero(k < nseg)[0]
            a = t0[idx].astype(np.float64) + k * FINE_STEP
            b = np.minimum(a + FINE_STEP, t1[idx].astype(np.float64))
            tm = 0.5 * (a + b)
            x = np.clip(o64[idx] + tm[:, None] * d64[idx], 0.0, 1.0)
            e = eidx.find(x)
            f = field(x, e)
            csrc, asrc, _, _, _ = source_terms(f, sc)
            csrc = sc.shaded(field, x, e, f, csrc, d[idx])
            Cs, As = C[idx], A[idx]
            composite(Cs, As, csrc, asrc, b - a, sc.xi)
            C[idx], A[idx] = Cs, As
            ns[idx] += 1
        return np.concatenate([C, A[:, None]], axis=1), ns, recs
    if sc.step_mode == "fixed":
        N = sc.n_fixed_steps
        dsf = (t1 - t0) / f32(N)
        for k in range(N):
            idx = np.nonzero(hit)[0]
            t = fixed_sample_t(t0[idx], dsf[idx], k)
            x32 = positions(o[idx], d[idx], t)
            x = x32.astype(np.float64)
            e = eidx.find(x)
            f = field(x, e)
            csrc, asrc, a_raw, v, st = source_terms(f, sc)
            csrc = sc.shaded(field, x, e, f, csrc, d[idx])
            Cs, As = C[idx], A[idx]
            Tbefore = 1.0 - As
            T = composite(Cs, As, csrc, asrc, dsf[idx].astype(np.float64), sc.xi)
            C[idx], A[idx] = Cs, As
            ns[idx] += 1
            if record:
                recs.append(dict(idx=idx, t=t, e=e, ds=dsf[idx], x=x, f=f, v=v, st=st, csrc=csrc,
                                 asrc=asrc, a_raw=a_raw, Tb=Tbefore, a=1.0 - T))
        return np.concatenate([C, A[:, None]], axis=1), ns, recs
    # adaptive, Eq. 4
    t = t0.copy()
    active = hit.copy()
    scale = f32(2.0 ** -dmax)
    while np.any(active):
        idx = np.nonzero(active)[0]
        ti = t[idx]
        x32 = positions(o[idx], d[idx], ti)
        x = x32.astype(np.float64)
        e = eidx.find(x)
        bx = elem_box[e].astype(f32)
        side = np.minimum(np.minimum(bx[:, 3] - bx[:, 0], bx[:, 4] - bx[:, 1]), bx[:, 5] - bx[:, 2])
        ds = side * scale
        dse = np.minimum(ds, t1[idx] - ti)
        f = field(x, e)
        csrc, asrc, a_raw, v, st = source_terms(f, sc)
        csrc = sc.shaded(field, x, e, f, csrc, d[idx])
        Cs, As = C[idx], A[idx]
        Tbefore = 1.0 - As
        T = composite(Cs, As, csrc, asrc, dse.astype(np.float64), sc.xi)
        C[idx], A[idx] = Cs, As
        ns[idx] += 1
        if record:
            recs.append(dict(idx=idx, t=ti, e=e, ds=dse, x=x, f=f, v=v, st=st, csrc=csrc,
                             asrc=asrc, a_raw=a_raw, Tb=Tbefore, a=1.0 - T))
        tn = ti + ds
        t[idx] = tn
        active[idx] = (tn < t1[idx]) & (ns[idx] < MAX_SAMPLES)
    return np.concatenate([C, A[:, None]], axis=1), ns, recs


def render_view(wl, view, field, eidx=None, ii=None, jj=None, mode="S", record=False, shading="none",
                light=(0.0, 0.0, 1.0)):
    """Render pixels (ii, jj) of a view (all pixels by default)."""
    from .camera import pixel_grid
    if ii is None:
        ii, jj = pixel_grid(view)
    if eidx is None:
        eidx = ElementIndex(wl.spline.elem_box)
    o, d, t0, t1, hit = primary_rays(view, ii, jj)
    return render_rays(Scene.of(wl, shading, light), wl.spline.elem_box, eidx, field, o, d, t0, t1, hit,
                       mode=mode, record=record)

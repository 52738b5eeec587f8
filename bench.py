"""Throughput of the LR-spline volume renderer on one MI355X.

Workload: the 1080p vector-field volume (tri-degree (2,2,2), 3 components,
~200k elements refined along a vortex tube; |v| through the table opacity,
hue from direction; 1920x1080 perspective view; Eq. 4 adaptive step; FP32).
A step is one frame: one lr_render launch over the whole view with the volume
resident in HBM.  Samples are the (ray, sample) evaluations of the schedule,
counted by a counting launch before the timed region.

Prints one JSON line: spline samples/s (value), frames/s, p50/p99 frame
latency, the roofline object of the render kernel, and the FP64 oracle timed
on a bounded sample of the same workload on the host cores; alongside, the
timed frame's accuracy against the oracle, the FP16-storage, illuminated,
streamline, adjoint and serving legs, and the other workloads (per_config).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3     # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("render.hip", "eval.h", "common.h", "lookup.h", "schedule.h")


def kernel_digest() -> str:
    """SHA-1 of the render kernel's code (its sources with comments and
    whitespace removed), so that the counters stay attached to the code they
    were taken on."""
    import hashlib
    import re
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1707_01170_amd", "csrc", name)) as f:
            code = re.sub(r"/\*.*?\*/", " ", f.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()


def measured_traffic(blocks: int):
    """HBM bytes per render launch from the committed counter summary, or None
    if the render kernel's code changed since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "render_kernel_vector1080p_traffic.json")) as f:
            rec = json.load(f)
        src = kernel_digest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_code_sha1") != src or rec.get("forest_blocks") != blocks:
        return None
    return float(rec["traffic_bytes_per_launch"])


# Algorithmic FP32 operations of one sample of the forward march (a fused
# multiply-add counts 2, a transcendental 1): the 1-D Bernstein bases (6, 15,
# 30 for p = 1, 2, 3), the tensor contraction 2((p+1)^3 + (p+1)^2 + (p+1))
# per component, about 40 for the position, local coordinates, table look-up
# and compositing (log1p/expm1 of the opacity correction), and for 3-vectors
# |v| with its square root (6) and the azimuth hue (atan2, hexcone, about 30):
# 133, 238 and 325 for the degree-2 scalar, degree-3 scalar and degree-2
# vector samples.
def flops_per_sample(p: int, ncomp: int) -> int:
    q = p + 1
    bases = {1: 6, 2: 15, 3: 30}[p]
    return bases + 2 * (q ** 3 + q ** 2 + q) * ncomp + 40 + (36 if ncomp == 3 else 0)


# The adjoint re-marches the forward (the forward's count) and per sample forms
# the compositing derivative (prefix/suffix terms, about 40), the table-row
# sums and slope (about 30) and scatters dv/dC_j = B_j(u) into the element's
# gradient (2 (p+1)^3 + 2 (p+1)^2 + ...: 72 for p = 2).
ADJOINT_EXTRA_FLOPS = {1: 40 + 30 + 24, 2: 40 + 30 + 72, 3: 40 + 30 + 160}


def oracle_pixels(wl, view, ii, jj):
    """The FP64 oracle's RGBA (schedule-matched mode) of pixels (ii, jj) of a
    view, over a fork pool of the host cores.  Returns (samples, seconds,
    cores, rgba).  Runs before any GPU initialisation (the pool forks)."""
    import multiprocessing as mp

    from oracle.bspline import LREvaluator
    from oracle.lookup import ElementIndex
    ev, ei = LREvaluator(wl.spline), ElementIndex(wl.spline.elem_box)
    cores = min(len(os.sched_getaffinity(0)), 16)
    chunks = np.array_split(np.arange(len(ii)), cores)
    global _CPU_JOB
    _CPU_JOB = (wl, view, ev, ei, ii, jj)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        parts = pool.map(_cpu_chunk, chunks)
    dt = time.perf_counter() - t0
    return sum(c for c, _ in parts), dt, cores, np.concatenate([r for _, r in parts])


def cpu_baseline(wl, n_rays: int, seed: int = 11):
    """The FP64 oracle (schedule-matched mode) on n_rays seeded pixels of the
    view, split over a fork pool of the host cores.  Returns samples/s, the
    cores used, the samples, the wall time, and the pixels with their oracle
    RGBA (compared with the GPU frames afterwards)."""
    view = wl.views[0]
    rng = np.random.default_rng(seed)
    ii = rng.integers(0, view.width, n_rays)
    jj = rng.integers(0, view.height, n_rays)
    counts, dt, cores, rgba = oracle_pixels(wl, view, ii, jj)
    return float(counts) / dt, cores, int(counts), dt, (ii, jj, rgba)


_CPU_JOB = None


def _cpu_chunk(idx):
    from oracle import render as orr
    wl, view, ev, ei, ii, jj = _CPU_JOB
    rgba, ns, _ = orr.render_view(wl, view, orr.LRField(ev), eidx=ei, ii=ii[idx], jj=jj[idx])
    return int(ns.sum()), rgba


def accuracy(frame, view, oracle_pix):
    """Peak-relative max and RMS difference of a GPU frame's pixels to the
    oracle's RGBA of the same pixels (max |x - ref| / max |ref|)."""
    ii, jj, ref = oracle_pix
    got = frame.view(view.height, view.width, 4)[torch_index(jj), torch_index(ii)].cpu().numpy().astype(np.float64)
    scale = np.abs(ref).max()
    return {"max": float(np.abs(got - ref).max() / scale), "rms": float(np.sqrt(((got - ref) ** 2).mean()) / scale)}


def torch_index(a):
    import torch
    return torch.from_numpy(np.asarray(a, dtype=np.int64))


# The other workloads, each as its parity tests and legs run it: name, label,
# forest blocks per axis, Bezier block storage, and the view (None: the
# workload's own views; "serve2048": the first 2048^2 request of the serving
# stream, launched as the server launches it, in centre-out order).  Rays against the oracle: every pixel of a view up to 64^2, else
# 1 024 seeded pixels of the first view.
PER_CONFIG = (("scalar_ortho64", "scalar (2,2,2), 4^3 mesh + 20 refinements, 64x64 ortho along z, 256 fixed steps",
               16, "f32", None),
              ("blobs50k", "scalar (3,3,3), ~50k elements, 1024x1024 persp, Eq. 4 steps", 256, "f32", None),
              ("blobs50k", "serving's largest request: the blob volume at 2048x2048, FP16 blocks, forest 128^3",
               128, "f16", "serve2048"),
              ("scalar20k", "scalar (2,2,2), ~20k elements, 4 x 512x512 persp, Eq. 4 steps (the differentiable "
               "step's forward)", 128, "f32", None))


def per_config_views(name, which):
    import lrgen
    wl = lrgen.cached(name)
    if which == "serve2048":
        return wl, [next(r.view for r in lrgen.blob_requests() if r.view.width == 2048)]
    return wl, list(wl.views)


def per_config_oracle(seed: int = 13):
    """Oracle pixels of every PER_CONFIG workload (before GPU initialisation)."""
    out = []
    for name, _, _, _, which in PER_CONFIG:
        wl, views = per_config_views(name, which)
        v = views[0]
        if v.width * v.height <= 64 * 64:
            jj, ii = np.divmod(np.arange(v.width * v.height), v.width)
        else:
            rng = np.random.default_rng(seed)
            ii, jj = rng.integers(0, v.width, 1024), rng.integers(0, v.height, 1024)
        _, dt, _, rgba = oracle_pixels(wl, v, ii, jj)
        log("oracle pixels of %s (%s): %d rays in %.1f s" % (name, which or "own views", len(ii), dt))
        out.append((ii, jj, rgba))
    return out


def per_config(dev, oracle, steps: int = 20):
    """Each other workload: frame time (p50/p99 over launches timed with HIP
    events), samples/s and frames/s, the fraction of the FP32 vector peak at
    the algorithmic flops per sample, the frame's pixels against the oracle,
    and the element look-up against the oracle's on 65 536 points (uniform,
    plus corners of elements: dyadic points on faces) -- bit-exact or not."""
    import torch

    import paper_1707_01170_amd as P
    from oracle.lookup import ElementIndex
    res = []
    for (name, label, blocks, dtype, which), opix in zip(PER_CONFIG, oracle):
        wl, views = per_config_views(name, which)
        vol = P.Volume(wl.spline, blocks=blocks, dtype=dtype, device=dev)
        sc = P.Scene(vol, P.RenderParams.of(wl))
        out, _, ns = P.render(sc, views, nsamples=True)
        samples = int(ns.to(torch.int64).sum())
        ws = P.render_workspace(views, dev)
        stream = torch.cuda.current_stream(dev)
        order = which != "serve2048"            # the server launches lr_render (centre-out)
        for _ in range(3):
            P.render(sc, views, out=out, workspace=ws, schedule=order)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            P.render(sc, views, out=out, workspace=ws, schedule=order)
            b.record(stream)
        torch.cuda.synchronize()
        t = np.array([a.elapsed_time(b) for a, b in ev])
        acc = accuracy(out[:views[0].width * views[0].height], views[0], opix)
        rng = np.random.default_rng(17)
        box = wl.spline.elem_box
        pts = np.concatenate([rng.random((65536 - 4096, 3)), box[rng.integers(0, box.shape[0], 4096), :3]])
        ids = P.lookup(vol, pts.astype(np.float32)).cpu().numpy()
        ref = ElementIndex(box).find(pts.astype(np.float32).astype(np.float64))
        fl = flops_per_sample(vol.p[0], vol.ncomp) * samples / (t.mean() / 1e3) / 1e12
        r = {"workload": label, "views": [[v.width, v.height] for v in views], "blocks": dtype,
             "forest_blocks": blocks, "samples_per_frame": samples, "ms_mean": float(t.mean()),
             "p50_ms": float(np.percentile(t, 50)), "p99_ms": float(np.percentile(t, 99)),
             "samples_per_s": samples / (t.mean() / 1e3), "frames_per_s": 1e3 / t.mean(),
             "roofline_frac": fl / PEAK_FP32_TFLOPS, "accuracy": dict(acc, rays=int(len(opix[0]))),
             "lookup_bit_exact": bool(np.array_equal(ids, ref)), "lookup_points": int(len(pts))}
        log("%s: %.3f ms (p99 %.3f), %.3g samples/s, %.1f%% of the FP32 peak; vs oracle max %.2e rms %.2e "
            "on %d rays; look-up bit-exact %s" % (name if which is None else which, r["ms_mean"], r["p99_ms"],
                                                  r["samples_per_s"], 100 * r["roofline_frac"], acc["max"],
                                                  acc["rms"], len(opix[0]), r["lookup_bit_exact"]))
        res.append(r)
        del vol, sc, out, ws
    return res


def adjoint_step(dev, steps: int = 10):
    """One differentiable render step on the (2,2,2) scalar volume: forward of
    4 views of 512^2, L2 loss against targets from the second coefficient set,
    backward to the Bezier blocks and the table."""
    import torch

    import lrgen
    import paper_1707_01170_amd as P
    wl = lrgen.cached("scalar20k")
    vol = P.Volume(wl.spline, blocks=128, device=dev)
    sc = P.Scene(vol, P.RenderParams.of(wl))
    tgt_bez, _ = vol.extract(wl.extra["coef_target"], "f32")
    tgt, _, _ = P.render(sc, wl.views, bezier=tgt_bez)
    rgba, _, ns = P.render(sc, wl.views, nsamples=True)
    samples = int(ns.to(torch.int64).sum())
    bez = vol.bezier.clone().requires_grad_(True)
    lut = sc.lut.clone().requires_grad_(True)

    def step():
        out = P.RenderFunction.apply(bez, lut, sc, wl.views)
        loss = ((out[:, :3] - tgt[:, :3]) ** 2).sum()
        loss.backward()
        return loss

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fa, fb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        step()
    b.record()
    fa.record()
    for _ in range(steps):
        P.render(sc, wl.views, bezier=bez.detach())
    fb.record()
    torch.cuda.synchronize()
    # adjoint of the extraction: dL/d(blocks) -> dL/d(LR coefficients)
    g = bez.grad.detach().clone()
    vol.extract_backward(g)
    xa, xb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    xa.record()
    for _ in range(steps):
        vol.extract_backward(g)
    xb.record()
    torch.cuda.synchronize()
    # the adjoint kernel alone: lr_render_backward into preallocated gradients
    # (it accumulates, so no clearing inside the timed region)
    import ctypes
    from paper_1707_01170_amd import _lib as L
    from paper_1707_01170_amd.api import view_array
    arr, _ = view_array(wl.views)
    gup = torch.randn_like(rgba)
    gbz = torch.zeros_like(vol.bezier)
    glt = torch.zeros((256, 4), dtype=torch.float32, device=dev)
    scs = sc.struct()
    st = torch.cuda.current_stream(dev)
    hs = ctypes.c_void_p(st.cuda_stream)

    def bwd():
        L.check(L.lib().lr_render_backward(ctypes.byref(scs), arr, len(wl.views), ctypes.c_void_p(rgba.data_ptr()),
                                           ctypes.c_void_p(gup.data_ptr()), ctypes.c_void_p(gbz.data_ptr()),
                                           ctypes.c_void_p(glt.data_ptr()), hs))
    for _ in range(2):
        bwd()
    ka, kb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ka.record(st)
    for _ in range(steps):
        bwd()
    kb.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    fms = fa.elapsed_time(fb) / steps
    xms = xa.elapsed_time(xb) / steps
    bms = ka.elapsed_time(kb) / steps
    fl = flops_per_sample(vol.p[0], 1) + ADJOINT_EXTRA_FLOPS[vol.p[0]]
    achieved = fl * samples / (bms / 1e3) / 1e12
    log("adjoint: forward+loss+backward %.3f ms (forward alone %.3f ms, adjoint kernel %.3f ms), %d samples per "
        "forward; extraction adjoint %.3f ms; adjoint %.2f TFLOP/s (%.1f%% of %.1f)"
        % (ms, fms, bms, samples, xms, achieved, 100 * achieved / PEAK_FP32_TFLOPS, PEAK_FP32_TFLOPS))
    return {"workload": "scalar (2,2,2), %d elements, 4 x 512^2 views, L2 loss, grad wrt Bezier blocks and table"
                        % vol.n_elem, "step_ms": ms, "forward_ms": fms, "backward_kernel_ms": bms,
            "samples_per_forward": samples, "samples_per_s_fwd_bwd": samples / (ms / 1e3),
            "extraction_adjoint_ms": xms,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP32_TFLOPS, "flops_per_sample": fl,
                         "kernel": "backward_kernel (re-march + adjoint)"}}


def lookup_sweep(dev, name: str, steps: int = 10):
    """Frame time through each look-up structure of Sec. 3.2 on one workload:
    k-d forests of 1 (a single k-d tree) to 512 blocks per axis (512 is the
    O(1) table for knots at level <= 9) and the octree.  Images are identical
    across structures; only the look-up cost differs."""
    import torch

    import lrgen
    import paper_1707_01170_amd as P
    wl = lrgen.cached(name)
    prm = P.RenderParams.of(wl)
    view = wl.views[0]
    rows = []
    ref = None
    for kind, blocks in [("forest", 1), ("forest", 4), ("forest", 16), ("forest", 64), ("forest", 128),
                         ("forest", 256), ("forest", 512), ("octree", 0)]:
        t0 = time.perf_counter()
        vol = P.Volume(wl.spline, blocks=max(blocks, 1), device=dev, lookup=kind)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        sc = P.Scene(vol, prm)
        out, _, _ = P.render(sc, [view])
        torch.cuda.synchronize()
        same = None
        if ref is None:
            ref = out.clone()
        else:
            same = bool(torch.equal(out, ref))
        for _ in range(2):
            P.render(sc, [view], out=out)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            P.render(sc, [view], out=out)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        st = vol.look_stats
        row = {"structure": kind if kind == "octree" else "forest %d^3" % blocks, "ms_per_frame": ms,
               "build_s": build_s, "n_nodes": st["n_nodes"], "n_heads": st["n_heads"], "n_direct": st["n_direct"],
               "depth_min": st["min_depth"], "depth_max": st["max_depth"], "depth_mean": st["mean_depth"],
               "depth_var": st["var_depth"], "image_identical_to_first": same}
        log("lookup sweep %s %-12s %8.3f ms  depth %d..%d mean %.3f var %.3f  nodes %d  direct %d/%d  build %.2f s"
            % (name, row["structure"], ms, st["min_depth"], st["max_depth"], st["mean_depth"], st["var_depth"],
               st["n_nodes"], st["n_direct"], st["n_heads"], build_s))
        rows.append(row)
        del vol, sc, out
        torch.cuda.empty_cache()
    return {"workload": "%s: %d elements, %dx%d view" % (name, wl.spline.n_elem, view.width, view.height),
            "rows": rows}


def dispatch_study(dev, name: str, steps: int = 20, blocks: int = 256):
    """Frame time of one view under each way of handing its tiles to the GPU:
    the hardware's dispatch of one workgroup per tile (ring order: lr_render;
    longest first: lr_render_scheduled) against persistent workgroups taking
    tiles from one atomic counter or from one per XCD (lr_render_persistent),
    in either order.  Every form renders the identical image."""
    import torch

    import lrgen
    import paper_1707_01170_amd as P
    wl = lrgen.cached(name)
    vol = P.Volume(wl.spline, blocks=blocks, device=dev)
    sc = P.Scene(vol, P.RenderParams.of(wl))
    view = wl.views[0]
    ws = P.render_workspace([view], dev)
    out = torch.empty((view.width * view.height, 4), dtype=torch.float32, device=dev)
    forms = [("hardware dispatch, ring order", dict(schedule=False)),
             ("hardware dispatch, longest first", dict(schedule=True)),
             ("1 queue, ring order", dict(schedule=False, queues=1)),
             ("1 queue, longest first", dict(schedule=True, queues=1)),
             ("8 queues (one per XCD), ring order", dict(schedule=False, queues=8)),
             ("8 queues (one per XCD), longest first", dict(schedule=True, queues=8))]
    rows, ref = [], None
    for label, kw in forms:
        P.render(sc, [view], out=out, workspace=ws, **kw)
        torch.cuda.synchronize()
        same = None
        if ref is None:
            ref = out.clone()
        else:
            same = bool(torch.equal(out, ref))
        for _ in range(2):
            P.render(sc, [view], out=out, workspace=ws, **kw)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            P.render(sc, [view], out=out, workspace=ws, **kw)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        log("dispatch study %s %-40s %8.3f ms  identical %s" % (name, label, ms, same))
        rows.append({"form": label, "ms_per_frame": ms, "image_identical_to_first": same})
    del vol, sc, out, ws
    torch.cuda.empty_cache()
    return {"workload": "%s: %d elements, %dx%d view, forest %d^3, FP32 blocks"
                        % (name, wl.spline.n_elem, view.width, view.height, blocks), "rows": rows}


def _stream_seeds(n: int, seed: int = 3):
    rng = np.random.default_rng(seed)
    lo, hi = np.array([0.35, 0.35, 0.2]), np.array([0.65, 0.65, 0.8])
    return lo + (hi - lo) * rng.random((n, 3))


def _timed_lines(sc, seeds, reps=3, **kw):
    import torch

    import paper_1707_01170_amd as P
    P.streamlines(sc, seeds, **kw)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        out = P.streamlines(sc, seeds, **kw)
    b.record()
    torch.cuda.synchronize()
    return out, a.elapsed_time(b) / reps


def stream_lines(sc, n_seeds: int = 16384, study: bool = False):
    """The streamline compute stage (Sec. 5.3) on the vortex volume: RK4 with
    the Eq. 4 heuristic step, mixed precision; accuracy by Eq. 7 against an
    RKF5 reference with a small constant step (computed by the library)."""
    from paper_1707_01170_amd import metrics
    seeds = _stream_seeds(n_seeds)
    kw = dict(method="rk4", step="heuristic", precision="mixed", base=1.0, t_end=1.0, max_samples=2048)
    (pts, tim, cnt), ms = _timed_lines(sc, seeds, **kw)
    steps = int((cnt.long() - 1).sum().item())
    sub = seeds[:256]
    ref = metrics.reference(sc, sub, 1.0, 2.0 ** -13)
    n_sub = 256
    E = metrics.error_metric(ref, pts[:n_sub].cpu().numpy(), tim[:n_sub].cpu().numpy(), cnt[:n_sub].cpu().numpy())
    log("streamlines: %d seeds, RK4 heuristic mixed: %.3f ms, %d steps (%.3g steps/s, %.3g field evaluations/s), "
        "E = %.3e" % (n_seeds, ms, steps, steps / (ms / 1e3), 4 * steps / (ms / 1e3), E))
    res = {"workload": "vortex volume (2,2,2) x3 comps, %d seeds in [0.35,0.65]^2 x [0.2,0.8], t_end 1, "
                       "at most 2048 points per line" % n_seeds,
           "method": "rk4, Eq. 4 heuristic step (base 1), FP64 outer loop / FP32 field", "ms": ms, "steps": steps,
           "steps_per_s": steps / (ms / 1e3), "field_evals_per_s": 4 * steps / (ms / 1e3),
           "error_eq7_first256": E}
    if study:
        rows = []
        cases = [(m, "heuristic", "mixed", b, None) for m in ("rk1", "rk2", "rk3", "rk4", "rk4_38", "rkf5")
                 for b in (1.0, 0.5, 0.25)]
        cases += [(m, "embedded", "mixed", 1.0, tol) for m in ("he", "bs", "rkf45") for tol in (1e-5, 1e-6, 1e-7, 1e-8)]
        cases += [("rk4", "constant", prec, b, None) for prec in ("mixed", "single") for b in (2.0 ** -6, 2.0 ** -9, 2.0 ** -12)]
        for m, step, prec, base, tol in cases:
            (p2, t2, c2), ms2 = _timed_lines(sc, sub, reps=1, method=m, step=step, precision=prec, base=base,
                                             t_end=1.0, tol=tol or 1e-6, max_samples=8192)
            e2 = metrics.error_metric(ref, p2.cpu().numpy(), t2.cpu().numpy(), c2.cpu().numpy())
            n2 = int((c2.long() - 1).sum().item())
            rows.append({"method": m, "step": step, "precision": prec, "base": base, "tol": tol, "E": e2,
                         "ms": ms2, "steps": n2})
            log("  study %-7s %-9s %-6s base %-9.4g tol %-7s E %.3e  %d steps  %.2f ms"
                % (m, step, prec, base, tol, e2, n2, ms2))
        res["study_256_seeds"] = rows
    return res


def serve_stream(n_req: int, dev):
    """The request stream on the (3,3,3) blob volume with FP16 Bezier storage:
    Poisson arrivals at 200/s, square views of 256..2048, continuous batching.
    Then the same requests with the arrival times compressed (time_scale < 1
    raises the offered rate; 0 offers everything at once), to find the rate
    the server sustains and how batching and latency respond to load."""
    import lrgen
    import paper_1707_01170_amd as P
    from paper_1707_01170_amd.serve import Server
    wl = lrgen.cached("blobs50k")
    vol = P.Volume(wl.spline, blocks=128, dtype="f16", device=dev)
    sc = P.Scene(vol, P.RenderParams.of(wl))
    reqs = lrgen.blob_requests(n=n_req)
    warm = Server(sc, budget_bytes=2 << 30).run(reqs[:8])
    log("serving: warm-up %d requests" % warm.n)
    srv = Server(sc, budget_bytes=2 << 30, n_streams=3)
    st = srv.run(reqs)
    log("serving: %d requests, p50 %.1f ms p99 %.1f ms, offered %.3g px/s served %.3g px/s, %d launches"
        % (st.n, st.p50_ms, st.p99_ms, st.offered_px_per_s, st.served_px_per_s, st.launches))
    sweep = []
    for scale in (0.5, 0.25, 0.1, 0.03, 0.0):
        r = srv.run(reqs, time_scale=scale)
        offered = r.offered_px_per_s if scale > 0 else None
        sweep.append({"time_scale": scale, "offered_px_per_s": offered, "served_px_per_s": r.served_px_per_s,
                      "p50_ms": r.p50_ms, "p99_ms": r.p99_ms, "launches": r.launches,
                      "views_per_launch": r.mean_views_per_launch, "max_inflight": r.max_inflight})
        log("serving load x%s: offered %s px/s, served %.3g px/s, %.2f views/launch, p50 %.1f ms p99 %.1f ms"
            % ("inf" if scale == 0 else "%.3g" % (1 / scale), "all at once" if offered is None else "%.3g" % offered,
               r.served_px_per_s, r.mean_views_per_launch, r.p50_ms, r.p99_ms))
    return {"workload": "blob volume (3,3,3) scalar, %d elements, FP16 blocks / FP32 arithmetic; %d requests, "
                        "Poisson 200/s, square 256..2048" % (vol.n_elem, st.n),
            "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms, "offered_px_per_s": st.offered_px_per_s,
            "served_px_per_s": st.served_px_per_s, "wall_s": st.wall_s, "launches": st.launches,
            "views_per_launch": st.mean_views_per_launch, "budget_bytes": 2 << 30,
            "load_sweep": sweep, "saturated_px_per_s": sweep[-1]["served_px_per_s"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--blocks", type=int, default=256)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16"])
    ap.add_argument("--cpu-rays", type=int, default=524288, help="rays of the oracle CPU baseline (0: skip)")
    ap.add_argument("--copy-calib", action="store_true", help="also run a plain copy of known size (counter scale)")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false", help="skip the adjoint step timing")
    ap.add_argument("--no-extras", dest="extras", action="store_false",
                    help="time only the plain frame (no FP16, illuminated or streamline legs; for counter runs)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the differentiable step on the scalar volume, printed as its own JSON line")
    ap.add_argument("--stream-study", action="store_true",
                    help="also compare every RK method / step rule / precision by the error metric Eq. 7")
    ap.add_argument("--lookup-sweep", action="store_true",
                    help="also time every look-up structure (forest sizes, octree) on the 1080p and blob workloads")
    ap.add_argument("--dispatch-study", action="store_true",
                    help="also time hardware dispatch against persistent work queues on the 1080p and blob workloads")
    ap.add_argument("--no-configs", dest="configs", action="store_false",
                    help="skip the other workloads (time, accuracy against the oracle, look-up check)")
    ap.add_argument("--serve", type=int, default=1000,
                    help="requests of the serving stream on the blob volume with FP16 blocks (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): the renderer has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    if args.adjoint_only:
        import torch
        print(json.dumps({"adjoint": adjoint_step(torch.device("cuda:0"), steps=args.steps)}), flush=True)
        return

    import lrgen
    log("generating workload")
    wl = lrgen.cached("vortex200k")
    view = wl.views[0]
    cpu = oracle_pix = None
    if args.cpu_rays > 0:       # before any GPU initialisation (the pool forks)
        log("oracle CPU baseline on %d rays" % args.cpu_rays)
        sps, cores, nsmp, dt, oracle_pix = cpu_baseline(wl, args.cpu_rays)
        cpu = {"value": sps, "unit": "samples/s", "cores": cores, "kind": "oracle",
               "sample": "%d seeded rays of the 1920x1080 view (%d samples, %.1f s), FP64, schedule-matched"
                         % (args.cpu_rays, nsmp, dt)}
        log("oracle %.3e samples/s on %d cores" % (sps, cores))
    cfg_oracle = per_config_oracle() if args.configs else None

    import torch

    import paper_1707_01170_amd as P
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    vol = P.Volume(wl.spline, blocks=args.blocks, dtype=args.dtype, device=dev)
    torch.cuda.synchronize()
    log("volume ready in %.2f s: %d elements, forest %s" % (time.perf_counter() - t0, vol.n_elem, vol.forest.stats))
    sc = P.Scene(vol, P.RenderParams.of(wl))
    views = [view]
    rgba, _, ns = P.render(sc, views, nsamples=True)
    torch.cuda.synchronize()
    samples = int(ns.to(torch.int64).sum().item())
    log("samples per frame %d (%.1f per hit ray)" % (samples, samples / max(1, int((ns > 0).sum().item()))))
    # lane efficiency of 8x8 tiles: samples / (64 * longest ray of the tile)
    H, W = view.height, view.width
    img = ns.view(H, W).to(torch.float32)
    img = torch.nn.functional.pad(img, (0, (-W) % 8, 0, (-H) % 8))
    tiles = img.view(img.shape[0] // 8, 8, img.shape[1] // 8, 8).permute(0, 2, 1, 3).reshape(-1, 64)
    lane_eff = float(tiles.sum() / (64 * tiles.max(1).values.sum()))
    log("tile lane efficiency %.3f" % lane_eff)
    out = torch.empty_like(rgba)
    ws = P.render_workspace(views, dev)     # the dispatch order's workspace, reused by every frame
    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        P.render(sc, views, out=out, workspace=ws)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        P.render(sc, views, out=out, workspace=ws)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = np.array([a.elapsed_time(b) for a, b in ev])      # ms, per launch, on the launch stream
    log("frame ms: mean %.3f p50 %.3f p99 %.3f; wall %.3f s" % (times.mean(), np.percentile(times, 50),
                                                               np.percentile(times, 99), wall))
    acc = None
    if oracle_pix is not None:     # the timed frame against the oracle's pixels
        acc = {args.dtype: accuracy(out, view, oracle_pix), "rays": int(oracle_pix[0].size)}
        log("accuracy of the timed frame (%s blocks) on %d oracle rays: peak-relative max %.2e rms %.2e"
            % (args.dtype, acc["rays"], acc[args.dtype]["max"], acc[args.dtype]["rms"]))
    fp16 = illumination = None
    if args.extras:
        # FP16 Bezier storage with FP32 arithmetic: the same frame
        vol16 = P.Volume(wl.spline, blocks=args.blocks, dtype="f16", device=dev)
        sc16 = P.Scene(vol16, P.RenderParams.of(wl))
        out16 = torch.empty_like(rgba)
        for _ in range(2):
            P.render(sc16, views, out=out16, workspace=ws)
        ha, hb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ha.record(stream)
        for _ in range(args.steps):
            P.render(sc16, views, out=out16, workspace=ws)
        hb.record(stream)
        torch.cuda.synchronize()
        f16_ms = ha.elapsed_time(hb) / args.steps
        f16_diff = float((out16 - rgba).abs().max() / rgba.abs().max())
        log("FP16 blocks: %.3f ms per frame (%.2fx), peak-relative difference to FP32 %.2e" % (f16_ms, times.mean() / f16_ms, f16_diff))
        fp16 = {"storage": "FP16 Bezier blocks, FP32 arithmetic", "ms_per_frame": f16_ms,
                "samples_per_s": samples / (f16_ms / 1e3), "peak_rel_diff_vs_f32": f16_diff}
        if oracle_pix is not None:
            acc["f16"] = accuracy(out16, view, oracle_pix)
            fp16["vs_oracle"] = acc["f16"]
            log("FP16 blocks against the oracle: peak-relative max %.2e rms %.2e" % (acc["f16"]["max"], acc["f16"]["rms"]))
        del vol16, sc16, out16
        # local illumination (Sec. 4.1): the same frame with a head light
        import dataclasses
        sc_lit = P.Scene(vol, dataclasses.replace(P.RenderParams.of(wl), shading="headlight"))
        for _ in range(2):
            P.render(sc_lit, views, out=out, workspace=ws)
        la, lb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        la.record(stream)
        for _ in range(args.steps):
            P.render(sc_lit, views, out=out, workspace=ws)
        lb.record(stream)
        torch.cuda.synchronize()
        lit_ms = la.elapsed_time(lb) / args.steps
        log("illuminated frame %.3f ms (%.2fx the plain frame)" % (lit_ms, lit_ms / times.mean()))
        illumination = {"shading": "headlight, I = max(0.4, |l.n|)", "ms_per_frame": lit_ms,
                        "ratio_to_plain": lit_ms / times.mean()}
    if args.copy_calib:
        n = 256 << 20
        src = torch.ones(n // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of %d bytes" % n)
    lines = stream_lines(sc, study=args.stream_study) if args.extras else None
    adjoint = adjoint_step(dev) if args.adjoint else None
    sweep = [lookup_sweep(dev, n) for n in ("vortex200k", "blobs50k")] if args.lookup_sweep else None
    study = ([dispatch_study(dev, "vortex200k", blocks=256), dispatch_study(dev, "blobs50k", blocks=128)]
             if args.dispatch_study else None)
    configs = per_config(dev, cfg_oracle) if cfg_oracle is not None else None
    serving = None
    if args.serve > 0:
        serving = serve_stream(args.serve, dev)
    fps = args.steps / wall
    value = samples * args.steps / wall
    fl = flops_per_sample(vol.p[0], vol.ncomp) * samples
    kern_s = times.mean() / 1e3
    achieved = fl / kern_s / 1e12
    traffic = measured_traffic(args.blocks)
    res = {
        "metric": "spline samples/s at 1080p (frames/s, p50/p99 frame latency alongside)",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "f32" else "f16-storage/f32",
        "data": "synthetic (seeded LR-spline volume; the paper's data sets are not available)",
        "config": {"workload": "vector field (2,2,2) x3 comps, %d elements, 1920x1080 persp, adaptive step (Eq. 4)"
                               % vol.n_elem, "samples_per_frame": samples, "forest_blocks": args.blocks,
                   "dispatch": "longest first by a per-frame cost estimate (lr_render_scheduled)"},
        "frames_per_s": fps,
        "tile_lane_efficiency": lane_eff,
        "p50_ms": float(np.percentile(times, 50)),
        "p99_ms": float(np.percentile(times, 99)),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     # FETCH_SIZE + WRITE_SIZE count L2 <-> fabric traffic (Infinity
                     # Cache hits included), an upper bound on the HBM bytes
                     "l2_fabric_GBps": None if traffic is None else traffic / kern_s / 1e9,
                     "flops_per_sample": flops_per_sample(vol.p[0], vol.ncomp), "kernel_ms": times.mean(),
                     # the frame's events also hold the two small kernels that estimate the dispatch order
                     "kernel": "render_kernel (with the dispatch-order pre-pass)"},
        "accuracy": acc,
        "cpu_baseline": cpu,
        "serving": serving,
        "adjoint": adjoint,
        "illumination": illumination,
        "fp16_storage": fp16,
        "streamlines": lines,
        "per_config": configs,
    }
    if sweep is not None:
        res["lookup_sweep"] = sweep
    if study is not None:
        res["dispatch_study"] = study
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

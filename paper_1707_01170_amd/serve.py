"""Continuous batching of camera views over a resident LR-spline volume.

Requests (a camera view of any size, with an arrival time) are admitted as
soon as output memory is free in a fixed arena (the memory budget), batched
up to LR_MAX_VIEWS_PER_LAUNCH views per lr_render launch, and launched on
whichever of a few streams has room, so a launch for new arrivals overlaps
launches already on the device.  The volume (forest, element boxes, Bezier
blocks) stays resident.  Completion is taken from device events; latency is
completion minus arrival.  A request's image does not depend on what it was
batched with (rays are independent), so results are identical alone and in
the mix.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .api import Scene, render


class Arena:
    """First-fit allocator over a fixed RGBA pixel arena (the memory budget)."""

    def __init__(self, pixels: int, device):
        self.buf = torch.empty((pixels, 4), dtype=torch.float32, device=device)
        self.free = [(0, pixels)]           # sorted (start, length)

    @property
    def capacity(self) -> int:
        return self.buf.shape[0]

    def alloc(self, n: int) -> Optional[int]:
        for k, (s, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (s + n, ln - n)
                return s
        return None

    def release(self, s: int, n: int):
        self.free.append((s, n))
        self.free.sort()
        merged = []
        for a, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((a, ln))
        self.free = merged


@dataclass
class Served:
    index: int
    arrival_s: float
    pixels: int
    admitted_s: float = -1.0
    launched_s: float = -1.0
    done_ms: float = -1.0              # device completion, ms after the start event
    image: Optional[torch.Tensor] = None

    @property
    def latency_ms(self) -> float:
        return self.done_ms - 1e3 * self.arrival_s


@dataclass
class ServeStats:
    n: int
    wall_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    max_ms: float
    pixels: int
    offered_px_per_s: float
    served_px_per_s: float
    launches: int
    mean_views_per_launch: float
    max_inflight: int
    budget_pixels: int
    results: List[Served] = field(default_factory=list, repr=False)


class Server:
    def __init__(self, scene: Scene, budget_bytes: int = 1 << 30, n_streams: int = 3,
                 max_views: int = L.LR_MAX_VIEWS_PER_LAUNCH, max_pixels_per_launch: int = 1 << 24,
                 schedule: bool = False):
        dev = scene.volume.device
        self.scene = scene
        self.arena = Arena(budget_bytes // 16, dev)
        # streams at the default priority
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
        self.max_views = max_views
        self.max_px = max_pixels_per_launch
        # schedule: launches deal their blocks longest first (lr_render_scheduled), in a
        # workspace per stream (one launch in flight per stream), sized up front for
        # max_views square views of max_pixels_per_launch pixels in all and grown when a
        # launch needs more (lr_render_workspace_size of its views)
        self.workspaces = None
        if schedule:
            from .api import view_array
            side = max(16, int((max_pixels_per_launch // max_views) ** 0.5))
            probe = [_square_view(side) for _ in range(max_views)]
            self.workspaces = [_workspace(_workspace_bytes(view_array(probe)[0], max_views), dev)
                               for _ in range(n_streams)]

    def run(self, requests: Sequence, keep_images: bool = False, time_scale: float = 1.0) -> ServeStats:
        """Serve requests (objects with .arrival_s and .view) in real time.
        time_scale < 1 compresses the arrival times."""
        order = sorted(range(len(requests)), key=lambda k: requests[k].arrival_s)
        recs = [Served(k, requests[k].arrival_s * time_scale, requests[k].view.width * requests[k].view.height)
                for k in range(len(requests))]
        for r in recs:
            if r.pixels > self.arena.capacity:
                raise ValueError("request %d needs %d pixels, more than the budget %d"
                                 % (r.index, r.pixels, self.arena.capacity))
        pending = deque(order)
        arrived = deque()
        ready = deque()            # admitted: (index, offset)
        inflight = []              # (event, stream_idx, [(index, offset)])
        copying = []               # (event, [(index, offset)]): images being copied out
        stream_busy = [0] * len(self.streams)
        dev = self.scene.volume.device
        start = torch.cuda.Event(enable_timing=True)
        start.record(torch.cuda.current_stream(dev))
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        launches = views_launched = max_inflight = 0
        done = 0
        n = len(recs)
        while done < n:
            now = time.perf_counter() - t0
            while pending and recs[pending[0]].arrival_s <= now:
                arrived.append(pending.popleft())
            while arrived:                                     # FIFO admission by memory
                k = arrived[0]
                off = self.arena.alloc(recs[k].pixels)
                if off is None:
                    break
                arrived.popleft()
                recs[k].admitted_s = now
                ready.append((k, off))
            progressed = False
            while ready:
                si = min(range(len(self.streams)), key=lambda i: stream_busy[i])
                if stream_busy[si] >= 1:
                    break
                batch, px = [], 0
                while ready and len(batch) < self.max_views and (not batch or px + recs[ready[0][0]].pixels <= self.max_px):
                    k, off = ready.popleft()
                    batch.append((k, off))
                    px += recs[k].pixels
                views = [requests[k].view for k, _ in batch]
                with torch.cuda.stream(self.streams[si]):
                    arr = _view_array_at(views, [off for _, off in batch])
                    s = self.scene.struct()
                    if self.workspaces is None:
                        L.check(L.lib().lr_render(_byref(s), arr, len(views), _ptr(self.arena.buf), None,
                                                  _stream_handle(self.streams[si])))
                    else:
                        need = _workspace_bytes(arr, len(views))
                        if self.workspaces[si].numel() < need:   # the stream has no launch in flight
                            self.workspaces[si] = _workspace(need, dev)
                        ws = self.workspaces[si]
                        L.check(L.lib().lr_render_scheduled(_byref(s), arr, len(views), _ptr(self.arena.buf), None,
                                                            _ptr(ws), ws.numel(), _stream_handle(self.streams[si])))
                    ev = torch.cuda.Event(enable_timing=True)
                    ev.record(self.streams[si])
                for k, _ in batch:
                    recs[k].launched_s = now
                inflight.append((ev, si, batch))
                stream_busy[si] += 1
                launches += 1
                views_launched += len(batch)
                progressed = True
            max_inflight = max(max_inflight, len(inflight))
            still = []
            for ev, si, batch in inflight:
                if ev.query():
                    t_ms = start.elapsed_time(ev)
                    for k, off in batch:
                        recs[k].done_ms = t_ms
                        done += 1
                    if keep_images:
                        # copy out on the launch's own stream; the regions are
                        # reused only once the copies have completed
                        with torch.cuda.stream(self.streams[si]):
                            for k, off in batch:
                                recs[k].image = self.arena.buf[off:off + recs[k].pixels].clone()
                            copied = torch.cuda.Event()
                            copied.record(self.streams[si])
                        copying.append((copied, batch))
                    else:
                        for k, off in batch:
                            self.arena.release(off, recs[k].pixels)
                    stream_busy[si] -= 1
                    progressed = True
                else:
                    still.append((ev, si, batch))
            inflight = still
            waiting = []
            for copied, batch in copying:
                if copied.query():
                    for k, off in batch:
                        self.arena.release(off, recs[k].pixels)
                    progressed = True
                else:
                    waiting.append((copied, batch))
            copying = waiting
            if not progressed:
                time.sleep(5e-5)
        torch.cuda.synchronize(dev)
        wall = time.perf_counter() - t0
        lat = np.array([r.latency_ms for r in recs])
        px = sum(r.pixels for r in recs)
        span = max(r.arrival_s for r in recs) - min(r.arrival_s for r in recs)
        return ServeStats(n=n, wall_s=wall, p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                          mean_ms=float(lat.mean()), max_ms=float(lat.max()), pixels=px,
                          offered_px_per_s=px / span if span > 0 else float("inf"),
                          served_px_per_s=px / wall, launches=launches,
                          mean_views_per_launch=views_launched / max(1, launches), max_inflight=max_inflight,
                          budget_pixels=self.arena.capacity, results=recs)


def _view_array_at(views, offsets):
    from .api import view_array
    arr, _ = view_array(views, offsets)
    return arr


def _workspace_bytes(arr, n: int) -> int:
    import ctypes
    nb = ctypes.c_int64(0)
    L.check(L.lib().lr_render_workspace_size(arr, n, ctypes.byref(nb)))
    return nb.value


def _workspace(nbytes: int, device) -> torch.Tensor:
    """nbytes of device memory, 256-byte aligned."""
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def _square_view(side: int):
    """A side x side orthographic view along z (only its size matters here)."""
    from types import SimpleNamespace
    return SimpleNamespace(proj="ortho", width=side, height=side, eye=(0.5, 0.5, -1.0), fwd=(0.0, 0.0, 1.0),
                           right=(1.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), tx=0.5, ty=0.5)


def _byref(s):
    import ctypes
    return ctypes.byref(s)


def _ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(st):
    import ctypes
    return ctypes.c_void_p(st.cuda_stream)


def render_alone(scene: Scene, view) -> torch.Tensor:
    """The same request rendered by itself (for comparison)."""
    out, _, _ = render(scene, [view])
    return out

"""Continuous-batching render server over the HIP path (forward only).

Requests (image size, camera, tau) are admitted into slots as they arrive and
as slots free up.  Each slot owns a frame (device workspace), a stream, an
output image per image size and one captured graph per image size
(lod_select + render, replayed with the request's camera and tau), so work of
different requests overlaps on the device and the host only updates the
per-view constants and launches.  The number of slots is set by free HBM at
start-up.  The scene and all per-request state stay on the device.

``baseline_loop`` is the comparison: one request at a time on one stream,
plain launches, FIFO.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from .lodgs import Frame, ViewGraph, camera_struct


@dataclass
class Request:
    rid: int
    arrival: float          # seconds since the start of the run
    cam: object             # scenegen.Camera or a ctypes camera with width/height
    tau: float
    latency: float = float("nan")
    status: int = 0


@dataclass
class _Slot:
    frame: Frame
    stream: torch.cuda.Stream
    graphs: dict
    event: torch.cuda.Event
    req: Request | None = None
    keep: dict = field(default_factory=dict)


def _size(cam):
    return (int(cam.width), int(cam.height))


class RenderServer:
    """Slots of (frame, stream, graphs); see the module docstring."""

    def __init__(self, scene, sizes, max_selected: int, max_instances: int, max_slots: int = 8,
                 hbm_fraction: float = 0.5, tau0: float = 1.0, cull: bool = True, template_cam=None):
        self.scene = scene
        self.sizes = [tuple(s) for s in sizes]
        wmax = max(w for w, _ in self.sizes)
        hmax = max(h for _, h in self.sizes)
        free, _ = torch.cuda.mem_get_info()
        per_slot = self.slot_bytes(max_selected, max_instances, self.sizes)
        n = int(min(max_slots, max(1, (free * hbm_fraction) // per_slot)))
        self.slot_bytes_estimate = per_slot
        self.slots = []
        for _ in range(n):
            f = Frame(scene, max_selected, max_instances, wmax, hmax)
            st = torch.cuda.Stream()
            graphs = {}
            for w, h in self.sizes:
                cam = template_cam(w, h)
                with torch.cuda.stream(st):
                    graphs[(w, h)] = ViewGraph(f, cam, tau0, st, cull=cull)
            st.synchronize()
            self.slots.append(_Slot(f, st, graphs, torch.cuda.Event()))

    @staticmethod
    def slot_bytes(max_selected, max_instances, sizes):
        """Device bytes of one slot: frame workspace plus one image per size."""
        per_sel = 64 + 4 * 7 + 8 + 36 + 4
        per_inst = 16
        tiles = max(((w + 15) // 16) * ((h + 15) // 16) for w, h in sizes)
        return max_selected * per_sel + max_instances * per_inst + tiles * 8 + sum(w * h * 12 for w, h in sizes)

    def run(self, requests, keep_images: bool = False, poll_sleep: float = 0.0):
        """Serves the requests by arrival time (open loop); returns them with
        latency filled in (completion - arrival, seconds)."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        free = deque(self.slots)
        busy = []
        cams = {r.rid: camera_struct(r.cam) for r in requests}
        images = {}
        t0 = time.perf_counter()
        n_done = 0
        total = len(requests)
        while n_done < total:
            now = time.perf_counter() - t0
            while pending and free and pending[0].arrival <= now:
                r = pending.popleft()
                s = free.popleft()
                s.req = r
                g = s.graphs[_size(r.cam)]
                g.launch(cams[r.rid], r.tau, s.stream)
                if keep_images:
                    with torch.cuda.stream(s.stream):
                        s.keep[r.rid] = g.out.clone()
                s.event.record(s.stream)
                busy.append(s)
            progressed = False
            for s in list(busy):
                if s.event.query():
                    t_done = time.perf_counter() - t0
                    r = s.req
                    r.latency = t_done - r.arrival
                    st = s.frame.stats(stream=s.stream)
                    r.status = st["status"]
                    if st["status"] != 0:
                        s.frame.clear_status(stream=s.stream)
                    if keep_images:
                        images[r.rid] = s.keep.pop(r.rid)
                    s.req = None
                    busy.remove(s)
                    free.append(s)
                    n_done += 1
                    progressed = True
            if not progressed and poll_sleep > 0 and not (pending and free and pending[0].arrival <= now):
                time.sleep(poll_sleep)
        makespan = time.perf_counter() - t0
        return requests, makespan, images


def baseline_loop(frame: Frame, requests, keep_images: bool = False, stream=None):
    """One request at a time, plain launches on one stream, FIFO, open loop."""
    st = stream or torch.cuda.current_stream()
    reqs = sorted(requests, key=lambda r: r.arrival)
    cams = {r.rid: camera_struct(r.cam) for r in requests}
    outs = {}
    images = {}
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            pass
        size = _size(r.cam)
        if size not in outs:
            outs[size] = torch.empty((size[1], size[0], 3), dtype=torch.float32, device=frame.scene.device)
        with torch.cuda.stream(st):
            frame.lod_select(cams[r.rid], r.tau, stream=st)
            img = frame.render(cams[r.rid], out=outs[size], stream=st)
            if keep_images:
                images[r.rid] = img.clone()
        st.synchronize()
        r.latency = time.perf_counter() - t0 - r.arrival
        stt = frame.stats(stream=st)
        r.status = stt["status"]
        if stt["status"] != 0:
            frame.clear_status(stream=st)
    makespan = time.perf_counter() - t0
    return reqs, makespan, images


def summarize(requests, makespan, warmup: int = 0):
    reqs = sorted(requests, key=lambda r: r.arrival)[warmup:]
    lat = np.array([r.latency for r in reqs]) * 1000.0
    span = max(r.arrival + r.latency for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
            "throughput_rps": round(len(reqs) / span, 1) if span > 0 else None,
            "overflows": int(sum(1 for r in reqs if r.status != 0))}


def poisson_requests(rng, lam: float, n: int, make_cam, taus=(0.5, 1.0, 2.0), start_id: int = 0):
    """Open-loop Poisson arrivals at rate lam (req/s) with cameras from make_cam(rng)."""
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / lam)
        out.append(Request(start_id + k, t, make_cam(rng), float(taus[rng.integers(len(taus))])))
    return out

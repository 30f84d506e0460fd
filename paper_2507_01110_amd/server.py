"""Continuous-batching render server over the HIP path (forward only).

``RenderServer`` is a thin caller of the library's server
(lodgs_server_create / submit / poll): requests (image size, camera, tau) are
queued as they arrive and admitted into slots as slots and free HBM allow;
each slot replays a captured view graph on its own stream, so the work of
different requests overlaps on the device.  A request that overflows its
slot's capacities is re-served on a larger slot by the library; one that no
slot can take is rejected (status LODGS_E_CAPACITY) and reported apart from
the served ones.

``baseline_loop`` is the comparison: one request at a time on one stream,
plain launches, FIFO, growing its frame and re-running a request that
overflowed.
"""
from __future__ import annotations

import ctypes
import time
from collections import defaultdict, deque
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check
from .lodgs import Frame, _ptr, camera_struct


@dataclass
class Request:
    rid: int
    arrival: float          # seconds since the start of the run
    cam: object             # scenegen.Camera or a ctypes camera with width/height
    tau: float
    latency: float = float("nan")
    status: int = 0
    attempts: int = 0


def _size(cam):
    return (int(cam.width), int(cam.height))


class RenderServer:
    """The library's slot server; see the module docstring."""

    def __init__(self, scene, sizes, max_selected: int, max_instances: int, max_slots: int = 8,
                 hbm_reserve: int = 16 << 30, cull: bool = True, bg=(0.0, 0.0, 0.0)):
        self.scene = scene
        self.sizes = [tuple(int(x) for x in s) for s in sizes]
        if not 1 <= len(self.sizes) <= _lib.SERVER_MAX_SIZES:
            raise ValueError("1 to %d image sizes" % _lib.SERVER_MAX_SIZES)
        caps = _lib.ServerCaps()
        caps.n_sizes = len(self.sizes)
        for k, (w, h) in enumerate(self.sizes):
            caps.sizes[k][0], caps.sizes[k][1] = w, h
        caps.max_slots = int(max_slots)
        caps.max_selected, caps.max_instances = int(max_selected), int(max_instances)
        caps.hbm_reserve = int(hbm_reserve)
        caps.flags = _lib.CULL if cull else 0
        for k in range(3):
            caps.bg[k] = float(bg[k])
        h = ctypes.c_void_p()
        check(_lib.load().lodgs_server_create(scene._h, ctypes.byref(caps), ctypes.byref(h)), "lodgs_server_create")
        self._h = h
        self._done = (_lib.Completion * 64)()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.lodgs_server_destroy(h)
            self._h = None

    def submit(self, cam, tau: float, out, user: int = 0) -> int:
        """Queues one request writing its image to `out` (device [H, W, 3]
        float32, kept alive by the caller until it completes); returns its
        ticket."""
        r = _lib.Request(camera_struct(cam), float(tau), _ptr(out), int(user))
        t = ctypes.c_uint64()
        check(_lib.load().lodgs_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "lodgs_server_submit")
        return t.value

    def poll(self):
        """Completions since the last poll (non-blocking)."""
        out = []
        n = ctypes.c_int32()
        while True:
            check(_lib.load().lodgs_server_poll(self._h, self._done, len(self._done), ctypes.byref(n)),
                  "lodgs_server_poll")
            out.extend(self._done[k] for k in range(n.value))
            if n.value < len(self._done):
                return [(c.ticket, c.user, c.status, c.attempts, c.t_done, c.n_selected, c.n_instances) for c in out]

    def stats(self) -> dict:
        s = _lib.ServerStats()
        check(_lib.load().lodgs_server_stats_read(self._h, ctypes.byref(s)), "lodgs_server_stats_read")
        return s.as_dict()

    def run(self, requests, keep_images: bool = False):
        """Serves the requests by arrival time (open loop); returns them with
        latency (completion seen by a poll - arrival, seconds), status and
        attempts filled in, the makespan and, with keep_images, the image of
        every served request."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        by_id = {r.rid: r for r in requests}
        pool = defaultdict(list)  # free output images per size
        busy = {}
        images = {}
        dev = self.scene.device
        t0 = time.perf_counter()
        n_done, total = 0, len(requests)
        while n_done < total:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                w, h = _size(r.cam)
                out = pool[(w, h)].pop() if (pool[(w, h)] and not keep_images) else \
                    torch.empty((h, w, 3), dtype=torch.float32, device=dev)
                busy[r.rid] = out
                self.submit(r.cam, r.tau, out, user=r.rid)
            for _, user, status, attempts, t_done, _, _ in self.poll():
                r = by_id[user]
                r.latency = t_done - t0 - r.arrival
                r.status, r.attempts = status, attempts
                out = busy.pop(user)
                if keep_images:
                    images[user] = out
                else:
                    pool[_size(r.cam)].append(out)
                n_done += 1
        makespan = time.perf_counter() - t0
        return requests, makespan, images


def baseline_loop(frame: Frame, requests, keep_images: bool = False, stream=None):
    """One request at a time, plain launches on one stream, FIFO, open loop.
    A request that overflows the frame's capacities runs again on a frame
    grown to the counts it reported.  Returns (requests, makespan, images,
    frame) with the last frame used."""
    st = stream or torch.cuda.current_stream()
    reqs = sorted(requests, key=lambda r: r.arrival)
    cams = {r.rid: camera_struct(r.cam) for r in requests}
    outs = {}
    images = {}
    c_scene = frame.scene
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            pass
        size = _size(r.cam)
        if size not in outs:
            outs[size] = torch.empty((size[1], size[0], 3), dtype=torch.float32, device=frame.scene.device)
        r.attempts = 0
        while True:
            r.attempts += 1
            with torch.cuda.stream(st):
                frame.lod_select(cams[r.rid], r.tau, stream=st)
                img = frame.render(cams[r.rid], out=outs[size], stream=st)
            stt = frame.stats(stream=st)  # synchronises the stream
            r.status = stt["status"]
            if r.status == 0:
                break
            frame.clear_status(stream=st)
            if r.attempts >= 6:
                break
            c = frame.caps
            sel = max(c.max_selected, stt["n_selected"] + stt["n_selected"] // 4 + 1024)
            inst = max(c.max_instances, stt["n_instances"] + stt["n_instances"] // 4 + 1024)
            del frame, img
            frame = Frame(c_scene, sel, inst, c.max_width, c.max_height)
        if keep_images and r.status == 0:
            images[r.rid] = img.clone()
        st.synchronize()
        r.latency = time.perf_counter() - t0 - r.arrival
    makespan = time.perf_counter() - t0
    return reqs, makespan, images, frame


def summarize(requests, makespan, warmup: int = 0):
    """p50 / p99 / mean latency and throughput over the served requests after
    the warm-up ones; rejected requests are counted apart and left out."""
    reqs = sorted(requests, key=lambda r: r.arrival)[warmup:]
    ok = [r for r in reqs if r.status == 0]
    lat = np.array([r.latency for r in ok]) * 1000.0
    span = (max(r.arrival + r.latency for r in ok) - min(r.arrival for r in reqs)) if ok else 0.0
    return {"requests": len(reqs), "served": len(ok), "rejected": len(reqs) - len(ok),
            "retried": int(sum(1 for r in ok if r.attempts > 1)),
            "p50_ms": round(float(np.percentile(lat, 50)), 3) if ok else None,
            "p99_ms": round(float(np.percentile(lat, 99)), 3) if ok else None,
            "mean_ms": round(float(lat.mean()), 3) if ok else None,
            "throughput_rps": round(len(ok) / span, 1) if span > 0 else None}


def poisson_requests(rng, lam: float, n: int, make_cam, taus=(0.5, 1.0, 2.0), start_id: int = 0):
    """Open-loop Poisson arrivals at rate lam (req/s) with cameras from make_cam(rng)."""
    t = 0.0
    out = []
    for k in range(n):
        t += rng.exponential(1.0 / lam)
        out.append(Request(start_id + k, t, make_cam(rng), float(taus[rng.integers(len(taus))])))
    return out

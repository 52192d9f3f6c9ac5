"""Continuous-batching relight server over the gs3 library.

Requests (camera view, point light, resolution) arrive over time; the scene
stays resident in device memory. A request is admitted as soon as it has
arrived and a buffer set for its resolution is free, or can be allocated
without exceeding the memory cap; its whole pipeline (light preprocess,
shadow splat, camera preprocess, shading + MLPs + camera splat) is enqueued
on its own HIP stream, so requests that arrive while others are on the GPU
run alongside them and the device overlaps their kernels. Completion is
detected with events, without blocking the host; a finished request frees
its buffer set for the next one. The plain baseline runs the same library
calls one request at a time, first come first served, and waits for each.

With ``share_lights`` the server also shares shadow splats: requests whose
light view is the same (position, target, resolution, field of view) reuse
one shadow pass (light preprocess, shadow splat, per-Gaussian T; Sec. 4.2
computes T per light, independent of the camera). The first such request
runs it and keeps a copy of T; later ones wait for that copy on the device
(a stream wait on its event) and run only their camera path. Copies are
kept for the most recently used lights, within the memory cap.

With ``batch`` > 1 the server launches requests in batches: the requests
waiting when the device has room (up to ``batch`` of them, mixed
resolutions) run as one launch sequence per stage over all their views
(``gs3.render_batched``: one projection + binning launch sequence for every
light and camera view, one shadow-splat sequence, one shading + camera-splat
sequence), on one stream; several batches can be in flight together. A light
seen twice in a batch gets one shadow pass.

Latency of a request = completion time - arrival time (queueing included).
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import OrderedDict, deque
from typing import Dict, List, Optional

import numpy as np
import torch

from . import gs3, synth


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    cam: synth.View
    light: synth.View


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    start: float
    done: float
    final: Optional[torch.Tensor] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_requests(count: int, qps: float, seed: int = 3, resolutions=(256, 512, 800, 1024),
                  light_res: int = 1024, fov: float = 40.0, radius: float = 4.0,
                  n_lights: Optional[int] = None) -> List[Request]:
    """Poisson arrivals at rate qps; camera and light uniform on the sphere
    of the given radius; camera resolution uniform over `resolutions`. With
    `n_lights`, each request's light is drawn from a fixed set of that many
    lights (a light stage's set of point lights) instead."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, count) if qps > 0 else np.zeros(count)
    t = np.cumsum(gaps) - gaps[0]
    light_set = None
    if n_lights:
        lrng = np.random.default_rng(seed + 1000)
        light_set = [synth.make_view(lrng.standard_normal(3), radius, light_res, light_res, fov)
                     for _ in range(n_lights)]
    out = []
    for i in range(count):
        r = int(resolutions[rng.integers(0, len(resolutions))])
        cam = synth.make_view(rng.standard_normal(3), radius, r, r, fov)
        d = rng.standard_normal(3)
        if light_set is not None:
            light = light_set[int(rng.integers(0, n_lights))]
        else:
            light = synth.make_view(d, radius, light_res, light_res, fov)
        out.append(Request(i, float(t[i]), cam, light))
    return out


def _ws_bytes(n: int, w: int, h: int, capacity: int) -> int:
    import ctypes as C
    size = C.c_size_t()
    gs3._check(gs3._lib.gs3_view_workspace_size(n, w, h, capacity, C.byref(size)), "gs3_view_workspace_size")
    return size.value + 256


class BufferSet:
    """Everything one in-flight request needs: a Renderer (view buffers, T,
    num/den, images) bound to one camera resolution, and its own stream."""

    def __init__(self, scene: gs3.DeviceScene, consts, res: int, light_res: int, capacity: int):
        self.res = res
        self.stream = torch.cuda.Stream()
        self.renderer = gs3.Renderer(scene, consts, pair_capacity=capacity)
        self.event = torch.cuda.Event()
        with torch.cuda.stream(self.stream):
            # allocate the buffers now, so admission accounting is exact
            self.renderer._vb("light", light_res, light_res, capacity)
            self.renderer._vb("cam", res, res, capacity)
            self.renderer._images(res, res)
        self.bytes = self.measure()

    def measure(self) -> int:
        """Device bytes this set holds now (view workspaces, images, shadow
        state)."""
        r = self.renderer
        return sum(vb.storage.numel() for vb in r.vbs.values()) + \
            sum(t.numel() * t.element_size() for im in r.images.values() for t in im.values()) + \
            (r.num_den.numel() + r.T.numel()) * 4

    @staticmethod
    def estimate(n: int, res: int, light_res: int, capacity: int) -> int:
        """Device bytes a new set for camera resolution `res` will hold."""
        images = 12 * res * res * 4 + 8 * max(n, 1) * 4
        return _ws_bytes(n, light_res, light_res, capacity) + _ws_bytes(n, res, res, capacity) + images + \
            3 * max(n, 1) * 4


@dataclasses.dataclass
class LightEntry:
    """A shared shadow pass: T of one light view, valid once `event` has
    completed on the device."""
    T: torch.Tensor
    event: torch.cuda.Event


def light_key(light: synth.View) -> tuple:
    return (tuple(float(x) for x in light.eye), tuple(float(x) for x in light.target), light.width,
            light.height, float(light.fov))


class Server:
    """Admission by a memory cap over per-resolution pools of buffer sets."""

    def __init__(self, scene: gs3.DeviceScene, mem_cap_bytes: int, consts=None, light_res: int = 1024,
                 capacity: Optional[int] = None, max_inflight: int = 8, overlap="auto",
                 share_lights: bool = False, max_lights: int = 256, batch: int = 1):
        self.scene = scene
        self.consts = consts if consts is not None else gs3.default_consts()
        self.cap = int(mem_cap_bytes)
        self.light_res = light_res
        self.capacity = capacity or max(1 << 16, 32 * scene.n)
        self.max_inflight = max_inflight
        # overlap the stages inside a request too: True, False, or "auto" (only
        # when it is admitted with fewer than two requests in flight: alone it
        # finishes sooner, while several requests already fill the device)
        self.overlap = overlap
        self.free: Dict[int, List[BufferSet]] = {}
        self.allocated = 0
        self.sets: List[BufferSet] = []
        self.share_lights = share_lights
        self.max_lights = max_lights
        self.lights: "OrderedDict[tuple, LightEntry]" = OrderedDict()
        self.light_passes = 0          # shadow passes run (not shared)
        self.batch = max(1, int(batch))
        self.batches = 0               # batched launches issued

    def _acquire(self, res: int) -> Optional[BufferSet]:
        pool = self.free.setdefault(res, [])
        if pool:
            return pool.pop()
        # size the new set before allocating it (the first set is always
        # allowed, so that every request can be served)
        probe = BufferSet.estimate(self.scene.n, res, self.light_res, self.capacity)
        if self.sets and self.allocated + probe > self.cap:
            # reclaim idle sets of other resolutions until the new one fits
            idle = [bs for p in self.free.values() for bs in p]
            if sum(bs.bytes for bs in idle) < self.allocated + probe - self.cap:
                return None          # not enough even then: wait for a request to finish
            for p in self.free.values():
                while p and self.allocated + probe > self.cap:
                    bs = p.pop()
                    self.allocated -= bs.bytes
                    self.sets.remove(bs)
                    del bs
            if self.allocated + probe > self.cap:
                return None
        bs = BufferSet(self.scene, self.consts, res, self.light_res, self.capacity)
        self.allocated += bs.bytes
        self.sets.append(bs)
        return bs

    def _launch(self, req: Request, bs: BufferSet, keep: bool, n_inflight: int = 0):
        overlap = (n_inflight < 2) if self.overlap == "auto" else bool(self.overlap)
        key = light_key(req.light) if self.share_lights else None
        entry = self.lights.get(key) if key is not None else None
        with torch.cuda.stream(bs.stream):
            if entry is not None:
                # the light's shadow values exist (or are being computed):
                # wait for them on the device, run only the camera path
                self.lights.move_to_end(key)
                bs.stream.wait_event(entry.event)
                entry.T.record_stream(bs.stream)     # not reused while this stream reads it
                out = bs.renderer.render_shadowed(req.cam, req.light, entry.T, check=False)
            else:
                out = bs.renderer.render(req.cam, req.light, check=False, overlap=overlap)
                self.light_passes += 1
                if key is not None:
                    self._keep_light(key, out["T"], bs.stream)
            final = out["final"].clone() if keep else None
            bs.event.record(bs.stream)
        return final

    def _launch_batch(self, reqs: List[Request], sets: List[BufferSet], keep: bool, n_inflight: int = 0) -> list:
        """Requests `reqs` with buffer sets `sets` as one batch on the first
        set's stream (its event marks the batch done). Returns the finals. A
        batch of one request runs the one-request path, whose frame overlaps
        its own stages when the device is otherwise idle."""
        if len(reqs) == 1:
            final = self._launch(reqs[0], sets[0], keep, n_inflight)
            self.batches += 1
            return [final]
        stream = sets[0].stream
        shadows = [None] * len(reqs)
        keys = [light_key(r.light) for r in reqs]
        with torch.cuda.stream(stream):
            if self.share_lights:
                for i, k in enumerate(keys):
                    entry = self.lights.get(k)
                    if entry is not None:
                        self.lights.move_to_end(k)
                        stream.wait_event(entry.event)
                        entry.T.record_stream(stream)
                        shadows[i] = entry.T
            outs = gs3.render_batched([bs.renderer for bs in sets], [r.cam for r in reqs],
                                      [r.light for r in reqs], shadows)
            fresh = {}
            for i, k in enumerate(keys):
                if shadows[i] is None and k not in fresh:
                    fresh[k] = outs[i]["T"]
            self.light_passes += len(fresh)
            if self.share_lights:
                for k, T in fresh.items():
                    self._keep_light(k, T, stream)
            finals = [o["final"].clone() if keep else None for o in outs]
            sets[0].event.record(stream)
        self.batches += 1
        return finals

    def _keep_light(self, key, T: torch.Tensor, stream):
        """Keep a copy of a light's shadow values for later requests (LRU;
        the oldest copies go when the count or the memory cap is reached)."""
        nbytes = T.numel() * T.element_size()
        while self.lights and (len(self.lights) >= self.max_lights or self.allocated + nbytes > self.cap):
            _, old = self.lights.popitem(last=False)
            self.allocated -= old.T.numel() * old.T.element_size()
        if self.allocated + nbytes > self.cap:
            return
        ev = torch.cuda.Event()
        copy = T.clone()           # on `stream`, after the shadow splat that wrote T
        ev.record(stream)
        self.lights[key] = LightEntry(copy, ev)
        self.allocated += nbytes

    def _check_done(self, bs: BufferSet, req: Request, keep: bool) -> Optional[torch.Tensor]:
        """After completion: a binning that overflowed its pair capacity is
        rerun with a larger buffer (rare; synchronous)."""
        with torch.cuda.stream(bs.stream):
            # the request's own stream has finished, so the views' status
            # blocks are final and this read waits for nothing
            if not bs.renderer.overflowed():
                return None
            out = bs.renderer.render(req.cam, req.light, check=True)
            final = out["final"].clone() if keep else None
        bs.stream.synchronize()
        # the rerun may have grown the view buffers: keep the accounting exact
        grown = bs.measure()
        self.allocated += grown - bs.bytes
        bs.bytes = grown
        return final

    def run(self, requests: List[Request], keep_results: bool = False) -> List[Result]:
        """Serve `requests` (sorted by arrival) in real time; returns one
        Result per request in request order."""
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        waiting: deque = deque()
        inflight: List[tuple] = []
        results: Dict[int, Result] = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            progressed = False
            # completions (a batch's requests complete with its first set's event)
            still = []
            for req, bs, start, final, ev in inflight:
                if ev.query():
                    redo = self._check_done(bs, req, keep_results)
                    done = time.perf_counter() - t0
                    results[req.rid] = Result(req.rid, req.arrival, start, done,
                                              redo if redo is not None else final)
                    self.free.setdefault(bs.res, []).append(bs)
                    progressed = True
                else:
                    still.append((req, bs, start, final, ev))
            inflight = still
            # admissions (first come first served; a request that cannot get
            # memory waits, and so do the ones behind it)
            if self.batch > 1:
                reqs, sets = [], []
                while waiting and len(inflight) + len(reqs) < self.max_inflight and len(reqs) < self.batch:
                    bs = self._acquire(waiting[0].cam.width)
                    if bs is None:
                        break
                    reqs.append(waiting.popleft())
                    sets.append(bs)
                if reqs:
                    start = time.perf_counter() - t0
                    finals = self._launch_batch(reqs, sets, keep_results, len(inflight))
                    for req, bs, final in zip(reqs, sets, finals):
                        inflight.append((req, bs, start, final, sets[0].event))
                    progressed = True
            while self.batch == 1 and waiting and len(inflight) < self.max_inflight:
                req = waiting[0]
                bs = self._acquire(req.cam.width)
                if bs is None:
                    break
                waiting.popleft()
                start = time.perf_counter() - t0
                final = self._launch(req, bs, keep_results, len(inflight))
                inflight.append((req, bs, start, final, bs.event))
                progressed = True
            if not progressed:
                if inflight:
                    # poll again at once: a sleep would add its granularity
                    # (tens of microseconds) to every completion
                    pass
                elif pending:
                    time.sleep(max(0.0, min(1e-3, pending[0].arrival - (time.perf_counter() - t0))))
        return [results[r.rid] for r in requests]


def run_plain(scene: gs3.DeviceScene, requests: List[Request], consts=None, light_res: int = 1024,
              capacity: Optional[int] = None, keep_results: bool = False, overlap: bool = True) -> List[Result]:
    """One request at a time, first come first served; the host waits for
    each frame before starting the next. Each frame uses the renderer's own
    stage overlap (``overlap``)."""
    consts = consts if consts is not None else gs3.default_consts()
    cap = capacity or max(1 << 16, 32 * scene.n)
    rnd = gs3.Renderer(scene, consts, pair_capacity=cap)
    out: Dict[int, Result] = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for req in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        start = time.perf_counter() - t0
        o = rnd.render(req.cam, req.light, check=False, overlap=overlap)
        final = o["final"].clone() if keep_results else None
        torch.cuda.synchronize()
        if rnd.overflowed():
            o = rnd.render(req.cam, req.light, check=True)
            final = o["final"].clone() if keep_results else None
            torch.cuda.current_stream().synchronize()
        out[req.rid] = Result(req.rid, req.arrival, start, time.perf_counter() - t0, final)
    return [out[r.rid] for r in requests]


def summarize(results: List[Result]) -> Dict[str, float]:
    lat = np.array([r.latency for r in results]) * 1e3
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "frames_per_s": len(results) / span if span > 0 else math.inf,
            "requests": len(results)}

"""Serving several robots' frame streams on one GPU with continuous batching.

Each robot owns a device-resident voxel map.  Frames arrive over time; a
frame is admitted as soon as (a) it has arrived, (b) its robot has a free
in-flight slot (frames of one robot run in arrival order, on the robot's own
stream), (c) a result slot is free and (d) the HBM budget for in-flight
frames can hold its points.  Admitted frames are enqueued immediately, so
frames of different robots run concurrently on the device while later ones
keep arriving; a finished frame frees its slot and budget, and the next
waiting frame is admitted.  Latency is arrival -> results in host memory.

A frame's results depend only on its robot's map and frame sequence (the
RANSAC frame counter is the robot's own frame number), so they are the same
alone and in the mix.

The scheduler (`Scheduler`) is independent of the device: `GpuBackend` drives
the C ABI with torch streams and events; tests can drive the same scheduler
with a simulated backend.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    robot: int
    seq: int                 # the robot's own frame number (RANSAC counter word)
    arrival: float           # seconds on the scheduler clock
    n_points: int
    payload: object = None   # backend-specific (e.g. pinned host points + pose)


@dataclasses.dataclass
class Completion:
    request: Request
    admitted: float
    finished: float
    result: object = None

    @property
    def latency(self) -> float:
        return self.finished - self.request.arrival


class Backend:
    """What the scheduler needs from the device side."""

    def bytes_for(self, req: Request) -> int:
        raise NotImplementedError

    def submit(self, req: Request, slot: int):
        """Enqueue the frame; returns a handle polled with done()."""
        raise NotImplementedError

    def done(self, handle) -> bool:
        raise NotImplementedError

    def result(self, handle, slot: int):
        return None


class Scheduler:
    """Continuous batching over robots with per-robot order, result slots and
    an HBM budget for in-flight frames."""

    def __init__(self, backend: Backend, n_robots: int, n_slots: int, budget_bytes: int,
                 per_robot_inflight: int = 2, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        if n_slots < 1 or per_robot_inflight < 1 or budget_bytes <= 0:
            raise ValueError("need at least one slot, one in-flight frame per robot and a positive budget")
        self.backend = backend
        self.n_robots = n_robots
        self.budget = int(budget_bytes)
        self.per_robot = per_robot_inflight
        self.free_slots = list(range(n_slots))[::-1]
        self.clock = clock
        self.sleep = sleep
        self.used = 0
        self.peak_used = 0
        self.peak_inflight = 0
        self.rejected: List[Request] = []

    def run(self, requests: Sequence[Request], t0: Optional[float] = None, idle_sleep: float = 50e-6,
            on_complete: Optional[Callable[[Completion], None]] = None) -> List[Completion]:
        """Serve `requests` (arrival times relative to t0) until all are done.
        Requests too large for the whole budget are rejected (listed in
        self.rejected) instead of blocking the queue forever."""
        t0 = self.clock() if t0 is None else t0
        pending = sorted(requests, key=lambda r: (r.arrival, r.robot, r.seq))
        waiting: Dict[int, List[Request]] = {r: [] for r in range(self.n_robots)}
        inflight = []                      # (handle, slot, req, admitted, bytes)
        per_robot = [0] * self.n_robots
        out: List[Completion] = []
        i = 0
        total = len(pending)
        while len(out) + len(self.rejected) < total:
            now = self.clock() - t0
            while i < total and pending[i].arrival <= now:
                waiting[pending[i].robot].append(pending[i])
                i += 1
            # completions free slots and budget
            still = []
            for h, slot, req, adm, nb in inflight:
                if self.backend.done(h):
                    fin = self.clock() - t0
                    c = Completion(req, adm, fin, self.backend.result(h, slot))
                    out.append(c)
                    if on_complete:
                        on_complete(c)
                    self.free_slots.append(slot)
                    self.used -= nb
                    per_robot[req.robot] -= 1
                else:
                    still.append((h, slot, req, adm, nb))
            inflight = still
            # admit: oldest arrivals first, across robots
            progressed = True
            while progressed:
                progressed = False
                cands = [(q[0].arrival, r) for r, q in waiting.items() if q]
                for _, r in sorted(cands):
                    q = waiting[r]
                    req = q[0]
                    nb = self.backend.bytes_for(req)
                    if nb > self.budget:
                        self.rejected.append(q.pop(0))
                        progressed = True
                        break
                    if per_robot[r] >= self.per_robot or not self.free_slots or self.used + nb > self.budget:
                        continue
                    q.pop(0)
                    slot = self.free_slots.pop()
                    self.used += nb
                    self.peak_used = max(self.peak_used, self.used)
                    per_robot[r] += 1
                    h = self.backend.submit(req, slot)
                    inflight.append((h, slot, req, self.clock() - t0, nb))
                    self.peak_inflight = max(self.peak_inflight, len(inflight))
                    progressed = True
                    break
            if not inflight and i < total and not any(waiting.values()):
                # nothing to do until the next arrival
                wait = pending[i].arrival - (self.clock() - t0)
                if wait > 0:
                    self.sleep(min(wait, 1e-3))
            elif idle_sleep:
                self.sleep(idle_sleep)
        return out


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process (exponential gaps) in [0, duration)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            return np.array(out)
        out.append(t)


def latency_summary(done: Sequence[Completion], t_span: Optional[float] = None) -> dict:
    lat = np.array([c.latency for c in done]) * 1e3
    s = {"frames": len(done), "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
         "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
         "max_ms": float(lat.max()) if len(lat) else None}
    if t_span:
        s["frames_per_s"] = len(done) / t_span
    return s


class GpuBackend(Backend):
    """Frames through vm_segment_frame on one stream per robot.

    payload of a Request: (pinned host float32 [N,3] tensor, R, t).  Each
    result slot owns its plane/hull output buffers and pinned host copies of
    the per-cluster results; the D2H copies are enqueued behind the frame, so a
    completed frame's results are already in host memory."""

    def __init__(self, maps, n_slots: int, n_hyp: int, min_cluster: int = 30, eps: float = 0.01,
                 seed: int = 0x5EED, k_cap: int = 8192, in_cap: int = 1 << 23, v_cap: int = 1 << 21):
        import torch

        import paper_2510_01592_amd as vm
        self.vm = vm
        self.torch = torch
        self.maps = maps
        self.streams = [torch.cuda.Stream() for _ in maps]
        self.kw = dict(min_cluster=min_cluster, n_hyp=n_hyp, eps=eps, seed=seed)
        self.k_cap = k_cap
        self.planes = [vm.PlaneBuffers.alloc(k_cap, in_cap, n_hyp) for _ in range(n_slots)]
        self.hulls = [vm.HullBuffers.alloc(k_cap, v_cap) for _ in range(n_slots)]
        self.host = [dict(plane=torch.empty((k_cap, 4), dtype=torch.float32).pin_memory(),
                          best=torch.empty(k_cap, dtype=torch.int32).pin_memory(),
                          area=torch.empty(k_cap, dtype=torch.float64).pin_memory(),
                          v_off=torch.empty(k_cap + 1, dtype=torch.int32).pin_memory(),
                          meta=torch.empty(2, dtype=torch.int32).pin_memory(),
                          status=torch.empty(2, dtype=torch.int32).pin_memory(),
                          stats=torch.empty(6, dtype=torch.int64).pin_memory())
                     for _ in range(n_slots)]
        self.stats_dev = [torch.empty(6, dtype=torch.int64, device="cuda") for _ in range(n_slots)]

    def bytes_for(self, req: Request) -> int:
        return 12 * int(req.n_points)

    def submit(self, req: Request, slot: int):
        torch, vm = self.torch, self.vm
        pts, R, t = req.payload
        s = self.streams[req.robot]
        with torch.cuda.stream(s):
            d = torch.empty((req.n_points, 3), dtype=torch.float32, device="cuda")
            d.copy_(pts, non_blocking=True)
            pb, hb, h = self.planes[slot], self.hulls[slot], self.host[slot]
            cl = self.maps[req.robot].segment_frame(d, pb, hb, R=R, t=t, frame=req.seq, stream=s, **self.kw)
            h["plane"].copy_(pb.plane, non_blocking=True)
            h["best"].copy_(pb.best_h, non_blocking=True)
            h["area"].copy_(hb.area, non_blocking=True)
            h["v_off"].copy_(hb.v_off, non_blocking=True)
            h["meta"].copy_(vm.device_view(cl.d_meta, 2, np.int32), non_blocking=True)
            h["status"][0:1].copy_(pb.status, non_blocking=True)
            h["status"][1:2].copy_(hb.status, non_blocking=True)
            self.maps[req.robot].stats_async(self.stats_dev[slot], stream=s)
            h["stats"].copy_(self.stats_dev[slot], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
            d.record_stream(s)
        return ev

    def done(self, handle) -> bool:
        return handle.query()

    def result(self, handle, slot: int):
        h = self.host[slot]
        K = min(int(h["meta"][0]), self.k_cap)
        return dict(K=int(h["meta"][0]), plane=h["plane"][:K].numpy().copy(), best=h["best"][:K].numpy().copy(),
                    area=h["area"][:K].numpy().copy(), v_off=h["v_off"][:K + 1].numpy().copy(),
                    status=h["status"].numpy().copy(), occupied=int(h["stats"][0]))

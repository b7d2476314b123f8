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
    """What the scheduler needs from the device side.  A backend that sets
    ``batching`` receives every admission round's frames together through
    submit_batch (at most one frame per robot per round)."""

    batching = False

    def bytes_for(self, req: Request) -> int:
        raise NotImplementedError

    def submit(self, req: Request, slot: int):
        """Enqueue the frame; returns a handle polled with done()."""
        raise NotImplementedError

    def submit_batch(self, items):
        """Enqueue frames [(req, slot)] as one batch; returns one handle per item."""
        return [self.submit(req, slot) for req, slot in items]

    def done(self, handle) -> bool:
        raise NotImplementedError

    def result(self, handle, slot: int):
        return None


class Scheduler:
    """Continuous batching over robots with per-robot order, result slots and
    an HBM budget for in-flight frames."""

    def __init__(self, backend: Backend, n_robots: int, n_slots: int, budget_bytes: int,
                 per_robot_inflight: int = 2, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, max_batches_inflight: int = 2):
        """max_batches_inflight: with a batching backend, frames that arrive
        while this many batches run wait and join the next batch together."""
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
        self.max_batches = max(1, int(max_batches_inflight))
        self.batches = 0
        self.batched_frames = 0

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
            # admit: oldest arrivals first, across robots; a batching backend
            # gets the round's frames together (one per robot)
            batching = getattr(self.backend, "batching", False)
            batch = []
            progressed = not batching or len({id(h[0]) for h in inflight}) < self.max_batches
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
                    if batching and any(b[0].robot == r for b in batch):
                        continue
                    q.pop(0)
                    slot = self.free_slots.pop()
                    self.used += nb
                    self.peak_used = max(self.peak_used, self.used)
                    per_robot[r] += 1
                    if batching:
                        batch.append((req, slot, nb))
                    else:
                        h = self.backend.submit(req, slot)
                        inflight.append((h, slot, req, self.clock() - t0, nb))
                    self.peak_inflight = max(self.peak_inflight, len(inflight) + len(batch))
                    progressed = True
                    break
            if batch:
                hs = self.backend.submit_batch([(req, slot) for req, slot, _ in batch])
                adm = self.clock() - t0
                for (req, slot, nb), h in zip(batch, hs):
                    inflight.append((h, slot, req, adm, nb))
                self.batches += 1
                self.batched_frames += len(batch)
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
    """Frames on the device, one stream per robot.

    payload of a Request: (pinned host float32 [N,3] tensor, R, t).  Each
    result slot owns its plane/hull output buffers and pinned host copies of
    the per-cluster results; the D2H copies are enqueued behind the frame, so a
    completed frame's results are already in host memory.

    batch=False: each frame is one vm_segment_frame on its robot's stream, so
    frames of different robots overlap on the device.
    batch=True (continuous batching): the frames admitted together are
    inserted and labelled on their robots' streams (concurrently), then the
    planes and polygons of all their clusters are computed by one merged
    sequence of launches (vm_planes_hulls_multi) on a batch stream, each
    cluster with its own robot's frame number.  A robot's next frame is labelled only after the
    batch that read its map's clusters; its insert may run before.  The
    results are the same in both modes and the same alone or in the mix."""

    def __init__(self, maps, n_slots: int, n_hyp: int, min_cluster: int = 30, eps: float = 0.01,
                 seed: int = 0x5EED, k_cap: int = 8192, in_cap: int = 1 << 23, v_cap: int = 1 << 21,
                 capture_cap: int = 0, batch: bool = False, batch_k_cap: int = 65536, batch_n_cap: int = 1 << 24):
        """capture_cap > 0: every frame's full results (labels, cluster CSR,
        inlier and hull lists) are copied to host memory too, behind the
        frame on its stream, for maps of at most capture_cap occupied voxels
        (for checks; costs large copies).  batch_k_cap / batch_n_cap bound the
        clusters and points of one merged pass; a batch whose frames exceed them is split into
        several passes (its frames' sizes are read back once their clustering is done)."""
        import torch

        import paper_2510_01592_amd as vm
        self.vm = vm
        self.torch = torch
        self.maps = maps
        self.streams = [torch.cuda.Stream() for _ in maps]
        self.kw = dict(min_cluster=min_cluster, n_hyp=n_hyp, eps=eps, seed=seed)
        self.k_cap = k_cap
        self.in_cap, self.v_cap, self.capture_cap = in_cap, v_cap, int(capture_cap)
        self.planes = [vm.PlaneBuffers.alloc(k_cap, in_cap, n_hyp) for _ in range(n_slots)]
        self.hulls = [vm.HullBuffers.alloc(k_cap, v_cap) for _ in range(n_slots)]
        self.batching = bool(batch)
        if self.batching:
            self.batch_stream = torch.cuda.Stream()
            self.bk, self.bn = int(batch_k_cap), int(batch_n_cap)
            self.mwork = torch.empty(vm.multi_workspace_bytes(self.bk, self.bn, n_hyp), dtype=torch.uint8,
                                     device="cuda")
            self.robot_last = [None] * len(maps)
            self.swork = None    # workspace of single-frame groups, if the batch's is too small
            self.kn_host = [torch.empty(2, dtype=torch.int32).pin_memory() for _ in range(n_slots)]
            self.groups = 0      # merged passes run (a batch splits where its clusters exceed the caps)
        self.host = [dict(plane=torch.empty((k_cap, 4), dtype=torch.float32).pin_memory(),
                          best=torch.empty(k_cap, dtype=torch.int32).pin_memory(),
                          nin=torch.empty(k_cap, dtype=torch.int32).pin_memory(),
                          area=torch.empty(k_cap, dtype=torch.float64).pin_memory(),
                          v_off=torch.empty(k_cap + 1, dtype=torch.int32).pin_memory(),
                          meta=torch.empty(2, dtype=torch.int32).pin_memory(),
                          status=torch.empty(2, dtype=torch.int32).pin_memory(),
                          stats=torch.empty(vm.STATS_WORDS, dtype=torch.int64).pin_memory())
                     for _ in range(n_slots)]
        self.stats_dev = [torch.empty(vm.STATS_WORDS, dtype=torch.int64, device="cuda") for _ in range(n_slots)]
        self.capture = None
        if self.capture_cap:
            c = self.capture_cap

            def pin(n, dt):
                return torch.empty(n, dtype=dt).pin_memory()
            i32, f32 = torch.int32, torch.float32
            self.labels_dev = [torch.empty(c, dtype=i32, device="cuda") for _ in range(n_slots)]
            self.capture = [dict(labels=pin(c, i32), off=pin(k_cap + 1, i32), tag=pin(k_cap, i32), x=pin(c, f32),
                                 y=pin(c, f32), z=pin(c, f32), key=pin(c, i32), nin=pin(k_cap, i32),
                                 in_off=pin(k_cap + 1, i32), in_idx=pin(in_cap, i32), v_idx=pin(v_cap, i32),
                                 v_xyz=pin((v_cap, 3), f32)) for _ in range(n_slots)]

    def bytes_for(self, req: Request) -> int:
        return 12 * int(req.n_points)

    def _upload(self, req: Request):
        torch = self.torch
        pts = req.payload[0]
        d = torch.empty((req.n_points, 3), dtype=torch.float32, device="cuda")
        d.copy_(pts, non_blocking=True)
        return d

    def _capture_clusters(self, slot: int, cl) -> None:
        """the map's cluster CSR and labels (right after its labelling)"""
        if not self.capture:
            return
        vm = self.vm
        c, kc, nc = self.capture[slot], self.k_cap, self.capture_cap
        c["labels"].copy_(self.labels_dev[slot], non_blocking=True)
        for name, ptr, n, dt in (("off", cl.d_off, kc + 1, np.uint32), ("tag", cl.d_tag, kc, np.uint32),
                                 ("x", cl.d_x, nc, np.float32), ("y", cl.d_y, nc, np.float32),
                                 ("z", cl.d_z, nc, np.float32), ("key", cl.d_key, nc, np.uint32)):
            c[name].copy_(vm.device_view(ptr, n, dt), non_blocking=True)

    def _fetch(self, slot: int, cl) -> None:
        """the frame's results to the slot's pinned host buffers (current stream)"""
        vm = self.vm
        pb, hb, h = self.planes[slot], self.hulls[slot], self.host[slot]
        if self.capture:
            c = self.capture[slot]
            c["nin"].copy_(pb.n_inliers, non_blocking=True)
            c["in_off"].copy_(pb.in_off, non_blocking=True)
            c["in_idx"].copy_(pb.in_idx[:self.in_cap], non_blocking=True)
            c["v_idx"].copy_(hb.v_idx[:self.v_cap], non_blocking=True)
            c["v_xyz"].copy_(hb.v_xyz[:self.v_cap], non_blocking=True)
        h["plane"].copy_(pb.plane, non_blocking=True)
        h["best"].copy_(pb.best_h, non_blocking=True)
        h["nin"].copy_(pb.n_inliers, non_blocking=True)
        h["area"].copy_(hb.area, non_blocking=True)
        h["v_off"].copy_(hb.v_off, non_blocking=True)
        h["meta"].copy_(vm.device_view(cl.d_meta, 2, np.int32), non_blocking=True)
        h["status"][0:1].copy_(pb.status, non_blocking=True)
        h["status"][1:2].copy_(hb.status, non_blocking=True)
        h["stats"].copy_(self.stats_dev[slot], non_blocking=True)

    def submit(self, req: Request, slot: int):
        torch = self.torch
        _, R, t = req.payload
        s = self.streams[req.robot]
        with torch.cuda.stream(s):
            d = self._upload(req)
            pb, hb = self.planes[slot], self.hulls[slot]
            pb.status.zero_()
            hb.status.zero_()
            labels = self.labels_dev[slot] if self.capture else None
            cl = self.maps[req.robot].segment_frame(d, pb, hb, R=R, t=t, frame=req.seq, labels=labels, stream=s,
                                                    **self.kw)
            self._capture_clusters(slot, cl)
            self.maps[req.robot].stats_async(self.stats_dev[slot], stream=s)
            self._fetch(slot, cl)
            ev = torch.cuda.Event()
            ev.record(s)
            d.record_stream(s)
        return ev

    def submit_batch(self, items):
        if not self.batching:
            return super().submit_batch(items)
        torch, vm = self.torch, self.vm
        views, frames, pbs, hbs, ready = [], [], [], [], []
        for req, slot in items:
            _, R, t = req.payload
            s = self.streams[req.robot]
            m = self.maps[req.robot]
            with torch.cuda.stream(s):
                d = self._upload(req)
                m.insert(d, R, t, stream=s)
                if self.robot_last[req.robot] is not None:
                    # the batch that read this map's previous clusters
                    s.wait_event(self.robot_last[req.robot])
                labels = self.labels_dev[slot] if self.capture else None
                cl = m.ccl(self.kw["min_cluster"], labels=labels, stream=s)
                self._capture_clusters(slot, cl)
                m.stats_async(self.stats_dev[slot], stream=s)
                self.planes[slot].status.zero_()
                self.hulls[slot].status.zero_()
                # the cluster and point counts, to pinned memory behind the labelling
                self.kn_host[slot].copy_(vm.device_view(cl.d_meta, 2, np.int32), non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(s)
                d.record_stream(s)
            views.append(cl)
            frames.append(req.seq)
            pbs.append(self.planes[slot])
            hbs.append(self.hulls[slot])
            ready.append(ev)
        # the frames' cluster and point counts (a host wait for their
        # clustering), then groups of consecutive frames within the batch
        # capacities: nothing is truncated by merging
        sizes = []
        for ev, (req, slot) in zip(ready, items):
            ev.synchronize()
            kn = self.kn_host[slot]
            sizes.append((int(kn[0]), int(kn[1])))
        groups, cur, ck, cn = [], [], 0, 0
        for i, (k, n) in enumerate(sizes):
            if cur and (ck + k > self.bk or cn + n > self.bn):
                groups.append(cur)
                cur, ck, cn = [], 0, 0
            cur.append(i)
            ck += k
            cn += n
        if cur:
            groups.append(cur)
        bs = self.batch_stream
        for ev in ready:
            bs.wait_event(ev)
        with torch.cuda.stream(bs):
            kw = self.kw
            for g in groups:
                if len(g) == 1:
                    # a frame alone (it may exceed the merged bounds): the two-pass
                    # kernels with its own frame word
                    i = g[0]
                    need = vm.workspace_bytes(min(views[i].k_cap, pbs[i].k_cap, hbs[i].k_cap), views[i].n_cap,
                                              kw["n_hyp"])
                    work = self.mwork
                    if work.numel() < need:
                        if self.swork is None or self.swork.numel() < need:
                            self.swork = torch.empty(need, dtype=torch.uint8, device="cuda")
                        work = self.swork
                    prm = vm.ransac_params(kw["n_hyp"], kw["eps"], kw["seed"], frames[i])
                    vm.ransac_planes(views[i], prm, pbs[i], work, stream=bs)
                    vm.hulls(views[i], pbs[i], hbs[i], work, stream=bs)
                else:
                    vm.planes_hulls_multi([views[i] for i in g], [frames[i] for i in g],
                                          vm.ransac_params(kw["n_hyp"], kw["eps"], kw["seed"]),
                                          [pbs[i] for i in g], [hbs[i] for i in g], self.bk, self.bn, self.mwork,
                                          stream=bs)
            self.groups += len(groups)
            for (req, slot), cl in zip(items, views):
                self._fetch(slot, cl)
            done = torch.cuda.Event()
            done.record(bs)
        for req, _ in items:
            self.robot_last[req.robot] = done
        return [done] * len(items)

    def done(self, handle) -> bool:
        return handle.query()

    def result(self, handle, slot: int):
        h = self.host[slot]
        K = min(int(h["meta"][0]), self.k_cap)
        out = dict(K=int(h["meta"][0]), N=int(h["meta"][1]), plane=h["plane"][:K].numpy().copy(),
                   best=h["best"][:K].numpy().copy(), nin=h["nin"][:K].numpy().copy(),
                   area=h["area"][:K].numpy().copy(), v_off=h["v_off"][:K + 1].numpy().copy(),
                   status=h["status"].numpy().copy(), occupied=int(h["stats"][0]))
        if self.capture:
            c = self.capture[slot]
            N, V = int(h["meta"][1]), out["occupied"]
            u32 = np.uint32
            out.update(N=N, labels=c["labels"][:V].numpy().view(u32).copy(), off=c["off"][:K + 1].numpy().view(u32).copy(),
                       tag=c["tag"][:K].numpy().view(u32).copy(),
                       xyz=np.stack([c[a][:N].numpy() for a in "xyz"], axis=1),
                       key=c["key"][:N].numpy().view(u32).copy(), nin=c["nin"][:K].numpy().copy())
            in_off = c["in_off"][:K + 1].numpy().view(u32).copy()
            v_off = out["v_off"].view(u32)
            out.update(in_off=in_off, in_idx=c["in_idx"][:int(in_off[K])].numpy().view(u32).copy(),
                       v_idx=c["v_idx"][:int(v_off[K])].numpy().view(u32).copy(),
                       v_xyz=c["v_xyz"][:int(v_off[K])].numpy().copy())
        return out

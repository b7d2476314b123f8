#!/usr/bin/env python3
"""Benchmark: occupied voxels segmented per second and frame latency on the
full local map workload (4x4x2 m at 0.01 m = 400x400x200 cells, 1M float32
points per frame with N(0, 3 mm) noise and 5 % outliers, 512 RANSAC
hypotheses, clusters below 30 voxels dropped), on one MI355X.

A step is one frame of the whole path: insert the frame into the resident
map, label all occupied voxels, group them, fit one plane per cluster and
outline it.  The map is warmed with 30 frames (about 1.95M occupied voxels)
and keeps growing by each frame's outliers, as an accumulating map does; the
metric sums the occupied voxels each step segmented.  Frames are resident in
HBM before a timed region starts.  Two forms run on the same starting map
(snapshot/restore) and the same frames:
  plain  -- one vm_segment_frame call per frame;
  graph  -- the frame captured once as a HIP graph and replayed (the frame's
            points copied into the captured input buffer, the RANSAC frame
            number advanced in device memory).
`value` is the plain form's throughput (the graph form adds a copy of the
frame into the captured buffer per step); the graph form is reported beside.

Prints one JSON line."""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "occupied voxels segmented/s and p50/p99 frame latency, plain vs batched/served @0.01 m"
HBM_PEAK_GBS = 8000.0
# vector ALU: 256 CUs x 64 lanes x 2.4 GHz lane-instructions/s; one inlier
# test is 3 v_fma_f32 + 1 v_cmp (packed fp32 off), so 4 lane-instructions
VALU_LANE_OPS = 256 * 64 * 2.4e9
COUNT_PEAK_GEVAL = VALU_LANE_OPS / 4 / 1e9


def _log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prewarm", type=int, default=30, help="frames inserted before the first step")
    ap.add_argument("--latency-frames", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=1)
    ap.add_argument("--no-batched", action="store_true", help="skip the 2000-cluster batched measurement")
    ap.add_argument("--no-served", action="store_true", help="skip the multi-robot served measurement")
    ap.add_argument("--served-seconds", type=float, default=3.0, help="span of the served arrival process")
    ap.add_argument("--counters", action="store_true",
                    help="run only the inlier-counting launches of the roofline and a 256 MiB copy (for rocprofv3 --pmc)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter files of a --counters run into profiles/k_count_traffic.json")
    args = ap.parse_args()
    if args.traffic_from:
        return _traffic_from(*args.traffic_from)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the segmentation path is a "
                                   "single-GPU kernel pipeline (one map per GPU); --gpus must be 1"}), flush=True)
        return 2

    import torch

    import paper_2510_01592_amd as vm
    import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()

    sc = scenes.scene_full_map(1)
    g = sc.geom
    H, eps, minc, seed = sc.n_hyp, sc.eps, sc.min_cluster, 0x5EED
    m = vm.Map(g.origin, g.voxel_size, g.dims, 23)

    # ---- pre-warm the map and keep a snapshot (not timed) -------------------
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for f in range(args.prewarm):
            m.insert(torch.from_numpy(scenes.frame_points(sc, 2 + f)).to(dev), stream=stream)
    stream.synchronize()
    snap = m.export(stream=stream)
    v_prewarm = int(snap[0].shape[0])
    _log(f"prewarm {args.prewarm} frames -> {v_prewarm} occupied voxels ({time.perf_counter() - t0:.1f}s)")

    def restore():
        with torch.cuda.stream(stream):
            m.import_(snap[0], snap[1], snap[2], stream=stream)
        stream.synchronize()

    n_frames = args.warmup + args.steps
    frames = [torch.from_numpy(scenes.frame_points(sc, 1000 + i)).to(dev) for i in range(n_frames)]
    k_cap = 16384
    planes = vm.PlaneBuffers.alloc(k_cap, 1 << 23, H)
    hulls = vm.HullBuffers.alloc(k_cap, 1 << 22)
    stats_dev = torch.zeros((n_frames + 1, 6), dtype=torch.int64, device=dev)
    stage = torch.empty((sc.n_points, 3), dtype=torch.float32, device=dev)
    frame_t = torch.zeros(1, dtype=torch.int32, device=dev)
    kw = dict(min_cluster=minc, n_hyp=H, eps=eps, seed=seed)
    last = {}
    if args.counters:
        return _counters_run(vm, torch, m, frames, planes, hulls, k_cap, H, eps, seed, kw, stream, dev, restore,
                             args.warmup, min(5, args.steps))

    # ---- plain form ------------------------------------------------------------
    def plain_step(i: int) -> None:
        last["cl"] = m.segment_frame(frames[i], planes, hulls, frame=i, stream=stream, **kw)
        m.stats_async(stats_dev[i], stream=stream)

    restore()
    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            plain_step(i)
        stream.synchronize()
        t_s = time.perf_counter()
        for i in range(args.warmup, n_frames):
            plain_step(i)
        stream.synchronize()
        t_plain = time.perf_counter() - t_s
    occ = stats_dev.cpu().numpy()[args.warmup:n_frames, 0].astype(np.int64)
    plain_value = float(occ.sum()) / t_plain
    _log(f"plain: {1e3 * t_plain / args.steps:.3f} ms/step, {plain_value / 1e6:.1f} M voxels/s, "
         f"occupied {occ[0]}..{occ[-1]}")

    # ---- graph form: the frame captured once, replayed per frame ---------------
    restore()
    stats_slot = torch.zeros(6, dtype=torch.int64, device=dev)
    with torch.cuda.stream(stream):
        with vm.capture(stream) as cap:
            last["cl"] = m.segment_frame(stage, planes, hulls, d_frame=frame_t, stream=stream, **kw)
            m.stats_async(stats_slot, stream=stream)
    graph = cap.graph
    stats_dev.zero_()

    def graph_step(i: int) -> None:
        stage.copy_(frames[i])
        frame_t.fill_(i)
        graph.launch(stream)
        stats_dev[i].copy_(stats_slot)

    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            graph_step(i)
        stream.synchronize()
        t_s = time.perf_counter()
        for i in range(args.warmup, n_frames):
            graph_step(i)
        stream.synchronize()
        t_graph = time.perf_counter() - t_s
    occ_g = stats_dev.cpu().numpy()[args.warmup:n_frames, 0].astype(np.int64)
    assert np.array_equal(occ_g, occ), "graph replays must see the same maps as direct calls"
    value = float(occ_g.sum()) / t_graph
    ms_per_step = 1e3 * t_graph / args.steps
    _log(f"graph: {ms_per_step:.3f} ms/step, {value / 1e6:.1f} M voxels/s")

    # ---- frame latency: pinned host frame -> results in host memory -------------
    host_frames = [torch.from_numpy(scenes.frame_points(sc, 5000 + i)).pin_memory() for i in range(4)]
    res_plane = torch.empty((k_cap, 4), dtype=torch.float32).pin_memory()
    res_area = torch.empty(k_cap, dtype=torch.float64).pin_memory()
    res_voff = torch.empty(k_cap + 1, dtype=torch.int32).pin_memory()
    res_stat = torch.empty(2, dtype=torch.int32).pin_memory()

    def fetch():
        res_plane.copy_(planes.plane, non_blocking=True)
        res_area.copy_(hulls.area, non_blocking=True)
        res_voff.copy_(hulls.v_off, non_blocking=True)
        res_stat[0:1].copy_(planes.status, non_blocking=True)
        res_stat[1:2].copy_(hulls.status, non_blocking=True)

    lat = {"plain": [], "graph": []}
    with torch.cuda.stream(stream):
        # one untimed pass over the host frames first (the first copy from a
        # pinned buffer pays for mapping it)
        for i, hf in enumerate(host_frames):
            stage.copy_(hf, non_blocking=True)
            frame_t.fill_(19000 + i)
            graph.launch(stream)
            fetch()
            stream.synchronize()
        for i in range(args.latency_frames):
            hf = host_frames[i % len(host_frames)]
            for form in ("graph", "plain"):
                stream.synchronize()
                ta = time.perf_counter()
                stage.copy_(hf, non_blocking=True)
                if form == "graph":
                    frame_t.fill_(20000 + i)
                    graph.launch(stream)
                else:
                    m.segment_frame(stage, planes, hulls, frame=20000 + i, stream=stream, **kw)
                fetch()
                stream.synchronize()
                lat[form].append(1e3 * (time.perf_counter() - ta))
    lat_out = {}
    for form, v in lat.items():
        a = np.array(v)
        lat_out[form] = {"p50": float(np.percentile(a, 50)), "p99": float(np.percentile(a, 99)), "frames": len(a)}
    _log(f"latency graph p50 {lat_out['graph']['p50']:.2f} p99 {lat_out['graph']['p99']:.2f} ms; "
         f"plain p50 {lat_out['plain']['p50']:.2f} p99 {lat_out['plain']['p99']:.2f} ms")

    # ---- per-stage device time (HIP events on the library's stream) -------------
    restore()
    vm.set_stage_timing(True)
    n_stage = min(5, args.steps)
    with torch.cuda.stream(stream):
        for i in range(n_stage):
            last["cl"] = m.segment_frame(frames[args.warmup + i], planes, hulls, frame=args.warmup + i,
                                         stream=stream, **kw)
        stream.synchronize()
    ms, _ = vm.stage_times()
    stage_ms = {name: float(ms[j]) / n_stage for j, name in enumerate(vm.STAGES)}
    # inlier counting timed alone (standalone calls keep the GPU busy, so the
    # events bracket the kernel itself); the last frame's clusters, all of them
    work = torch.empty(vm.workspace_bytes(k_cap, last["cl"].n_cap, H), dtype=torch.uint8, device=dev)
    reps = 10
    with torch.cuda.stream(stream):
        for r in range(reps):
            vm.ransac_planes(last["cl"], vm.ransac_params(H, eps, seed, r), planes, work, stream=stream)
        stream.synchronize()
    ms2, n2 = vm.stage_times()
    vm.set_stage_timing(False)
    count_ms = float(ms2[vm.STAGES.index("count")]) / reps
    cl_meta = vm.read_clusters(last["cl"])
    n_pts = cl_meta["N"]
    evals = float(n_pts) * H
    _log("stage ms/frame: " + ", ".join(f"{k}={v:.3f}" for k, v in stage_ms.items()) +
         f"; k_count alone {count_ms:.3f} ms for {evals / 1e6:.0f}M evaluations")
    ach = evals / (count_ms * 1e-3) / 1e9
    roof = {"bound": "alu", "achieved": ach, "peak": COUNT_PEAK_GEVAL, "unit": "Geval/s",
            "frac": ach / COUNT_PEAK_GEVAL, "traffic": _traffic(),
            "kernel": "inlier counting: k_count_small (a wave per cluster of <= %d points) + k_count (tiles)"
                      % vm.get_count_config()["wave_max_points"],
            "work_per_launch": f"{n_pts} points x {H} hypotheses",
            "peak_derivation": "256 CU x 64 lanes x 2.4 GHz / 4 VALU instructions per point-plane test"}

    # ---- batched clusters: 2000 log-uniform clusters, one pass, graph replays ------
    batched = None
    if not args.no_batched:
        batched = _batched(vm, torch, dev, stream)
        _log(f"batched: {batched}")

    # ---- served: 8 robots, Poisson arrivals, continuous admission ---------------
    served = None
    if not args.no_served:
        served = _served(vm, torch, args.served_seconds)
        _log(f"served: {served}")

    # ---- the oracle on the host, bounded sample ---------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(sc, args.prewarm, args.cpu_frames, H, eps, minc, seed)
        _log(f"cpu baseline: {cpu}")

    graph.close()
    out = {
        "metric": METRIC,
        "value": plain_value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_plain / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "full local map: 4x4x2 m at 0.01 m (400x400x200 cells), floor + 12-step open-tread "
                        "staircase + tabletop + 20 tilted patches, 1M float32 points/frame, N(0,3 mm), 5% outliers, "
                        "512 hypotheses, eps 0.01 m, min cluster 30",
            "form": "plain (one vm_segment_frame call per frame)",
            "prewarm_frames": args.prewarm,
            "occupied_first_step": int(occ[0]),
            "occupied_last_step": int(occ[-1]),
            "points_per_frame": sc.n_points,
            "n_hyp": H,
        },
        "forms": {
            "plain": {"value": plain_value, "ms_per_step": 1e3 * t_plain / args.steps},
            "graph": {"value": value, "ms_per_step": ms_per_step},
        },
        "latency_ms": dict(lat_out, includes="H2D of the frame from pinned host memory, the frame, D2H of planes, "
                                             "areas, polygon offsets and status words"),
        "stage_ms_per_frame": stage_ms,
        "roofline": roof,
        "batched": batched,
        "served": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


def _batched(vm, torch, dev, stream, replays: int = 100):
    """2000 clusters of log-uniform size (50..200k points, about 48.5M in all),
    1024 hypotheses: planes and hulls of all clusters in one pass, captured as
    a graph and replayed `replays` times with the frame number advanced in
    device memory (the data stays resident)."""
    import scenes
    t0 = time.perf_counter()
    off, xyz = scenes.batched_clusters(seed=3)
    K, N, H = len(off) - 1, len(xyz), 1024
    cl, keep = vm.clusters_from_host(off, xyz, np.arange(K, dtype=np.uint32))
    gen_s = time.perf_counter() - t0
    work = torch.empty(vm.workspace_bytes(K, N, H), dtype=torch.uint8, device=dev)
    planes = vm.PlaneBuffers.alloc(K, N, H)
    hulls = vm.HullBuffers.alloc(K, N)
    frame_t = torch.zeros(1, dtype=torch.int32, device=dev)
    with torch.cuda.stream(stream):
        vm.ransac_planes(cl, vm.ransac_params(H, 0.01, 0x5EED, 0), planes, work, stream=stream)
        vm.hulls(cl, planes, hulls, work, stream=stream)
        stream.synchronize()
        t_s = time.perf_counter()
        for f in range(3):
            vm.ransac_planes(cl, vm.ransac_params(H, 0.01, 0x5EED, f), planes, work, stream=stream)
            vm.hulls(cl, planes, hulls, work, stream=stream)
        stream.synchronize()
        plain_ms = 1e3 * (time.perf_counter() - t_s) / 3
        with vm.capture(stream) as cap:
            vm.ransac_planes(cl, vm.ransac_params(H, 0.01, 0x5EED, d_frame=frame_t), planes, work, stream=stream)
            vm.hulls(cl, planes, hulls, work, stream=stream)
        cap.graph.launch(stream)
        stream.synchronize()
        t_s = time.perf_counter()
        for f in range(replays):
            frame_t.fill_(f)
            cap.graph.launch(stream)
        stream.synchronize()
        graph_ms = 1e3 * (time.perf_counter() - t_s) / replays
        vm.set_stage_timing(True)
        for f in range(3):
            vm.ransac_planes(cl, vm.ransac_params(H, 0.01, 0x5EED, f), planes, work, stream=stream)
        stream.synchronize()
        ms, _ = vm.stage_times()
        vm.set_stage_timing(False)
        # the counting decomposition tuned on this workload (results are
        # identical under every setting; only the counting time changes)
        t_s = time.perf_counter()
        tuned = vm.autotune_count(cl, vm.ransac_params(H, 0.01, 0x5EED, 0), planes, work, stream=stream, reps=2)
        tune_s = time.perf_counter() - t_s
        vm.set_stage_timing(True)
        for f in range(3):
            vm.ransac_planes(cl, vm.ransac_params(H, 0.01, 0x5EED, f), planes, work, stream=stream)
        stream.synchronize()
        ms_t, _ = vm.stage_times()
        vm.set_stage_timing(False)
        vm.set_count_config(None)
    cap.graph.close()
    count_ms = float(ms[vm.STAGES.index("count")]) / 3
    count_ms_tuned = float(ms_t[vm.STAGES.index("count")]) / 3
    evals = float(N) * H
    ach = evals / (count_ms * 1e-3) / 1e9
    st = int(planes.status.cpu()[0]) | int(hulls.status.cpu()[0])
    del keep
    return {"workload": f"{K} clusters, log-uniform 50..200k points ({N} in all), {H} hypotheses, "
                        "planes + hulls of all clusters per frame",
            "ms_per_frame_graph": graph_ms, "ms_per_frame_plain": plain_ms, "replays": replays,
            "points_per_s_graph": N / (graph_ms * 1e-3), "evaluations_per_s_graph": evals / (graph_ms * 1e-3),
            "k_count_ms": count_ms,
            "count_autotune": {"config": tuned, "k_count_ms": count_ms_tuned, "tuning_s": tune_s,
                               "default": vm.get_count_config()},
            "roofline_k_count": {"bound": "alu", "achieved": ach, "peak": COUNT_PEAK_GEVAL, "unit": "Geval/s",
                                 "frac": ach / COUNT_PEAK_GEVAL},
            "status_flags": st, "generation_s": gen_s}


def _served(vm, torch, seconds: float, n_robots: int = 8, rate_hz: float = 30.0, pool: int = 3):
    """Several robots, each with its own map of the full-map workload (scene
    seed = robot), send frames as Poisson processes at `rate_hz`; a frame has
    U(200k, 2M) points (a prefix of one of the robot's `pool` shuffled
    pre-generated frames, each taken at its own pose of a random walk).  The
    scheduler admits frames as they arrive, subject to per-robot order, result
    slots and an HBM budget for in-flight frames; latency is arrival ->
    results in pinned host memory."""
    import scenes
    from paper_2510_01592_amd.serve import GpuBackend, Request, Scheduler, latency_summary, poisson_arrivals
    t0 = time.perf_counter()
    maps, host = [], []
    n_max = 2_000_000
    for r in range(n_robots):
        sc = scenes.scene_full_map(1 + r)
        g = sc.geom
        maps.append(vm.Map(g.origin, g.voxel_size, g.dims, 23))
        poses = scenes.random_walk_poses(100 + r, pool, sigma_t=0.01, sigma_rot_deg=0.5)
        host.append([(torch.from_numpy(scenes.frame_points(sc, 7000 + 10 * r + k, n=n_max, pose=poses[k])).pin_memory(),
                      poses[k][0], poses[k][1]) for k in range(pool)])
    gen_s = time.perf_counter() - t0
    n_slots, budget = 16, 256 << 20
    be = GpuBackend(maps, n_slots=n_slots, n_hyp=512)
    rng = np.random.default_rng(12345)
    reqs = []
    # one untimed warm-up frame per robot (allocates each map's workspace)
    warm = [Request(r, 0, 0.0, 1_000_000, (host[r][0][0][:1_000_000], host[r][0][1], host[r][0][2]))
            for r in range(n_robots)]
    Scheduler(be, n_robots, n_slots, budget).run(warm)
    for r in range(n_robots):
        for k, ta in enumerate(poisson_arrivals(rate_hz, seconds, 500 + r)):
            n = int(rng.integers(200_000, n_max + 1))
            src = host[r][k % pool]
            reqs.append(Request(r, k + 1, float(ta), n, (src[0][:n], src[1], src[2])))
    sch = Scheduler(be, n_robots, n_slots, budget)
    torch.cuda.synchronize()
    t_s = time.perf_counter()
    done = sch.run(reqs, t0=t_s)
    t_span = time.perf_counter() - t_s
    summ = latency_summary(done, t_span)
    vox = sum(c.result["occupied"] for c in done)
    bad = sum(1 for c in done if c.result["status"].any())
    for m in maps:
        m.close()
    return dict(summ, robots=n_robots, rate_hz_per_robot=rate_hz, arrival_span_s=seconds, wall_s=t_span,
                points_per_frame="U(200k, 2M)", n_hyp=512, slots=n_slots, budget_mib=budget >> 20,
                peak_inflight=sch.peak_inflight, rejected=len(sch.rejected), frames_with_status_flags=bad,
                voxels_per_s=vox / t_span, points_per_s=sum(c.request.n_points for c in done) / t_span,
                generation_s=gen_s)


COPY_BYTES = 256 << 20
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "k_count_traffic.json")
COUNT_SRC = os.path.join(ROOT, "paper_2510_01592_amd", "csrc", "vm_ransac.hip")


def _sha256(path: str) -> str:
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _counters_run(vm, torch, m, frames, planes, hulls, k_cap, H, eps, seed, kw, stream, dev, restore, first, n):
    """The launches the roofline is measured on -- n frames, then 10
    standalone inlier-counting passes over the last frame's clusters -- and a
    256 MiB device copy whose counters scale FETCH_SIZE/WRITE_SIZE to bytes."""
    restore()
    with torch.cuda.stream(stream):
        cl = None
        for i in range(n):
            cl = m.segment_frame(frames[first + i], planes, hulls, frame=first + i, stream=stream, **kw)
        work = torch.empty(vm.workspace_bytes(k_cap, cl.n_cap, H), dtype=torch.uint8, device=dev)
        for r in range(10):
            vm.ransac_planes(cl, vm.ransac_params(H, eps, seed, r), planes, work, stream=stream)
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        stream.synchronize()
    meta = vm.read_clusters(cl)
    print(json.dumps({"counters_run": True, "k_count_launches": 10, "points": int(meta["N"]),
                      "clusters": int(meta["K"]), "n_hyp": H, "copy_bytes": COPY_BYTES}), flush=True)
    return 0


def _pmc_rows(path: str):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _traffic_from(fetch_csv: str, write_csv: str) -> int:
    """HBM bytes per counting pass (the last 10 passes, two dispatches each):
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) each scaled by what the same
    counter reads for the 256 MiB copy of the --counters run."""
    out = {"kernel": "k_count_small + k_count (one counting pass)", "source": os.path.relpath(COUNT_SRC, ROOT),
           "source_sha256": _sha256(COUNT_SRC)}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _pmc_rows(path)
        cnt = "FETCH_SIZE" if name == "fetch" else "WRITE_SIZE"
        rows = [r for r in rows if r["Counter_Name"] == cnt]
        # each counting pass is two dispatches (clusters of one wave, then tiled)
        kc = [float(r["Counter_Value"]) for r in rows if "k_count" in r["Kernel_Name"]][-20:]
        cp = max(float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                 or "elementwise" in r["Kernel_Name"])
        scale = COPY_BYTES / (cp * 1024.0)
        out[f"{name}_kib_per_launch_raw"] = sum(kc) / 10
        out[f"{name}_copy_kib_raw"] = cp
        out[f"{name}_scale"] = scale
        out[f"{name}_bytes_per_launch"] = sum(kc) / 10 * 1024.0 * scale
    out["traffic_bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)
    return 0


def _traffic():
    """Measured HBM bytes per k_count launch, if the counters were taken on the
    kernel source as it is now; else None."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
        if t.get("source_sha256") != _sha256(COUNT_SRC):
            return None
        return float(t["traffic_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def _cpu_baseline(sc, prewarm, n_frames, H, eps, minc, seed):
    """The oracle (single-threaded C + numpy grouping) on the same workload:
    the warmed map is rebuilt untimed, then n_frames frames are inserted and
    segmented (all clusters) and timed."""
    import oracle
    import scenes
    g = sc.geom
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    for f in range(prewarm):
        om.insert(scenes.frame_points(sc, 2 + f))
    frames = [scenes.frame_points(sc, 1000 + i) for i in range(n_frames)]
    voxels = 0
    t0 = time.perf_counter()
    for i, pts in enumerate(frames):
        om.insert(pts)
        voxels += len(om.key)
        oracle.segment(om, minc, H, eps, seed, i)
    t = time.perf_counter() - t0
    return {"value": voxels / t, "unit": "voxels/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_frames} frame(s) of the same workload after the same {prewarm}-frame warm-up "
                      f"({voxels} occupied voxels segmented in {t:.1f} s, single thread)"}


if __name__ == "__main__":
    sys.exit(main())

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

Beside the headline: frame latency over 100 frames per form, per-stage
device time, the rooflines of the labelling (HBM), counting (fp32 VALU),
insert and grouping stages with the published peaks and the peaks measured
by microbenchmarks in the same run, the 2000-cluster batched set, the
8-robot served stream (and the same trace one frame at a time), the
0.005 m stress map, and the oracle on the host cores.

Prints one JSON line."""
from __future__ import annotations

import argparse
import concurrent.futures
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "occupied voxels segmented/s and p50/p99 frame latency, plain vs batched/served @0.01 m"
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3        # MI355X fp32 vector, published
FLOP_PER_TEST = 6               # an inlier test is three fused multiply-adds (and a compare)
COUNT_PEAK_TTESTS = FP32_PEAK_TFLOPS / FLOP_PER_TEST   # the published fp32 peak in inlier tests/s (26.2 T)
PEAKS_LIB = os.path.join(ROOT, "paper_2510_01592_amd", "libvm_peaks.so")
CSRC = os.path.join(ROOT, "paper_2510_01592_amd", "csrc")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "kernel_traffic.json")
COPY_BYTES = 256 << 20
HOST_THREADS = max(1, min(16, os.cpu_count() or 1))

# kernels of each measured unit, and the source file each lives in
UNITS = {
    "ccl": (["k_ccl_tile", "k_ccl_boundary", "k_ccl_pairs", "k_ccl_flatten"], "vm_ccl.hip"),
    "count": (["k_count_small", "k_count"], "vm_ransac.hip"),
    "insert": (["k_vox_bucket", "k_bucket_scatter", "k_bucket_insert"], "vm_map.hip"),
    "group": (["k_group_pairs", "k_group_gather"], "vm_ccl.hip"),
    "fused": (["k_fused_hyp", "k_fused"], "vm_fused.hip"),
}
# headers every kernel file includes: part of each unit's source fingerprint
SHARED_HEADERS = ("vm_common.h", "vm_dev.h", "vm_tilescan.h")


def _log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prewarm", type=int, default=30, help="frames inserted before the first step")
    ap.add_argument("--latency-frames", type=int, default=100, help="frames per form in the latency measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=3)
    ap.add_argument("--no-batched", action="store_true", help="skip the 2000-cluster batched measurement")
    ap.add_argument("--no-served", action="store_true", help="skip the multi-robot served measurement")
    ap.add_argument("--no-stress", action="store_true", help="skip the 0.005 m stress map")
    ap.add_argument("--served-seconds", type=float, default=4.0, help="span of the served arrival process")
    ap.add_argument("--no-clearing", action="store_true", help="skip the ray-cast clearing measurement")
    ap.add_argument("--no-ablation", action="store_true", help="skip the cluster-parallel ablation")
    ap.add_argument("--only", choices=["batched", "served", "stress", "clearing", "ablation"],
                    help="run one side measurement alone (no headline line; for profiling)")
    ap.add_argument("--counters", action="store_true",
                    help="run only the frames, counting passes and a 256 MiB copy whose counters "
                         "rocprofv3 --pmc collects")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter files of a --counters run into profiles/kernel_traffic.json")
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

    if args.only == "batched":
        print(json.dumps({"batched": _batched(vm, torch, dev, stream)}), flush=True)
        return 0
    if args.only == "served":
        print(json.dumps({"served": _served(vm, torch, args.served_seconds)}), flush=True)
        return 0
    if args.only == "stress":
        print(json.dumps({"stress": _stress(vm, torch, dev, stream, with_oracle=False)}), flush=True)
        return 0
    if args.only == "clearing":
        print(json.dumps({"clearing": _clearing(vm, torch, dev, stream)}), flush=True)
        return 0
    if args.only == "ablation":
        print(json.dumps({"cluster_ablation": _cluster_ablation(vm, torch, dev, stream)}), flush=True)
        return 0

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
    stats_dev = torch.zeros((n_frames + 1, vm.STATS_WORDS), dtype=torch.int64, device=dev)
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

    # ---- accuracy: plane IoU against the generator's rectangles (last frame) ------
    iou = {"plain": _plane_iou(vm, sc, planes, hulls, last["cl"])}
    with torch.cuda.stream(stream):
        cl_st = m.segment_frame(frames[n_frames - 1], planes, hulls, frame=n_frames - 1, stream=stream,
                                step=vm.step_params(), **kw)
        stream.synchronize()
    # the steppable path keeps only near-horizontal surfaces: scored on those
    iou["steppable"] = _plane_iou(vm, sc, planes, hulls, cl_st, max_tilt_deg=15.0)
    _log(f"plane IoU: {json.dumps(iou)}")

    # ---- graph form: the frame captured once, replayed per frame ---------------
    restore()
    stats_slot = torch.zeros(vm.STATS_WORDS, dtype=torch.int64, device=dev)
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

    # the latency frames grow the map further; they start from the snapshot
    restore()
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
    lat_out = {form: {"p50": _pct(v, 50), "p99": _pct(v, 99), "max": float(max(v)), "frames": len(v)}
               for form, v in lat.items()}
    lat_occ = int(m.stats(stream).occupied)
    _log(f"latency graph p50 {lat_out['graph']['p50']:.2f} p99 {lat_out['graph']['p99']:.2f} ms; "
         f"plain p50 {lat_out['plain']['p50']:.2f} p99 {lat_out['plain']['p99']:.2f} ms "
         f"({args.latency_frames} frames each, map grows to {lat_occ} voxels)")

    # ---- per-stage device time (HIP events on the library's stream) -------------
    restore()
    vm.set_stage_timing(True)
    n_stage = min(5, args.steps)
    st_stats = torch.zeros((n_stage, vm.STATS_WORDS), dtype=torch.int64, device=dev)
    with torch.cuda.stream(stream):
        for i in range(n_stage):
            last["cl"] = m.segment_frame(frames[args.warmup + i], planes, hulls, frame=args.warmup + i,
                                         stream=stream, **kw)
            m.stats_async(st_stats[i], stream=stream)
        stream.synchronize()
    ms, _ = vm.stage_times()
    stage_ms = {name: float(ms[j]) / n_stage for j, name in enumerate(vm.STAGES)}
    st_np = st_stats.cpu().numpy()
    v_stage = float(st_np[:, 0].mean())              # occupied voxels segmented per stage frame
    touched = float(st_np[:, 5].mean())              # slot updates of each frame's insert
    cl_meta = vm.read_clusters(last["cl"])
    kept = float(cl_meta["N"])
    key_np = m.export(stream=stream)[0].cpu().numpy().view(np.uint32)
    bricks = _touched_bricks(key_np, g.dims)
    # inlier counting timed alone (standalone calls keep the GPU busy, so the
    # events bracket the kernels themselves); the last frame's clusters
    work = torch.empty(vm.workspace_bytes(k_cap, last["cl"].n_cap, H), dtype=torch.uint8, device=dev)
    reps = 10
    with torch.cuda.stream(stream):
        for r in range(reps):
            vm.ransac_planes(last["cl"], vm.ransac_params(H, eps, seed, r), planes, work, stream=stream)
        stream.synchronize()
    ms2, _ = vm.stage_times()
    vm.set_stage_timing(False)
    count_ms = float(ms2[vm.STAGES.index("count")]) / reps
    n_pts = cl_meta["N"]
    tests = float(n_pts) * H
    _log("stage ms/frame: " + ", ".join(f"{k}={v:.3f}" for k, v in stage_ms.items()) +
         f"; counting pass alone {count_ms:.3f} ms for {tests / 1e6:.0f}M tests")

    # ---- Alg. 1's label propagation against the union-find labelling (same map) --
    restore()
    ccl_cmp = _ccl_compare(vm, m, stream)
    _log(f"ccl compare: {json.dumps(ccl_cmp)}")

    # ---- measured peaks (microbenchmarks, same run) --------------------------------
    peaks = _measured_peaks(torch, stream)
    _log(f"measured peaks: {peaks}")

    traffic = _traffic_per_unit()
    ccl_ms = stage_ms["ccl"] + stage_ms["ccl_link"]
    rooflines = {
        "ccl": _hbm_roof("labelling + linking (k_ccl_tile, k_ccl_boundary, k_ccl_pairs, k_ccl_flatten), one frame",
                         8.0 * v_stage + 64.0 * bricks, ccl_ms, peaks, traffic.get("ccl"),
                         f"8 B per occupied voxel x {v_stage:.0f} + 64 B per touched 8^3 brick x {bricks}"),
        "insert": _hbm_roof("grouped insert (k_vox_bucket, scan, k_bucket_scatter, k_bucket_insert), one frame",
                            12.0 * sc.n_points + 64.0 * touched, stage_ms["insert"], peaks, traffic.get("insert"),
                            f"12 B per point x {sc.n_points} + 64 B per touched voxel x {touched:.0f}"),
        "group": _hbm_roof("grouping (scan, sort, gather), one frame", 24.0 * kept, stage_ms["group"], peaks,
                           traffic.get("group"), f"24 B per kept voxel x {kept:.0f}"),
        "count": _alu_roof(tests, count_ms, peaks, traffic.get("count"),
                           f"{n_pts} points x {H} hypotheses (the last stage frame's clusters)",
                           "inlier counting: k_count_small (a wave per cluster of <= %d points) + k_count (tiles)"
                           % vm.get_count_config()["wave_max_points"]),
    }
    roof = dict(rooflines["ccl"])

    # ---- batched clusters: 2000 log-uniform clusters, one pass, graph replays ------
    batched = None
    if not args.no_batched:
        batched = _batched(vm, torch, dev, stream, peaks=peaks)
        _log(f"batched: {json.dumps(batched)}")

    # ---- served: 8 robots, Poisson arrivals, continuous admission ---------------
    served = None
    if not args.no_served:
        served = _served(vm, torch, args.served_seconds)
        _log(f"served: {json.dumps(served)}")

    # ---- stress: 0.005 m, 800x800x400 cells, 8M points per frame -----------------
    stress = None
    if not args.no_stress:
        stress = _stress(vm, torch, dev, stream, with_oracle=not args.no_cpu_baseline)
        _log(f"stress: {json.dumps(stress)}")

    # ---- cluster-level parallelism: 1..16 clusters of 10k..30k points -------------
    ablation = None
    if not args.no_ablation:
        ablation = _cluster_ablation(vm, torch, dev, stream)
        _log(f"cluster ablation: {json.dumps(ablation)}")

    # ---- ray-cast clearing: physically consistent frames, clear + insert + segment --
    clearing = None
    if not args.no_clearing:
        clearing = _clearing(vm, torch, dev, stream)
        _log(f"clearing: {json.dumps(clearing)}")

    # ---- the oracle on the host, bounded sample ---------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(sc, args.prewarm, args.cpu_frames, H, eps, minc, seed)
        if stress and "oracle_ms_per_frame_all_cores" in stress:
            cpu["stress_frame_ms_all_cores"] = stress.pop("oracle_ms_per_frame_all_cores")
        _log(f"cpu baseline: {json.dumps(cpu)}")

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
                                             "areas, polygon offsets and status words",
                           occupied_at_end=lat_occ),
        "plane_iou": iou,
        "stage_ms_per_frame": stage_ms,
        "roofline": roof,
        "rooflines": rooflines,
        "measured_peaks": peaks,
        "batched": batched,
        "served": served,
        "stress": stress,
        "clearing": clearing,
        "ccl_compare": ccl_cmp,
        "cluster_ablation": ablation,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


# ---------------------------------------------------------------------------
# rooflines and measured peaks
# ---------------------------------------------------------------------------
def _touched_bricks(keys: np.ndarray, dims) -> int:
    """Distinct 8x8x8 bricks holding an occupied voxel."""
    k = keys.astype(np.int64)
    nx, ny = int(dims[0]), int(dims[1])
    x, y, z = k % nx, (k // nx) % ny, k // (nx * ny)
    bx, by = (nx + 7) // 8, (ny + 7) // 8
    return int(np.unique((x // 8) + bx * ((y // 8) + by * (z // 8))).size)


def _hbm_roof(kernel, alg_bytes, ms, peaks, traffic, per_unit):
    ach = alg_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic, "kernel": kernel, "algorithmic_bytes": alg_bytes, "ms": ms,
            "work_per_launch": per_unit,
            "measured_peak": peaks.get("copy_gbs"), "frac_of_measured": ach / peaks["copy_gbs"]
            if peaks.get("copy_gbs") else None}


def _alu_roof(tests, ms, peaks, traffic, per_unit, kernel):
    tflops = tests * FLOP_PER_TEST / (ms * 1e-3) / 1e12
    tt = tests / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tflops / FP32_PEAK_TFLOPS, "traffic": traffic, "kernel": kernel, "ms": ms,
            "work_per_launch": per_unit, "tests_per_s": tt * 1e12,
            "peak_derivation": f"published fp32 vector peak; an inlier test counted as {FLOP_PER_TEST} flop "
                               "(three fused multiply-adds), i.e. %.1f T tests/s" % COUNT_PEAK_TTESTS,
            "measured_test_loop_peak_tests_per_s": peaks.get("test_loop_tests_per_s"),
            "frac_of_measured_test_loop": tt * 1e12 / peaks["test_loop_tests_per_s"]
            if peaks.get("test_loop_tests_per_s") else None}


def _measured_peaks(torch, stream) -> dict:
    """Attainable peaks measured in this run: a streaming copy (HBM), an
    independent fp32 fma loop, and a register-resident loop of the inlier
    test exactly as the counting kernels issue it (libvm_peaks.so)."""
    if not os.path.exists(PEAKS_LIB):
        return {}
    L = ctypes.CDLL(PEAKS_LIB)
    sink = torch.zeros(1 << 16, dtype=torch.float32, device="cuda")
    P = ctypes.c_void_p
    s = P(stream.cuda_stream)

    def timed(f, reps=5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            assert f() == 0
            stream.synchronize()
            e0.record(stream)
            for _ in range(reps):
                f()
            e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    blocks, it = 8192, 4096
    t_fma = timed(lambda: L.vmp_fma_loop(blocks, it, P(sink.data_ptr()), s))
    t_test = timed(lambda: L.vmp_test_loop(blocks, 1024, ctypes.c_float(0.01), P(sink.data_ptr()), s))
    n = 1 << 30
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    t_copy = timed(lambda: L.vmp_copy(P(a.data_ptr()), P(b.data_ptr()), ctypes.c_uint64(n // 16), 32768, s))
    del a, b
    return {"fma_loop_tflops": 2.0 * blocks * 256 * 8 * it / t_fma / 1e12,
            "test_loop_tests_per_s": blocks * 256 * 16 * 1024 / t_test,
            "copy_gbs": 2.0 * n / t_copy / 1e9,
            "note": "fma loop: independent v_fma_f32 chains; test loop: the counting kernels' inlier test on "
                    "register-resident points and wave-uniform planes; copy: 1 GiB read + 1 GiB written"}


# ---------------------------------------------------------------------------
# batched clusters (2000 log-uniform clusters)
# ---------------------------------------------------------------------------
def _batched(vm, torch, dev, stream, replays: int = 100, peaks=None):
    """2000 clusters of log-uniform size (50..200k points, about 48.5M in all),
    1024 hypotheses: planes and polygons of all clusters per frame.  Forms:
    two-pass (vm_ransac_planes + vm_hulls, a dozen dependent launches) and
    persistent (vm_planes_hulls: one preparation, one persistent launch, the
    tail chain, one pack); the persistent form's split is autotuned, the frame
    captured as a graph and replayed `replays` times with the frame number
    advanced in device memory (the data stays resident)."""
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

    def two_pass(f):
        vm.ransac_planes(cl, vm.ransac_params(H, 0.01, 0x5EED, f), planes, work, stream=stream)
        vm.hulls(cl, planes, hulls, work, stream=stream)

    def fused(f):
        vm.planes_hulls(cl, vm.ransac_params(H, 0.01, 0x5EED, f), planes, hulls, work, stream=stream)

    def per_frame(fn, reps=3):
        fn(0)
        stream.synchronize()
        t_s = time.perf_counter()
        for f in range(reps):
            fn(f)
        stream.synchronize()
        return 1e3 * (time.perf_counter() - t_s) / reps

    def stages(fn, reps=3):
        vm.set_stage_timing(True)
        for f in range(reps):
            fn(f)
        stream.synchronize()
        ms, _ = vm.stage_times()
        vm.set_stage_timing(False)
        return {name: float(ms[j]) / reps for j, name in enumerate(vm.STAGES) if ms[j] > 0}

    with torch.cuda.stream(stream):
        vm.set_fused_config(None)
        two_ms = per_frame(two_pass)
        two_st = stages(two_pass)
        fused_ms = per_frame(fused)
        t_s = time.perf_counter()
        tuned = vm.autotune_fused(cl, vm.ransac_params(H, 0.01, 0x5EED, 0), planes, hulls, work, stream=stream,
                                  reps=2)
        tune_s = time.perf_counter() - t_s
        tuned_ms = per_frame(fused)
        fused_st = stages(fused)
        with vm.capture(stream) as cap:
            vm.planes_hulls(cl, vm.ransac_params(H, 0.01, 0x5EED, d_frame=frame_t), planes, hulls, work,
                            stream=stream)
        cap.graph.launch(stream)
        stream.synchronize()
        t_s = time.perf_counter()
        for f in range(replays):
            frame_t.fill_(f)
            cap.graph.launch(stream)
        stream.synchronize()
        graph_ms = 1e3 * (time.perf_counter() - t_s) / replays
        vm.set_fused_config(None)
    cap.graph.close()
    tests = float(N) * H
    st = int(planes.status.cpu()[0]) | int(hulls.status.cpu()[0])
    del keep
    count_ms = two_st.get("count", 0.0)
    return {"workload": f"{K} clusters, log-uniform 50..200k points ({N} in all), {H} hypotheses, "
                        "planes + polygons of all clusters per frame",
            "ms_per_frame_graph": graph_ms, "replays": replays,
            "ms_per_frame_persistent": tuned_ms, "ms_per_frame_persistent_default_split": fused_ms,
            "ms_per_frame_two_pass": two_ms,
            "tests_per_s_graph": tests / (graph_ms * 1e-3),
            "stage_ms_two_pass": two_st, "stage_ms_persistent": fused_st,
            "autotune": {"config": tuned, "tuning_s": tune_s},
            "roofline_persistent_frame": _alu_roof(tests, graph_ms, peaks or {}, _traffic_per_unit().get("fused"),
                                                   f"{N} points x {H} hypotheses, whole frame",
                                                   "persistent planes + polygons (graph replay)"),
            "roofline_count_two_pass": _alu_roof(tests, count_ms, peaks or {}, None, f"{N} points x {H} hypotheses",
                                                 "inlier counting of the two-pass form (k_count_small + k_count)")
            if count_ms else None,
            "status_flags": st, "generation_s": gen_s}


# ---------------------------------------------------------------------------
# served: 8 robots, Poisson arrivals at 30 Hz, U(200k, 2M)-point posed frames
# ---------------------------------------------------------------------------
def _served(vm, torch, seconds: float, n_robots: int = 8, rate_hz: float = 30.0, warm_frames: int = 30,
            speedup: float = 5.0):
    """Robot r maps the full-map scene with scene seed 10 + r into its own map
    (2^24 slots), warmed with `warm_frames` 1M-point frames (about 2M occupied
    voxels).  Frames arrive as Poisson processes at `rate_hz` per robot over
    `seconds`; a frame has U(200k, 2M) points -- a random window of the
    robot's 8M-sample surface pool plus fresh outliers -- seen from its own
    pose of a 6-DoF random walk.  The same trace runs three times from the
    warmed maps: served (continuous admission, one stream per robot),
    one frame at a time on one stream (the plain form), and served again with
    the arrival times divided by `speedup` (a saturating rate)."""
    import scenes
    from paper_2510_01592_amd.serve import GpuBackend, Request, Scheduler, latency_summary
    t0 = time.perf_counter()
    scs = [scenes.scene_full_map(10 + r) for r in range(n_robots)]
    pools = [scenes.surface_pool(sc, 30 + r, 8_000_000) for r, sc in enumerate(scs)]
    trace = scenes.served_trace(n_robots, seconds, rate_hz, seed=20)
    # frames in the sensor frame of their poses, in pinned host memory
    with concurrent.futures.ThreadPoolExecutor(max_workers=HOST_THREADS) as ex:
        host = list(ex.map(lambda f: scenes.stream_frame(scs[f.robot], pools[f.robot], f.frame_seed, f.n_points,
                                                         f.pose), trace))
    pinned = []
    for h in host:
        t = torch.empty(h.shape, dtype=torch.float32, pin_memory=True)
        t.numpy()[:] = h
        pinned.append(t)
    del host
    gen_s = time.perf_counter() - t0
    maps, snaps = [], []
    s = torch.cuda.Stream()
    for r, sc in enumerate(scs):
        g = sc.geom
        mp = vm.Map(g.origin, g.voxel_size, g.dims, 24)
        with torch.cuda.stream(s):
            for f in range(warm_frames):
                pts = scenes.stream_frame(sc, pools[r], 900_000 + 100 * r + f, 1_000_000)
                mp.insert(torch.from_numpy(pts).cuda(), stream=s)
        s.synchronize()
        snaps.append(mp.export(stream=s))
        maps.append(mp)
    warm_occ = [int(sn[0].shape[0]) for sn in snaps]
    del pools
    n_slots, budget = 16, 8 << 30
    # an accumulating map's outliers form thousands of small clusters: room for 65536 per frame
    be = GpuBackend(maps, n_slots=n_slots, n_hyp=512, k_cap=65536)
    be_b = GpuBackend(maps, n_slots=n_slots, n_hyp=512, k_cap=65536, batch=True, batch_k_cap=65536,
                      batch_n_cap=1 << 26)

    def reset():
        with torch.cuda.stream(s):
            for mp, sn in zip(maps, snaps):
                mp.import_(sn[0], sn[1], sn[2], stream=s)
        s.synchronize()

    def requests(scale):
        return [Request(f.robot, f.seq, f.arrival / scale, f.n_points, (pinned[i], f.pose[0], f.pose[1]))
                for i, f in enumerate(trace)]

    # one untimed frame per robot in each form (allocates each map's workspace)
    first = [Request(r, 0, 0.0, 200_000, (pinned[i][:200_000], f.pose[0], f.pose[1]))
             for r in range(n_robots) for i, f in enumerate(trace) if f.robot == r and f.seq == 0]
    for b in (be, be_b):
        reset()
        Scheduler(b, n_robots, n_slots, budget).run(first)

    def run(scale, per_robot, slots, label, backend=be):
        reset()
        sch = Scheduler(backend, n_robots, slots, budget, per_robot_inflight=per_robot)
        g0 = getattr(backend, "groups", 0)
        torch.cuda.synchronize()
        t_s = time.perf_counter()
        done = sch.run(requests(scale), t0=t_s)
        t_span = time.perf_counter() - t_s
        summ = latency_summary(done, t_span)
        vox = sum(c.result["occupied"] for c in done)
        occ_end = max(c.result["occupied"] for c in done)
        bad = sum(1 for c in done if c.result["status"].any())
        flags = {}
        for c in done:
            f = int(np.bitwise_or.reduce(c.result["status"].astype(np.uint32)))
            for bit, name in ((1, "hash_full"), (2, "clusters_cap"), (4, "inliers_cap"), (8, "hull_cap"),
                              (16, "bad_clusters")):
                if f & bit:
                    flags[name] = flags.get(name, 0) + 1
        out = dict(summ, wall_s=t_span, voxels_per_s=vox / t_span,
                   points_per_s=sum(c.request.n_points for c in done) / t_span, peak_inflight=sch.peak_inflight,
                   rejected=len(sch.rejected), frames_with_status_flags=bad, status_flag_counts=flags,
                   max_occupied=occ_end)
        if sch.batches:
            out["batches"] = sch.batches
            out["mean_batch"] = sch.batched_frames / sch.batches
            out["persistent_passes"] = getattr(backend, "groups", 0) - g0
        _log(f"served [{label}]: {out}")
        return out, {(c.request.robot, c.request.seq): c.result for c in done}

    served, res_a = run(1.0, 2, n_slots, "served (streams), 30 Hz")
    batched, res_c = run(1.0, 2, n_slots, "served (batched), 30 Hz", be_b)
    one, res_b = run(1.0, 1, 1, "one at a time, 30 Hz")
    fast, _ = run(speedup, 2, n_slots, f"served (streams), x{speedup:g}")
    fast_b, _ = run(speedup, 2, n_slots, f"served (batched), x{speedup:g}", be_b)
    fast_one, _ = run(speedup, 1, 1, f"one at a time, x{speedup:g}")
    # the same frames give the same results in every schedule (bit patterns:
    # a NaN compares equal to itself)
    def differ(x, y):
        return [k for k in x if not (x[k]["K"] == y[k]["K"] and x[k]["N"] == y[k]["N"] and
                                     np.array_equal(x[k]["best"], y[k]["best"]) and
                                     np.array_equal(x[k]["nin"], y[k]["nin"]) and
                                     np.array_equal(x[k]["plane"].view(np.uint32), y[k]["plane"].view(np.uint32)) and
                                     np.array_equal(x[k]["area"].view(np.uint64), y[k]["area"].view(np.uint64)) and
                                     np.array_equal(x[k]["v_off"], y[k]["v_off"]))]
    diff_b, diff_c = differ(res_a, res_b), differ(res_a, res_c)
    for name, dk in (("one at a time", diff_b), ("batched", diff_c)):
        for k in dk[:3]:
            x, y = res_a[k], (res_b if name == "one at a time" else res_c)[k]
            kk = min(x["K"], y["K"])
            bad = [c for c in range(kk) if x["best"][c] != y["best"][c] or
                   x["plane"][c].view(np.uint32).tolist() != y["plane"][c].view(np.uint32).tolist() or
                   x["area"][c].view(np.uint64) != y["area"][c].view(np.uint64) or
                   x["v_off"][c + 1] - x["v_off"][c] != y["v_off"][c + 1] - y["v_off"][c]]
            first = ""
            if bad:
                c = bad[0]
                first = (f"; {len(bad)} clusters, first {c}: best {x['best'][c]} / {y['best'][c]}, inliers "
                         f"{x['nin'][c]} / {y['nin'][c]}, area "
                         f"{x['area'][c]!r} / {y['area'][c]!r}, vertices {x['v_off'][c + 1] - x['v_off'][c]} / "
                         f"{y['v_off'][c + 1] - y['v_off'][c]}")
            _log(f"served: frame {k} differs from the streams form in the {name} form: K {x['K']} / {y['K']}, "
                 f"N {x['N']} / {y['N']}, occupied {x['occupied']} / {y['occupied']}{first}")
    same = not diff_b and not diff_c
    for mp in maps:
        mp.close()
    return dict(served, robots=n_robots, rate_hz_per_robot=rate_hz, arrival_span_s=seconds,
                frames_in_trace=len(trace), points_per_frame="U(200k, 2M)", n_hyp=512, slots=n_slots,
                budget_mib=budget >> 20, warm_occupied=warm_occ,
                form="streams: one vm_segment_frame per frame on its robot's stream",
                batched=dict(batched, form="continuous batching: frames admitted together share one "
                                           "vm_planes_hulls_multi pass"),
                one_at_a_time=one, saturating={"rate_hz_per_robot": rate_hz * speedup, "served": fast,
                                               "batched": fast_b, "one_at_a_time": fast_one},
                results_equal_in_every_form=bool(same),
                frames_differing={"one_at_a_time": len(diff_b), "batched": len(diff_c)}, generation_s=gen_s)


# ---------------------------------------------------------------------------
# stress: 0.005 m voxels, 800x800x400 cells, 8M points per frame
# ---------------------------------------------------------------------------
def _stress(vm, torch, dev, stream, warm: int = 5, timed: int = 5, with_oracle: bool = True):
    """The stress scene (floor, staircase, two tables, 500 floating boxes) at
    0.005 m: `warm` 8M-point frames warm the map, then `timed` frames run the
    whole path (1024 hypotheses) one at a time from pinned host memory
    (latency = H2D of the frame -> results in host memory)."""
    import scenes
    t0 = time.perf_counter()
    sc = scenes.scene_stress(5)
    g = sc.geom
    H = sc.n_hyp
    with concurrent.futures.ThreadPoolExecutor(max_workers=HOST_THREADS) as ex:
        warm_pts = list(ex.map(lambda f: scenes.frame_points(sc, 100 + f), range(warm)))
        timed_pts = list(ex.map(lambda f: scenes.frame_points(sc, 200 + f), range(timed)))
    gen_s = time.perf_counter() - t0
    m = vm.Map(g.origin, g.voxel_size, g.dims, 25)
    with torch.cuda.stream(stream):
        for p in warm_pts:
            m.insert(torch.from_numpy(p).to(dev), stream=stream)
    stream.synchronize()
    warm_occ = int(m.stats(stream).occupied)
    k_cap = 1 << 16
    planes = vm.PlaneBuffers.alloc(k_cap, 1 << 24, H)
    hulls = vm.HullBuffers.alloc(k_cap, 1 << 22)
    stage = torch.empty((sc.n_points, 3), dtype=torch.float32, device=dev)
    res = torch.empty(2, dtype=torch.int32).pin_memory()
    res_area = torch.empty(k_cap, dtype=torch.float64).pin_memory()
    host = [torch.from_numpy(p).pin_memory() for p in timed_pts]
    kw = dict(min_cluster=sc.min_cluster, n_hyp=H, eps=sc.eps, seed=0x5EED)
    lat, occ, kk = [], [], []
    stats = torch.zeros(vm.STATS_WORDS, dtype=torch.int64, device=dev)
    with torch.cuda.stream(stream):
        # an untimed first frame (allocates the map's workspace)
        stage.copy_(host[0], non_blocking=True)
        m.segment_frame(stage, planes, hulls, frame=0, stream=stream, **kw)
        stream.synchronize()
        for i, hf in enumerate(host):
            stream.synchronize()
            ta = time.perf_counter()
            stage.copy_(hf, non_blocking=True)
            cl = m.segment_frame(stage, planes, hulls, frame=1 + i, stream=stream, **kw)
            res[0:1].copy_(planes.status, non_blocking=True)
            res[1:2].copy_(hulls.status, non_blocking=True)
            res_area.copy_(hulls.area, non_blocking=True)
            stream.synchronize()
            lat.append(1e3 * (time.perf_counter() - ta))
            m.stats_async(stats, stream=stream)
            occ.append(int(stats.cpu()[0]))
            kk.append(vm.read_clusters(cl)["K"])
    vm.set_stage_timing(True)
    with torch.cuda.stream(stream):
        m.segment_frame(stage, planes, hulls, frame=99, stream=stream, **kw)
        stream.synchronize()
    ms, _ = vm.stage_times()
    vm.set_stage_timing(False)
    out = {"workload": "stress: 4x4x2 m at 0.005 m (800x800x400 cells), floor + staircase + 2 tables + 500 floating "
                       "boxes, 8M float32 points/frame, N(0,1.5 mm), 5% outliers, 1024 hypotheses, min cluster 30",
           "warm_frames": warm, "occupied_after_warm": warm_occ, "timed_frames": timed,
           "occupied_per_frame": occ, "clusters_per_frame": kk,
           "ms_per_frame": float(np.mean(lat)), "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99),
           "voxels_per_s": float(np.sum(occ)) / (np.sum(lat) * 1e-3),
           "latency_includes": "H2D of the 96 MB frame from pinned host memory, the frame, D2H of status and areas",
           "stage_ms_one_frame": {name: float(ms[j]) for j, name in enumerate(vm.STAGES)},
           "status_flags": int(res[0]) | int(res[1]), "generation_s": gen_s}
    if with_oracle:
        import oracle
        om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
        for p in warm_pts + timed_pts[:1]:
            om.insert(p)
        t_s = time.perf_counter()
        oracle.segment(om, sc.min_cluster, H, sc.eps, 0x5EED, 1, threads=HOST_THREADS)
        out["oracle_ms_per_frame_all_cores"] = {"ms": 1e3 * (time.perf_counter() - t_s), "threads": HOST_THREADS,
                                                "occupied": int(len(om.key))}
    m.close()
    return out


# ---------------------------------------------------------------------------
# rocprofv3 counters: HBM traffic per kernel
# ---------------------------------------------------------------------------
def _plane_iou(vm, sc, planes, hulls, cl, max_tilt_deg: float = 90.0) -> dict:
    """The analogue of Table I's IoU: every ground-truth rectangle lying wholly
    inside the grid (and tilted at most max_tilt_deg from horizontal) against
    the detected polygons (best match with a normal within 10 degrees and the
    plane within 5 cm of the rectangle's centre)."""
    import scenes
    K = int(vm.read_clusters(cl)["K"])
    K = min(K, planes.k_cap, hulls.k_cap)
    P = planes.plane[:K].cpu().numpy().astype(np.float64)
    voff = hulls.v_off[:K + 1].cpu().numpy().astype(np.int64)
    vxyz = hulls.v_xyz[:max(int(voff[-1]) if K else 0, 1)].cpu().numpy().astype(np.float64)
    polys = [vxyz[voff[k]:voff[k + 1]] for k in range(K)]
    lo, hi = np.asarray(sc.geom.origin), sc.geom.hi
    cos_tilt = np.cos(np.deg2rad(max_tilt_deg)) - 1e-12
    rects = [r for r in sc.rects if np.all((r.corners() >= lo) & (r.corners() < hi)) and abs(r.normal[2]) >= cos_tilt]
    v = scenes.plane_iou(rects, P, polys)
    return {"mean": float(v.mean()) if len(v) else None, "min": float(v.min()) if len(v) else None,
            "rects": len(rects), "rects_over_0_5": int((v > 0.5).sum()), "planes": K}


def _ccl_compare(vm, m, stream, reps: int = 5) -> dict:
    """The map's labelling and grouping by union-find (vm_ccl) and by Alg. 1's
    label propagation (vm_ccl_propagate, the host checking between batches of
    sweeps); both give the same clusters."""
    occ = int(m.stats(stream).occupied)
    out = {"occupied": occ}
    for name, fn in (("union_find", lambda: m.ccl(30, stream=stream)),
                     ("label_propagation", lambda: m.ccl_propagate(30, stream=stream))):
        fn()
        stream.synchronize()
        t_s = time.perf_counter()
        r = None
        for _ in range(reps):
            r = fn()
        stream.synchronize()
        out[name] = {"ms": 1e3 * (time.perf_counter() - t_s) / reps}
        if name == "label_propagation":
            out[name]["sweeps"] = r[1]
            out[name]["clusters"] = int(vm.read_clusters(r[0])["K"])
        else:
            out[name]["clusters"] = int(vm.read_clusters(r)["K"])
    out["speedup_union_find"] = out["label_propagation"]["ms"] / out["union_find"]["ms"]
    return out


def _cluster_ablation(vm, torch, dev, stream, runs: int = 1000, n_hyp: int = 100) -> dict:
    """Cluster-level parallelism (the paper's ablation of Sec. IV-C): sets of
    1, 2, 4, 8 and 16 clusters of 10k..30k points (log-uniform), planes and
    polygons of all clusters of a set in one call (vm_planes_hulls) against
    one call per cluster in turn, each timed as the mean of `runs` runs with
    I = 100 hypotheses."""
    import scenes
    out = {"workload": f"1..16 clusters of 10k..30k points, {n_hyp} hypotheses, mean of {runs} runs", "sets": []}
    for nc in (1, 2, 4, 8, 16):
        off, xyz = scenes.batched_clusters(seed=50 + nc, n_clusters=nc, n_min=10_000, n_max=30_000)
        N = len(xyz)
        cl, keep = vm.clusters_from_host(off, xyz, np.arange(nc, dtype=np.uint32))
        singles = [vm.clusters_from_host(off[k:k + 2] - off[k], xyz[off[k]:off[k + 1]],
                                         np.array([k], dtype=np.uint32)) for k in range(nc)]
        work = torch.empty(vm.workspace_bytes(nc, N, n_hyp), dtype=torch.uint8, device=dev)
        planes = vm.PlaneBuffers.alloc(nc, N, n_hyp)
        hulls = vm.HullBuffers.alloc(nc, N)
        with torch.cuda.stream(stream):
            def together(f):
                vm.planes_hulls(cl, vm.ransac_params(n_hyp, 0.01, 0x5EED, f), planes, hulls, work, stream=stream)

            def one_by_one(f):
                for c, _k in singles:
                    vm.planes_hulls(c, vm.ransac_params(n_hyp, 0.01, 0x5EED, f), planes, hulls, work, stream=stream)

            res = {}
            for name, fn in (("all_clusters_one_call_ms", together), ("one_call_per_cluster_ms", one_by_one)):
                fn(0)
                stream.synchronize()
                t_s = time.perf_counter()
                for f in range(runs):
                    fn(f)
                stream.synchronize()
                res[name] = 1e3 * (time.perf_counter() - t_s) / runs
        del keep, singles
        out["sets"].append({"clusters": nc, "points": N, **res,
                            "speedup": res["one_call_per_cluster_ms"] / res["all_clusters_one_call_ms"]})
    return out


def _clearing(vm, torch, dev, stream, n_distinct: int = 4, timed: int = 12):
    """Sec. III-B's clearing on the full map: frames ray-cast from a sensor
    about 1 m above the floor (each return the first surface hit, 5 % spurious
    early returns), 1M points each; the map is segmented every frame with and
    without VM_SEG_CLEAR_RAYS.  Reports the clearing stage's device time, the
    frame time of both forms and how the occupied count evolves."""
    import scenes
    sc = scenes.scene_full_map(1)
    g = sc.geom
    t_gen = time.perf_counter()
    poses = scenes.random_walk_poses(41, n_distinct, sigma_t=0.05, sigma_rot_deg=2.0)
    lift = np.array([0.0, 0.0, 1.0])
    frames = []
    for f, (R, t) in enumerate(poses):
        tt = t + lift
        pts = scenes.raycast_frame(sc, tt, 600 + f, sc.n_points, pose=(R, tt))
        frames.append((torch.from_numpy(pts).to(dev), R, tt))
    gen_s = time.perf_counter() - t_gen
    H, eps, minc = sc.n_hyp, sc.eps, sc.min_cluster
    planes = vm.PlaneBuffers.alloc(16384, 1 << 23, H)
    hulls = vm.HullBuffers.alloc(16384, 1 << 22)
    out = {"workload": f"full map 400x400x200 at 0.01 m, {n_distinct} ray-cast frames of {sc.n_points} points "
                       f"(sensor 1 m above the floor, random-walk poses) repeated, {timed} timed frames after "
                       f"{n_distinct} warm-up frames", "generation_s": gen_s}
    for clear in (True, False):
        m = vm.Map(g.origin, g.voxel_size, g.dims, 23)
        occ = []
        with torch.cuda.stream(stream):
            for f in range(n_distinct):
                pts, R, t = frames[f]
                m.segment_frame(pts, planes, hulls, R, t, min_cluster=minc, n_hyp=H, eps=eps, frame=f,
                                stream=stream, clear=clear)
            stream.synchronize()
            ta = time.perf_counter()
            for i in range(timed):
                pts, R, t = frames[i % n_distinct]
                m.segment_frame(pts, planes, hulls, R, t, min_cluster=minc, n_hyp=H, eps=eps, frame=100 + i,
                                stream=stream, clear=clear)
            stream.synchronize()
            frame_ms = 1e3 * (time.perf_counter() - ta) / timed
            vm.set_stage_timing(True)
            for i in range(4):
                pts, R, t = frames[i % n_distinct]
                m.segment_frame(pts, planes, hulls, R, t, min_cluster=minc, n_hyp=H, eps=eps, frame=200 + i,
                                stream=stream, clear=clear)
                occ.append(int(m.stats(stream).occupied))
            ms, _ = vm.stage_times()
            vm.set_stage_timing(False)
        st = m.stats(stream)
        key = "with_clearing" if clear else "without_clearing"
        out[key] = {"frame_ms": frame_ms, "stage_ms": {n: float(ms[j]) / 4 for j, n in enumerate(vm.STAGES)},
                    "occupied_last_frames": occ, "voxels_cleared_total": int(st.voxels_cleared),
                    "frames_total": n_distinct + timed + 4}
        if clear:
            c_ms = out[key]["stage_ms"]["clear"]
            out[key]["rays_per_s"] = sc.n_points / (c_ms * 1e-3) if c_ms > 0 else None
        m.close()
    return out


def _sha256(path: str) -> str:
    """SHA-256 of a kernel file followed by the headers it shares with the others."""
    h = hashlib.sha256()
    for q in [path] + [os.path.join(os.path.dirname(path), x) for x in SHARED_HEADERS]:
        with open(q, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counters_run(vm, torch, m, frames, planes, hulls, k_cap, H, eps, seed, kw, stream, dev, restore, first, n):
    """The launches the rooflines are measured on -- n frames, then 10
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
        # three persistent passes over the 2000-cluster set
        import scenes
        off, xyz = scenes.batched_clusters(seed=3)
        K2, N2, H2 = len(off) - 1, len(xyz), 1024
        cl2, keep = vm.clusters_from_host(off, xyz, np.arange(K2, dtype=np.uint32))
        work2 = torch.empty(vm.workspace_bytes(K2, N2, H2), dtype=torch.uint8, device=dev)
        pl2, hl2 = vm.PlaneBuffers.alloc(K2, N2, H2), vm.HullBuffers.alloc(K2, N2)
        for r in range(3):
            vm.planes_hulls(cl2, vm.ransac_params(H2, 0.01, 0x5EED, r), pl2, hl2, work2, stream=stream)
        # the reference: a plain copy kernel over COPY_BYTES (libvm_peaks.so's k_copy),
        # and the register-only loop of the inlier test (instruction counters per test)
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        stream.synchronize()
        PL = ctypes.CDLL(PEAKS_LIB)
        assert PL.vmp_test_loop(2048, 256, ctypes.c_float(0.01), ctypes.c_void_p(dst.data_ptr()),
                                ctypes.c_void_p(stream.cuda_stream)) == 0
        assert PL.vmp_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                           ctypes.c_uint64(COPY_BYTES // 16), 32768, ctypes.c_void_p(stream.cuda_stream)) == 0
        stream.synchronize()
        del keep
    meta = vm.read_clusters(cl)
    print(json.dumps({"counters_run": True, "frames": n, "count_passes": 10, "points": int(meta["N"]),
                      "clusters": int(meta["K"]), "n_hyp": H, "persistent_passes": 3, "persistent_points": N2,
                      "copy_bytes": COPY_BYTES}), flush=True)
    return 0


def _pmc_rows(path: str):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _traffic_from(fetch_csv: str, write_csv: str) -> int:
    """HBM bytes per dispatch of every kernel of a --counters run: FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch) each scaled by what the same counter
    reads for the 256 MiB copy.  The counting kernels are averaged over the
    10 standalone passes (their last 10 dispatches), the others over the
    run's frames.  Each unit keeps the SHA-256 of its source file, so the
    bench reports the figure only while the kernels are unchanged."""
    out = {"units": {}, "kernels": {}}
    per = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        rows = _pmc_rows(path)
        cnt = "FETCH_SIZE" if name == "fetch" else "WRITE_SIZE"
        rows = [r for r in rows if r["Counter_Name"] == cnt]
        cp = max(float(r["Counter_Value"]) for r in rows if "k_copy" in r["Kernel_Name"])
        scale = COPY_BYTES / (cp * 1024.0)
        out[f"{name}_copy_kib_raw"] = cp
        out[f"{name}_scale"] = scale
        by = {}
        for r in rows:
            kn = r["Kernel_Name"]
            short = kn.replace("(anonymous namespace)::", "").split("(")[0].split("::")[-1].split("<")[0].strip()
            by.setdefault(short, []).append(float(r["Counter_Value"]) * 1024.0 * scale)
        for short, v in by.items():
            if short in ("k_count", "k_count_small"):
                v = v[-10:]
            per.setdefault(short, {})[name] = float(np.mean(v))
            per[short]["dispatches"] = len(v)
    out["kernels"] = per
    for unit, (kernels, src) in UNITS.items():
        if all(k in per for k in kernels):
            f = sum(per[k]["fetch"] for k in kernels)
            w = sum(per[k]["write"] for k in kernels)
            out["units"][unit] = {"kernels": kernels, "fetch_bytes": f, "write_bytes": w, "bytes": f + w,
                                  "source": os.path.relpath(os.path.join(CSRC, src), ROOT),
                                  "source_sha256": _sha256(os.path.join(CSRC, src))}
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["units"]), flush=True)
    return 0


def _traffic_per_unit() -> dict:
    """Measured HBM bytes per launch of each unit, for the units whose kernel
    source is unchanged since the counters were taken."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return {}
    out = {}
    for unit, u in t.get("units", {}).items():
        try:
            if u["source_sha256"] == _sha256(os.path.join(ROOT, u["source"])):
                out[unit] = float(u["bytes"])
        except (OSError, KeyError):
            pass
    return out


# ---------------------------------------------------------------------------
# the oracle on the host cores
# ---------------------------------------------------------------------------
def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _cpu_baseline(sc, prewarm, n_frames, H, eps, minc, seed):
    """The oracle (C, with numpy grouping) on the same workload: the warmed
    map is rebuilt untimed, then n_frames frames are inserted and segmented
    (all clusters), once on one thread and once with the clusters' planes and
    hulls spread over the host cores (identical results); plus one frame of
    the 2000-cluster batched set on all cores."""
    import oracle
    import scenes
    g = sc.geom
    frames = [scenes.frame_points(sc, 1000 + i) for i in range(n_frames)]
    res = {}
    for label, threads in (("single", 1), ("all_cores", HOST_THREADS)):
        om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
        for f in range(prewarm):
            om.insert(scenes.frame_points(sc, 2 + f))
        voxels = 0
        t0 = time.perf_counter()
        for i, pts in enumerate(frames):
            om.insert(pts)
            voxels += len(om.key)
            oracle.segment(om, minc, H, eps, seed, i, threads=threads)
        t = time.perf_counter() - t0
        res[label] = {"value": voxels / t, "s": t, "voxels": voxels, "threads": threads}
    off, xyz = scenes.batched_clusters(seed=3)
    t0 = time.perf_counter()
    oracle.planes_and_hulls(off, xyz, np.arange(len(off) - 1, dtype=np.uint32), 1024, 0.01, 0x5EED, 0,
                            threads=HOST_THREADS)
    batched_s = time.perf_counter() - t0
    a = res["all_cores"]
    return {"value": a["value"], "unit": "voxels/s", "cores": a["threads"], "kind": "oracle",
            "sample": f"{n_frames} frame(s) of the full-map workload after the same {prewarm}-frame warm-up "
                      f"({a['voxels']} occupied voxels segmented in {a['s']:.1f} s; labelling and grouping on one "
                      f"thread, planes and hulls of the clusters over {a['threads']} threads)",
            "single_thread": {"value": res["single"]["value"], "cores": 1, "s": res["single"]["s"]},
            "batched_frame_s_all_cores": batched_s,
            "host": {"nproc": os.cpu_count(), "threads_used": HOST_THREADS, "cpu_model": _cpu_model()}}


if __name__ == "__main__":
    sys.exit(main())

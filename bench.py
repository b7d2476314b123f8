#!/usr/bin/env python3
"""Benchmark: occupied voxels segmented per second, and frame latency, on the
full local map workload (4x4x2 m at 0.01 m = 400x400x200 cells, 1M float32
points per frame with N(0, 3 mm) noise and 5 % outliers, 512 RANSAC
hypotheses, clusters below 30 voxels dropped), on one MI355X.

A step is one frame of the whole path (vm_segment_frame): insert the frame
into the resident map, label all occupied voxels, group them, fit one plane
per cluster and outline it.  The map is first warmed with 30 frames (about
2M occupied voxels) and keeps growing by the outliers of each new frame, as
an accumulating map does; the metric sums the occupied voxels each step
segmented.  Frames are resident in HBM before the timed region starts.

Prints one JSON line (see the keys below)."""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "occupied voxels segmented/s and p50/p99 frame latency, plain vs batched/served @0.01 m"
HBM_PEAK_GBS = 8000.0


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
    args = ap.parse_args()

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

    sc = scenes.scene_full_map(1)
    g = sc.geom
    H, eps, minc, seed = sc.n_hyp, sc.eps, sc.min_cluster, 0x5EED
    m = vm.Map(g.origin, g.voxel_size, g.dims, 23)

    # ---- pre-warm the map (not timed) -------------------------------------
    t0 = time.perf_counter()
    for f in range(args.prewarm):
        m.insert(torch.from_numpy(scenes.frame_points(sc, 2 + f)).to(dev))
    torch.cuda.synchronize()
    v_prewarm = int(m.stats().occupied)
    _log(f"prewarm {args.prewarm} frames -> {v_prewarm} occupied voxels ({time.perf_counter() - t0:.1f}s)")

    n_frames = args.warmup + args.steps
    frames = [torch.from_numpy(scenes.frame_points(sc, 1000 + i)).to(dev) for i in range(n_frames)]
    k_cap = 16384
    planes = vm.PlaneBuffers.alloc(k_cap, 1 << 23, H)
    hulls = vm.HullBuffers.alloc(k_cap, 1 << 22)
    stats_dev = torch.zeros((n_frames + 1, 6), dtype=torch.int64, device=dev)

    last = {}

    def step(i: int) -> None:
        last["cl"] = m.segment_frame(frames[i], planes, hulls, min_cluster=minc, n_hyp=H, eps=eps, seed=seed,
                                     frame=i)
        m.stats_async(stats_dev[i])

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    _log(f"warmup {args.warmup} steps done")

    # ---- timed region: K steps back to back on one stream -------------------
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.warmup, n_frames):
        step(i)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    st = stats_dev.cpu().numpy()
    occ = st[args.warmup:n_frames, 0].astype(np.int64)       # occupied voxels segmented by each step
    voxels = int(occ.sum())
    value = voxels / t_total
    ms_per_step = 1e3 * t_total / args.steps
    _log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value / 1e6:.1f} M voxels/s, "
         f"occupied {occ[0]}..{occ[-1]}")

    # ---- per-stage device time (HIP events on the stream the kernels run on) --
    vm.set_stage_timing(True)
    n_stage = min(5, args.steps)
    for i in range(n_stage):
        step(args.warmup + i)
    torch.cuda.synchronize()
    ms, launches = vm.stage_times()
    vm.set_stage_timing(False)
    stage_ms = {name: float(ms[j]) / n_stage for j, name in enumerate(vm.STAGES)}
    _log("stage ms/frame: " + ", ".join(f"{k}={v:.3f}" for k, v in stage_ms.items()))

    # ---- frame latency: pinned host frame -> results in host memory ----------
    lat = []
    host_frames = [torch.from_numpy(scenes.frame_points(sc, 5000 + i)).pin_memory()
                   for i in range(min(args.latency_frames, 8))]
    res_plane = torch.empty((k_cap, 4), dtype=torch.float32).pin_memory()
    res_area = torch.empty(k_cap, dtype=torch.float64).pin_memory()
    res_voff = torch.empty(k_cap + 1, dtype=torch.int32).pin_memory()
    res_stat = torch.empty(2, dtype=torch.int32).pin_memory()
    dframe = torch.empty((sc.n_points, 3), dtype=torch.float32, device=dev)
    for i in range(args.latency_frames):
        hf = host_frames[i % len(host_frames)]
        torch.cuda.synchronize()
        ta = time.perf_counter()
        dframe.copy_(hf, non_blocking=True)
        last["cl"] = m.segment_frame(dframe, planes, hulls, min_cluster=minc, n_hyp=H, eps=eps, seed=seed,
                                     frame=10000 + i)
        res_plane.copy_(planes.plane, non_blocking=True)
        res_area.copy_(hulls.area, non_blocking=True)
        res_voff.copy_(hulls.v_off, non_blocking=True)
        res_stat[0:1].copy_(planes.status, non_blocking=True)
        res_stat[1:2].copy_(hulls.status, non_blocking=True)
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - ta))
    lat = np.array(lat)
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))
    _log(f"latency p50 {p50:.2f} ms p99 {p99:.2f} ms over {len(lat)} frames")

    # ---- roofline of the dominant kernel --------------------------------------
    # inlier counting: 3 fma + 1 abs-compare per point x hypothesis, all lanes
    # (vector ALU bound); its work per launch is sum_k n_k * H evaluations.
    cl_meta = vm.read_clusters(last["cl"])
    n_pts = cl_meta["N"]
    evals = float(n_pts) * H
    stage_name = max(stage_ms, key=stage_ms.get)
    roof = None
    insert_bytes = 12.0 * sc.n_points
    if stage_name == "count":
        # peak: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s; 4 ops per evaluation
        peak_geval = 256 * 64 * 2.4e9 / 4 / 1e9
        ach = evals / (stage_ms["count"] * 1e-3) / 1e9
        roof = {"bound": "alu", "achieved": ach, "peak": peak_geval, "unit": "Geval/s", "frac": ach / peak_geval,
                "traffic": None, "kernel": "k_count"}
    else:
        per = {"insert": insert_bytes}
        algo = per.get(stage_name)
        if algo is not None:
            ach = algo / (stage_ms[stage_name] * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                    "traffic": None, "kernel": stage_name}
        else:
            roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                    "traffic": None, "kernel": stage_name}

    # ---- the oracle on the host, bounded sample ---------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(sc, args.prewarm, args.cpu_frames, H, eps, minc, seed)
        _log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "full local map: 4x4x2 m at 0.01 m (400x400x200 cells), floor + 12-step open-tread "
                        "staircase + tabletop + 20 tilted patches, 1M float32 points/frame, N(0,3 mm), 5% outliers, "
                        "512 hypotheses, eps 0.01 m, min cluster 30",
            "form": "plain",
            "prewarm_frames": args.prewarm,
            "occupied_first_step": int(occ[0]),
            "occupied_last_step": int(occ[-1]),
            "points_per_frame": sc.n_points,
            "n_hyp": H,
        },
        "latency_ms": {"p50": p50, "p99": p99, "frames": len(lat),
                       "includes": "H2D of the frame from pinned host memory, vm_segment_frame, D2H of planes, "
                                   "areas, polygon offsets and status words"},
        "stage_ms_per_frame": stage_ms,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


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

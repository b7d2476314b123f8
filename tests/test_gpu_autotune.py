"""The counting decomposition (vm_count_config) and its autotuner: every
setting gives bit-identical RANSAC results (counts are integer sums of the same
tests), and the default setting matches the oracle.  Cluster sizes straddle
every threshold of the decomposition (3, 64-multiples up to 1024, the 4096-point
tiles) with ragged tails."""
import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_util import cluster_tensors, compare_cluster, hulls_np, note, planes_np

pytestmark = pytest.mark.gpu

SEED = 0x5EED
H = 256
EPS = 0.01
FRAME = 3
SIZES = [0, 1, 2, 3, 5, 63, 64, 65, 100, 191, 192, 193, 255, 256, 257, 500, 511, 512, 513, 767, 768, 769,
         1000, 1023, 1024, 1025, 2000, 4095, 4096, 4097, 9000, 17000]
CONFIGS = [
    dict(count_grid=16384, chunk_mult=2, wave_max_points=256, plane_max_points=256),   # the defaults
    dict(count_grid=4096, chunk_mult=2, wave_max_points=1024, plane_max_points=256),
    dict(count_grid=4096, chunk_mult=2, wave_max_points=0, plane_max_points=0),        # all tiled
    dict(count_grid=4096, chunk_mult=2, wave_max_points=1024, plane_max_points=0),
    dict(count_grid=4096, chunk_mult=2, wave_max_points=512, plane_max_points=64),
    dict(count_grid=4096, chunk_mult=2, wave_max_points=256, plane_max_points=256),
    dict(count_grid=8, chunk_mult=1, wave_max_points=1024, plane_max_points=256),
    dict(count_grid=65536, chunk_mult=16, wave_max_points=100, plane_max_points=3),
    dict(count_grid=1024, chunk_mult=8, wave_max_points=768, plane_max_points=192),
]


def _clusters():
    off1, big = scenes.batched_clusters(seed=11, n_clusters=3, n_min=20_000, n_max=20_001)
    parts = []
    for i, n in enumerate(SIZES):
        src = big[off1[i % 3]:off1[i % 3 + 1]]
        s = (i * 97) % max(1, len(src) - n)
        parts.append(src[s:s + n])
    t = np.linspace(0, 1, 300)
    parts.append(np.c_[t, 2 * t, t].astype(np.float32))   # collinear: no valid hypothesis
    sizes = [len(p) for p in parts]
    assert sizes[:len(SIZES)] == SIZES
    off = np.zeros(len(parts) + 1, np.uint32)
    off[1:] = np.cumsum(sizes)
    xyz = np.concatenate(parts).astype(np.float32)
    tag = np.arange(len(parts), dtype=np.uint32) * 104729 + 11
    return off, xyz, tag


def _run(vm, cl, K, N, work):
    import torch
    pb = vm.PlaneBuffers.alloc(K, N, H, with_all=True)
    vm.ransac_planes(cl, vm.ransac_params(H, EPS, SEED, FRAME), pb, work)
    torch.cuda.synchronize()
    return pb


def _same(a, b):
    for key in ("plane", "best", "nin", "in_off", "in_idx", "counts", "hyp"):
        assert np.array_equal(np.asarray(a[key]).view(np.uint8), np.asarray(b[key]).view(np.uint8)), key
    assert a["status"] == b["status"] == 0


def test_every_count_config_gives_identical_results():
    import torch

    import paper_2510_01592_amd as vm
    off, xyz, tag = _clusters()
    K, N = len(tag), len(xyz)
    T = cluster_tensors(off, xyz, tag)
    cl = vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"])
    work = torch.empty(vm.workspace_bytes(K, N, H), dtype=torch.uint8, device="cuda")
    try:
        results = []
        for c in CONFIGS:
            note(f"count config {c}")
            vm.set_count_config(c)
            assert vm.get_count_config() == c
            results.append(planes_np(_run(vm, cl, K, N, work)))
        for r in results[1:]:
            _same(results[0], r)
        # the default setting against the oracle, cluster by cluster (hulls
        # from the same planes)
        vm.set_count_config(None)
        pb = _run(vm, cl, K, N, work)
        hb = vm.HullBuffers.alloc(K, N)
        vm.hulls(cl, pb, hb, work)
        torch.cuda.synchronize()
        P, Hh = planes_np(pb), hulls_np(hb)
        _same(results[0], P)
        for k in range(K):
            a, b = int(off[k]), int(off[k + 1])
            r = oracle.plane_and_hull(xyz[a:b, 0], xyz[a:b, 1], xyz[a:b, 2], H, EPS, SEED, int(tag[k]), FRAME)
            compare_cluster(k, P, Hh, r)
        # the autotuner keeps one valid setting, and results stay identical
        note("autotune count")
        pb = vm.PlaneBuffers.alloc(K, N, H, with_all=True)
        best = vm.autotune_count(cl, vm.ransac_params(H, EPS, SEED, FRAME), pb, work, reps=1)
        torch.cuda.synchronize()
        assert best == vm.get_count_config()
        assert best["count_grid"] % 8 == 0 and 1 <= best["chunk_mult"] <= 16
        assert best["plane_max_points"] <= min(256, best["wave_max_points"]) and best["wave_max_points"] <= 1024
        _same(results[0], planes_np(pb))
        _same(results[0], planes_np(_run(vm, cl, K, N, work)))
    finally:
        vm.set_count_config(None)

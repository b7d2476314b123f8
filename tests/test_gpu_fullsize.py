"""Parity at full workload sizes, in the launch configuration the benchmark
times: the 4x4x2 m map at 0.01 m (400x400x200 cells, 1M points per frame,
512 hypotheses) and the 2000-cluster batched set (log-uniform 50..200k
points, 1024 hypotheses).  The map, labels and clusters are compared in full,
and so are the planes, inlier lists and polygons of every cluster (the
oracle's clusters spread over the host's cores)."""
import os

import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_util import (assert_map_equal, bits, cluster_tensors, compare_cluster, hulls_np, note, planes_np,
                            run_planes_and_hulls)

pytestmark = pytest.mark.gpu

SEED = 0x5EED
THREADS = max(1, min(16, os.cpu_count() or 1))


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_full_map_frame_all_clusters():
    import torch
    import paper_2510_01592_amd as vm
    sc = scenes.scene_full_map(1)
    g = sc.geom
    n_warm = 8
    m = vm.Map(g.origin, g.voxel_size, g.dims, 23)
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    for f in range(n_warm):
        pts = scenes.frame_points(sc, 2 + f)
        note(f"full map warm frame {f}")
        m.insert(_t(pts))
        om.insert(pts)
    pts = scenes.frame_points(sc, 100)
    om.insert(pts)
    V = len(om.key)
    k_cap = 4096
    pb = vm.PlaneBuffers.alloc(k_cap, 1 << 23, sc.n_hyp)
    hb = vm.HullBuffers.alloc(k_cap, 1 << 22)
    labels = torch.zeros(V, dtype=torch.int32, device="cuda")
    note("full map segment_frame")
    cl = m.segment_frame(_t(pts), pb, hb, min_cluster=sc.min_cluster, n_hyp=sc.n_hyp, eps=sc.eps, seed=SEED,
                         frame=7, labels=labels)
    torch.cuda.synchronize()
    got = vm.read_clusters(cl)
    assert_map_equal(m, om)
    lab_ref, _ = oracle.ccl26(om.key, g.dims)
    assert np.array_equal(labels.cpu().numpy().view(np.uint32), lab_ref)
    c = oracle.group(om.key, lab_ref, om.means(), sc.min_cluster)
    assert got["K"] == len(c.tag) and np.array_equal(got["off"], c.off) and np.array_equal(got["tag"], c.tag)
    assert np.array_equal(got["key"], c.key)
    assert np.array_equal(bits(np.c_[got["x"], got["y"], got["z"]]), bits(c.xyz))
    P, H = planes_np(pb), hulls_np(hb)
    assert P["status"] == 0 and H["status"] == 0
    note(f"full map: oracle planes and hulls of all {len(c.tag)} clusters")
    refs = oracle.planes_and_hulls(c.off, c.xyz, c.tag, sc.n_hyp, sc.eps, SEED, 7, threads=THREADS)
    for k, r in enumerate(refs):
        compare_cluster(k, P, H, r, check_all_hyp=False)
    m.close()


def test_batched_fullsize_all_clusters():
    import paper_2510_01592_amd as vm
    off, xyz = scenes.batched_clusters(seed=3)
    K = len(off) - 1
    tag = np.arange(K, dtype=np.uint32)
    T = cluster_tensors(off, xyz, tag)
    cl = vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"])
    H = 1024
    note(f"batched 2000 clusters, {len(xyz)} points, H={H}")
    pb, hb = run_planes_and_hulls(vm, cl, K, len(xyz), H, 0.01, SEED, 0, with_all=False)
    P, Hh = planes_np(pb), hulls_np(hb)
    assert P["status"] == 0 and Hh["status"] == 0
    sizes = np.diff(off.astype(np.int64))
    note(f"batched: oracle planes and hulls of all {K} clusters on {THREADS} threads")
    refs = oracle.planes_and_hulls(off, xyz, tag, H, 0.01, SEED, 0, threads=THREADS)
    for k, r in enumerate(refs):
        compare_cluster(k, P, Hh, r, check_all_hyp=False)
    # every cluster found its plane, with most of its points as inliers
    assert np.all(P["best"] >= 0)
    assert np.all(P["nin"] >= 0.8 * sizes)

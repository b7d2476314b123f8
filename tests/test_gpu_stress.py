"""Parity on the stress map: 4x4x2 m at 0.005 m (800x800x400 cells in a
2^25-slot hash), three warm frames and one segmented frame of 8M points
each (about 10M occupied voxels), 1024 hypotheses.  The map, every voxel's
label and the cluster layout are compared in full, and so are the planes,
inlier lists and polygons of every cluster (the largest is the floor, about
a million voxels)."""
import concurrent.futures
import os

import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_util import assert_map_equal, bits, compare_cluster, hulls_np, note, planes_np

pytestmark = pytest.mark.gpu

SEED = 0x5EED
THREADS = max(1, min(16, os.cpu_count() or 1))


def test_stress_map_full():
    import torch

    import paper_2510_01592_amd as vm
    sc = scenes.scene_stress(5)
    g = sc.geom
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        frames = list(ex.map(lambda f: scenes.frame_points(sc, 100 + f), range(4)))
    m = vm.Map(g.origin, g.voxel_size, g.dims, 25)
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    for f, pts in enumerate(frames[:3]):
        note(f"stress warm frame {f} ({len(pts)} points)")
        m.insert(torch.from_numpy(pts).cuda())
        om.insert(pts)
    om.insert(frames[3])
    V = len(om.key)
    assert V > 8_000_000
    k_cap = 4096
    pb = vm.PlaneBuffers.alloc(k_cap, 1 << 24, sc.n_hyp)
    hb = vm.HullBuffers.alloc(k_cap, 1 << 22)
    labels = torch.zeros(V, dtype=torch.int32, device="cuda")
    note(f"stress segment_frame ({V} occupied voxels after it)")
    cl = m.segment_frame(torch.from_numpy(frames[3]).cuda(), pb, hb, min_cluster=sc.min_cluster, n_hyp=sc.n_hyp,
                         eps=sc.eps, seed=SEED, frame=3, labels=labels)
    torch.cuda.synchronize()
    st = m.stats()
    assert st.status_flags == 0 and st.points_lost == 0
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
    sizes = np.diff(c.off.astype(np.int64))
    assert sizes.max() > 500_000
    note(f"stress: oracle planes and hulls of all {len(c.tag)} clusters on {THREADS} threads")
    refs = oracle.planes_and_hulls(c.off, c.xyz, c.tag, sc.n_hyp, sc.eps, SEED, 3, threads=THREADS)
    for k, r in enumerate(refs):
        compare_cluster(k, P, H, r, check_all_hyp=False)
    m.close()

"""Voxel clearing (Sec. III-B, Eq. (2)) on the GPU against the oracle: the
map after each clear + insert is bit-identical (keys, counts, sums, means),
with the occupied and cleared counters, on walls crossed by rays, random
posed frames with points outside the grid, non-finite and far away, a moved
object in a ray-cast scene, graph replays, and the full 400x400x200 map
segmented with clearing on (clusters, planes and polygons)."""
import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_util import assert_map_equal, compare_cluster, hulls_np, note, planes_np

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pair(origin, s, dims, log2cap=16):
    import paper_2510_01592_amd as vm
    return vm.Map(origin, s, dims, log2cap), oracle.OracleMap(origin, s, dims)


def _step(m, om, pts_sensor, R, t, removed_total):
    """clear + insert one frame on both sides; returns the oracle's running total of cleared voxels"""
    m.clear_rays(_t(pts_sensor), R, t)
    removed_total += om.clear_rays(pts_sensor, R, t)
    m.insert(_t(pts_sensor), R, t)
    om.insert(pts_sensor, R, t)
    return removed_total


def _check(m, om, removed_total):
    assert_map_equal(m, om)
    st = m.stats()
    assert st.occupied == len(om.key)
    assert st.voxels_cleared == removed_total


def test_wall_crossed_by_rays():
    s = 0.01
    dims = (50, 40, 30)
    wall = np.array([[20, y, z] for y in range(10, 30) for z in range(5, 25)], np.float64)
    m, om = _pair((0.0, 0.0, 0.0), s, dims)
    pts = ((wall + 0.5) * s).astype(np.float32)
    m.insert(_t(pts))
    om.insert(pts)
    sensor = np.array([5.5, 20.5, 15.5]) * s
    target = np.array([[40.5, 20.5, 15.5], [40.5, 12.5, 8.5], [20.5, 20.5, 15.5]]) * s
    note("clearing: wall crossed by rays")
    tot = _step(m, om, (target - sensor).astype(np.float32), np.eye(3), sensor, 0)
    assert tot == 1
    _check(m, om, tot)


@pytest.mark.parametrize("seed", range(3))
def test_random_posed_frames(seed):
    """a random map, then frames from random sensor poses inside the grid; the
    frames hold points outside the grid, non-finite and absurdly far away"""
    rng = np.random.default_rng(900 + seed)
    dims = (64, 48, 40)
    s = 0.02
    origin = (-0.3, -0.2, -0.1)
    lo, hi = np.array(origin), np.array(origin) + s * np.array(dims)
    m, om = _pair(origin, s, dims)
    blob = rng.uniform(lo, hi, size=(30_000, 3)).astype(np.float32)
    m.insert(_t(blob))
    om.insert(blob)
    tot = 0
    for f in range(6):
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        R = q * np.sign(np.linalg.det(q))
        t = rng.uniform(lo + 0.1, hi - 0.1)
        pw = rng.uniform(lo - 0.3, hi + 0.3, size=(4000, 3))
        ps = ((pw - t) @ R).astype(np.float32)
        ps[:5] = np.nan
        ps[5:8] = np.float32(1e20)
        ps[8:10] = np.inf
        note(f"clearing: random posed frame seed {seed} frame {f}")
        tot = _step(m, om, ps, R, t, tot)
        _check(m, om, tot)
    assert tot > 0


def test_moved_object_disappears_and_graph_replays():
    """a box in a ray-cast scene moves; its old voxels are cleared, then the same
    clear + insert pair captured in a graph and replayed on new frames agrees
    with the eager calls on a twin map"""
    import torch
    import paper_2510_01592_amd as vm
    sc = scenes.scene_tiny(4)
    g = sc.geom
    box = scenes.Rect((0.3, 0.9, 0.2), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), 0.1, 0.15)
    moved = scenes.Rect((1.0, 0.9, 0.2), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), 0.1, 0.15)
    # a back wall catches the rays that pass the box's old place
    back = scenes.Rect((0.64, 1.25, 0.0), (1.0, 0.0, 0.0), (0.0, 0.0, 1.0), 0.64, 0.6)
    sc.rects = sc.rects + [back]
    sensor = np.array([0.64, 0.2, 0.5])
    pose = (np.eye(3), sensor)
    m, om = _pair(g.origin, g.voxel_size, g.dims, 18)
    tot = 0
    for f in range(3):
        pts = scenes.raycast_frame(sc, sensor, 40 + f, 60_000, pose=pose, rects=sc.rects + [box])
        note(f"clearing: ray-cast frame {f} (box at x=0.3)")
        tot = _step(m, om, pts, *pose, tot)
    _check(m, om, tot)
    before = set(om.key.tolist())
    for f in range(3):
        pts = scenes.raycast_frame(sc, sensor, 50 + f, 60_000, pose=pose, rects=sc.rects + [moved])
        note(f"clearing: ray-cast frame {f} (box moved to x=1.0)")
        tot = _step(m, om, pts, *pose, tot)
        _check(m, om, tot)
    # the box's old place, seen from the sensor through empty space, is gone
    old = scenes.raycast_frame(sc, sensor, 60, 20_000, rects=[box], outlier_frac=0.0)
    k_old = set(oracle.voxelize(old, np.eye(3), np.zeros(3), g.origin, g.voxel_size, g.dims)[0].tolist())
    assert len(k_old & before) > 100
    assert len(k_old & set(om.key.tolist())) < 0.1 * len(k_old & before)   # 3 frames clear most of it
    # graph capture of clear + insert on a twin map, replayed on new frames
    twin = vm.Map(g.origin, g.voxel_size, g.dims, 18)
    key, cnt, sums = om.key, om.cnt, om.sums
    twin.import_(_t(key.view(np.int32)), _t(cnt.view(np.int32)), _t(sums.view(np.int64)))
    buf = torch.zeros((60_000, 3), dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        twin.clear_rays(buf[:0], *pose, stream=s)   # allocates its bitmaps outside the capture
        s.synchronize()
        with vm.capture(s) as cap:
            twin.clear_rays(buf, *pose, stream=s)
            twin.insert(buf, *pose, stream=s)
        gr = cap.graph
    s.synchronize()
    for f in range(3):
        pts = scenes.raycast_frame(sc, sensor, 70 + f, 60_000, pose=pose, rects=sc.rects + [moved])
        buf.copy_(_t(pts))
        torch.cuda.synchronize()
        note(f"clearing: graph replay {f}")
        gr.launch(s)
        s.synchronize()
        om.clear_rays(pts, *pose)
        om.insert(pts, *pose)
        assert_map_equal(twin, om)
    gr.close()
    twin.close()
    m.close()


def test_full_map_segmented_with_clearing():
    import torch
    import paper_2510_01592_amd as vm
    sc = scenes.scene_full_map(1)
    g = sc.geom
    m, om = _pair(g.origin, g.voxel_size, g.dims, 23)
    poses = scenes.random_walk_poses(31, 3, sigma_t=0.05, sigma_rot_deg=2.0)
    pb = vm.PlaneBuffers.alloc(4096, 1 << 22, sc.n_hyp)
    hb = vm.HullBuffers.alloc(4096, 1 << 22)
    for f, (R, t0) in enumerate(poses):
        t = t0 + np.array([0.0, 0.0, 1.0])
        pts = scenes.raycast_frame(sc, t, 300 + f, 1_000_000, pose=(R, t))
        note(f"clearing: full map frame {f}, segment_frame(clear=True)")
        cl = m.segment_frame(_t(pts), pb, hb, R, t, min_cluster=30, n_hyp=sc.n_hyp, eps=sc.eps, seed=77, frame=f,
                             clear=True)
        torch.cuda.synchronize()
        om.clear_rays(pts, R, t)
        om.insert(pts, R, t)
        assert_map_equal(m, om)
    fr = oracle.segment(om, 30, sc.n_hyp, sc.eps, 77, len(poses) - 1, threads=8)
    got = vm.read_clusters(cl)
    assert got["K"] == len(fr.clusters.tag)
    assert np.array_equal(got["tag"], fr.clusters.tag) and np.array_equal(got["off"], fr.clusters.off)
    P, H = planes_np(pb), hulls_np(hb)
    for k, r in enumerate(fr.results):
        compare_cluster(k, P, H, r, check_all_hyp=False)
    assert m.stats().voxels_cleared > 0
    m.close()

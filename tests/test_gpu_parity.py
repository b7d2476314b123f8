"""GPU parity: every C-ABI call against the oracle on the same seeded inputs.

Bars: voxel maps, labels, clusters, hypothesis counts, best hypotheses and
inlier lists bit-exact; planes bit-exact (the contract allows 1e-5 on normals
and 1e-5 m on offsets); hull areas within 1e-5 relative (vertex lists and
projected vertices expected bit-exact)."""
import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_util import (assert_map_equal, bits, cluster_tensors, compare_cluster, export_np, hull_path_clusters,
                            hulls_np, note,
                            planes_np, run_planes_and_hulls)

pytestmark = pytest.mark.gpu

SEED = 0x5EED


@pytest.fixture(scope="module")
def vm():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_01592_amd as vm
    return vm


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_insert_tiny_bitexact(vm):
    sc = scenes.scene_tiny(0)
    g = sc.geom
    pts = scenes.frame_points(sc, 0)
    note("insert tiny 50k")
    m = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    m.insert(_t(pts))
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    om.insert(pts)
    assert_map_equal(m, om)
    st = m.stats()
    assert st.occupied == len(om.key) and st.points_in == om.points_in and st.points_dropped == 0
    assert st.status_flags == 0


def test_insert_posed_frames(vm):
    sc = scenes.scene_full_map(1)
    g = sc.geom
    poses = scenes.random_walk_poses(21, 3, sigma_t=0.05, sigma_rot_deg=3.0)
    m = vm.Map(g.origin, g.voxel_size, g.dims, 20)
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    for f, (R, t) in enumerate(poses):
        pts = scenes.frame_points(sc, 100 + f, n=150_000, pose=(R, t))
        note(f"insert posed frame {f}")
        m.insert(_t(pts), R, t)
        om.insert(pts, R, t)
    assert_map_equal(m, om)
    st = m.stats()
    assert st.points_dropped == om.points_dropped and st.points_in == om.points_in


@pytest.mark.parametrize("batch_log2", [0, 16])
def test_insert_grouped_and_atomic_paths_agree(vm, batch_log2):
    # one large call (grouped path, split into batches of 2^16 when batch_log2=16)
    # against many small calls (per-point atomics) and against the oracle
    sc = scenes.scene_full_map(1)
    g = sc.geom
    pts = scenes.frame_points(sc, 77, n=400_000)
    note(f"insert grouped vs atomic, batch_log2={batch_log2}")
    a = vm.Map(g.origin, g.voxel_size, g.dims, 21, insert_batch_log2=batch_log2)
    a.insert(_t(pts))
    b = vm.Map(g.origin, g.voxel_size, g.dims, 21)
    for c in range(0, len(pts), 50_000):
        b.insert(_t(pts[c:c + 50_000]))
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    om.insert(pts)
    assert_map_equal(a, om)
    assert_map_equal(b, om)
    sa, sb = a.stats(), b.stats()
    assert sa.points_in == sb.points_in == om.points_in
    assert sa.points_dropped == sb.points_dropped == om.points_dropped
    key, _, _ = oracle.voxelize(pts, np.eye(3), np.zeros(3), g.origin, g.voxel_size, g.dims)
    if batch_log2 == 0:      # one grouped batch: one update per distinct voxel
        assert sa.last_touched == len(np.unique(key[key != oracle.NO_KEY]))
    else:                    # one update per distinct voxel of each 2^16-point batch
        B = 1 << batch_log2
        expect = sum(len(np.unique(kb[kb != oracle.NO_KEY])) for kb in (key[i:i + B] for i in range(0, len(key), B)))
        assert sa.last_touched == expect


def test_insert_drops_and_bounds(vm):
    g = scenes.MapGeom((0.0, 0.0, 0.0), 0.25, (8, 8, 8))
    pts = np.array([[np.nan, 0.1, 0.1], [0.1, np.inf, 0.1], [0.1, 0.1, -np.inf], [2.0, 0.1, 0.1],
                    [1.999, 0.1, 0.1], [0.25, 0.5, 0.75], [0.0, 0.0, 0.0], [-1e-7, 0.0, 0.0]], np.float32)
    note("insert drops")
    m = vm.Map(g.origin, g.voxel_size, g.dims, 10)
    m.insert(_t(pts))
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    om.insert(pts)
    assert_map_equal(m, om)
    st = m.stats()
    assert st.points_dropped == om.points_dropped == 5
    assert st.points_in == 3


def _grid_points(grid, origin=(0.0, 0.0, 0.0), s=0.01):
    zz, yy, xx = np.nonzero(grid)
    return (np.c_[xx, yy, zz] * s + np.asarray(origin) + 0.5 * s).astype(np.float32)


@pytest.mark.parametrize("shape,p,seed", [((11, 23, 37), 0.3, 0), ((16, 64, 64), 0.08, 1), ((5, 5, 5), 0.6, 2),
                                          ((30, 70, 33), 0.15, 3), ((1, 1, 200), 0.5, 4), ((40, 1, 1), 0.5, 5),
                                          ((40, 96, 96), 0.06, 6), ((32, 48, 64), 0.5, 8), ((16, 32, 96), 0.3, 9)])
def test_ccl_random_grids(vm, shape, p, seed):
    """Labels and the cluster CSR.  The (40, 96, 96) grid has 8693 components,
    so the grouping sort takes two digit passes (cluster ids of 1024 and
    more); the dense grids give labelling tiles thousands of run hooks, more
    than one round of the tile's pair list."""
    import torch
    grid = np.random.default_rng(seed).random(shape) < p
    nz, ny, nx = shape
    pts = _grid_points(grid)
    note(f"ccl grid {shape} p={p}")
    m = vm.Map((0.0, 0.0, 0.0), 0.01, (nx, ny, nz), 18)
    m.insert(_t(pts))
    V = int(m.stats().occupied)
    keys = np.flatnonzero(grid.ravel()).astype(np.uint32)
    ref, _ = oracle.ccl26(keys, (nx, ny, nz))
    assert V == len(keys)
    om = oracle.OracleMap((0.0, 0.0, 0.0), 0.01, (nx, ny, nz))
    om.insert(pts)
    assert np.array_equal(om.key, keys)
    mu = om.means()
    for minc in (1, 2, 3):
        labels = torch.zeros(max(V, 1), dtype=torch.int32, device="cuda")
        cl = m.ccl(minc, labels=labels)
        got = vm.read_clusters(cl)
        assert np.array_equal(labels.cpu().numpy()[:V].view(np.uint32), ref)
        c = oracle.group(keys, ref, mu, minc)
        assert got["K"] == len(c.tag) and got["N"] == int(c.off[-1]), minc
        assert np.array_equal(got["off"], c.off) and np.array_equal(got["tag"], c.tag)
        assert np.array_equal(got["key"], c.key)
        assert np.array_equal(bits(np.c_[got["x"], got["y"], got["z"]]), bits(c.xyz))


def _oracle_frame(sc, frames, n_hyp=None, subset=None):
    g = sc.geom
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    for pts in frames:
        om.insert(pts)
    fr = oracle.segment(om, sc.min_cluster, n_hyp or sc.n_hyp, sc.eps, SEED, 0, cluster_subset=subset)
    return om, fr


def test_ccl_clusters_tiny(vm):
    import torch
    sc = scenes.scene_tiny(0)
    g = sc.geom
    pts = scenes.frame_points(sc, 0)
    note("ccl + clusters tiny")
    m = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    m.insert(_t(pts))
    V = int(m.stats().occupied)
    labels = torch.zeros(V, dtype=torch.int32, device="cuda")
    cl = m.ccl(sc.min_cluster, labels=labels)
    got = vm.read_clusters(cl)
    om, fr = _oracle_frame(sc, [pts], subset=[])
    assert np.array_equal(labels.cpu().numpy().view(np.uint32), fr.labels)
    c = fr.clusters
    assert got["K"] == len(c.tag) and got["N"] == int(c.off[-1])
    assert np.array_equal(got["off"], c.off) and np.array_equal(got["tag"], c.tag)
    assert np.array_equal(got["key"], c.key)
    assert np.array_equal(bits(np.c_[got["x"], got["y"], got["z"]]), bits(c.xyz))


def test_ransac_hull_tiny_all_hypotheses(vm):
    sc = scenes.scene_tiny(0)
    g = sc.geom
    pts = scenes.frame_points(sc, 0)
    note("ransac + hull tiny")
    m = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    m.insert(_t(pts))
    cl = m.ccl(sc.min_cluster)
    pb, hb = run_planes_and_hulls(vm, cl, 64, 1 << 17, sc.n_hyp, sc.eps, SEED, 0)
    om, fr = _oracle_frame(sc, [pts])
    P, H = planes_np(pb), hulls_np(hb)
    assert P["status"] == 0 and H["status"] == 0
    for k, r in enumerate(fr.results):
        compare_cluster(k, P, H, r)


@pytest.mark.parametrize("exact", [False, True])
def test_segment_frame_tiny(vm, exact):
    sc = scenes.scene_tiny_exact(0) if exact else scenes.scene_tiny(0)
    g = sc.geom
    pts = scenes.frame_points(sc, 0)
    note(f"segment_frame tiny exact={exact}")
    m = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    pb = vm.PlaneBuffers.alloc(64, 1 << 17, sc.n_hyp)
    hb = vm.HullBuffers.alloc(64, 1 << 17)
    cl = m.segment_frame(_t(pts), pb, hb, min_cluster=sc.min_cluster, n_hyp=sc.n_hyp, eps=sc.eps, seed=SEED, frame=0)
    got = vm.read_clusters(cl)
    om, fr = _oracle_frame(sc, [pts])
    assert got["K"] == len(fr.clusters.tag) == 3
    P, H = planes_np(pb), hulls_np(hb)
    for k, r in enumerate(fr.results):
        compare_cluster(k, P, H, r, check_all_hyp=False)


def test_batched_clusters_ragged(vm):
    # log-uniform sizes plus the degenerate sizes 0, 1, 2, 3 and a collinear cluster
    off, xyz = scenes.batched_clusters(seed=7, n_clusters=60, n_min=3, n_max=30_000)
    sizes = list(np.diff(off.astype(np.int64)))
    parts = [xyz[off[i]:off[i + 1]] for i in range(60)]
    t = np.linspace(0, 1, 40)
    parts += [np.zeros((0, 3), np.float32), xyz[:1], xyz[:2], xyz[:3], np.c_[t, 2 * t, t].astype(np.float32)]
    sizes = [len(p) for p in parts]
    off = np.zeros(len(parts) + 1, np.uint32)
    off[1:] = np.cumsum(sizes)
    xyz = np.concatenate(parts).astype(np.float32)
    tag = np.arange(len(parts), dtype=np.uint32) * 7919 + 3
    T = cluster_tensors(off, xyz, tag)
    import paper_2510_01592_amd as _vm
    cl = _vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"])
    H = 384
    note("batched clusters ragged")
    pb, hb = run_planes_and_hulls(vm, cl, len(parts), len(xyz), H, 0.01, SEED, 5)
    P, Hh = planes_np(pb), hulls_np(hb)
    for k in range(len(parts)):
        a, b = int(off[k]), int(off[k + 1])
        r = oracle.plane_and_hull(xyz[a:b, 0], xyz[a:b, 1], xyz[a:b, 2], H, 0.01, SEED, int(tag[k]), 5)
        compare_cluster(k, P, Hh, r)


def test_determinism_repeat(vm):
    sc = scenes.scene_tiny(0)
    g = sc.geom
    pts = scenes.frame_points(sc, 0)
    outs = []
    for rep in range(2):
        note(f"determinism rep {rep}")
        m = vm.Map(g.origin, g.voxel_size, g.dims, 17)
        pb = vm.PlaneBuffers.alloc(64, 1 << 17, sc.n_hyp, with_all=True)
        hb = vm.HullBuffers.alloc(64, 1 << 17)
        m.segment_frame(_t(pts[np.random.default_rng(rep).permutation(len(pts))]), pb, hb, min_cluster=30,
                        n_hyp=sc.n_hyp, eps=sc.eps, seed=SEED, frame=0)
        outs.append((planes_np(pb), hulls_np(hb)))
    for key in ("plane", "best", "nin", "in_off", "in_idx", "counts", "hyp"):
        assert np.array_equal(outs[0][0][key], outs[1][0][key]), key
    for key in ("v_off", "v_idx", "v_xyz", "area"):
        assert np.array_equal(outs[0][1][key], outs[1][1][key]), key


def test_empty_and_small(vm):
    g = scenes.scene_tiny(0).geom
    note("empty frame")
    m = vm.Map(g.origin, g.voxel_size, g.dims, 12)
    pb = vm.PlaneBuffers.alloc(8, 1024, 16)
    hb = vm.HullBuffers.alloc(8, 1024)
    cl = m.segment_frame(None, pb, hb, min_cluster=30, n_hyp=16)
    got = vm.read_clusters(cl)
    assert got["K"] == 0 and got["N"] == 0
    # a handful of points: clusters below the minimum size are dropped
    pts = np.array([[0.105, 0.105, 0.105], [0.115, 0.105, 0.105], [0.505, 0.505, 0.505]], np.float32)
    note("tiny frame")
    cl = m.segment_frame(_t(pts), pb, hb, min_cluster=2, n_hyp=16)
    got = vm.read_clusters(cl)
    assert got["K"] == 1 and got["N"] == 2
    assert int(pb.best_h.cpu()[0]) == -1


def test_overflow_flags(vm):
    import torch
    sc = scenes.scene_tiny(0)
    g = sc.geom
    pts = scenes.frame_points(sc, 0)
    note("hash overflow")
    m = vm.Map(g.origin, g.voxel_size, g.dims, 10)       # 1024 slots for ~29k voxels
    m.insert(_t(pts))
    st = m.stats()
    assert st.status_flags & vm.FLAG_HASH_FULL and st.points_lost > 0 and st.occupied <= 1024
    note("output capacity overflow")
    m2 = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    m2.insert(_t(pts))
    cl = m2.ccl(30)
    pb, hb = run_planes_and_hulls(vm, cl, 64, 1 << 17, 32, 0.01, SEED, 0, with_all=False)
    full = planes_np(pb)
    # only two of the three clusters fit; few hull slots
    work = torch.empty(vm.workspace_bytes(4, cl.n_cap, 32), dtype=torch.uint8, device="cuda")
    small = vm.PlaneBuffers.alloc(2, 30000, 32)
    hsmall = vm.HullBuffers.alloc(2, 10)
    vm.ransac_planes(cl, vm.ransac_params(32, 0.01, SEED, 0), small, work)
    vm.hulls(cl, small, hsmall, work)
    torch.cuda.synchronize()
    assert int(small.status.cpu()[0]) == vm.FLAG_CLUSTERS_CAP
    assert int(hsmall.status.cpu()[0]) == vm.FLAG_HULL_CAP
    assert np.array_equal(small.best_h.cpu().numpy(), full["best"][:2])
    assert np.array_equal(small.plane.cpu().numpy().view(np.uint32), full["plane"][:2].view(np.uint32))
    na = int(small.in_off.cpu()[2])
    assert np.array_equal(small.in_idx.cpu().numpy()[:na], full["in_idx"][:na])
    # too few inlier slots: flagged, nothing written out of bounds
    tiny = vm.PlaneBuffers.alloc(4, 1000, 32)
    vm.ransac_planes(cl, vm.ransac_params(32, 0.01, SEED, 0), tiny, work)
    torch.cuda.synchronize()
    assert int(tiny.status.cpu()[0]) & vm.FLAG_INLIERS_CAP


def test_stage_timing(vm):
    sc = scenes.scene_tiny(0)
    g = sc.geom
    pts = scenes.frame_points(sc, 0)
    vm.set_stage_timing(True)
    try:
        note("stage timing")
        m = vm.Map(g.origin, g.voxel_size, g.dims, 17)
        pb = vm.PlaneBuffers.alloc(64, 1 << 17, sc.n_hyp)
        hb = vm.HullBuffers.alloc(64, 1 << 17)
        m.segment_frame(_t(pts), pb, hb, min_cluster=30, n_hyp=sc.n_hyp, clear=True)   # every stage runs
        ms, n = vm.stage_times()
    finally:
        vm.set_stage_timing(False)
    assert np.all(n >= 1) and np.all(ms > 0)


def test_many_clusters_both_launch_forms(vm):
    """More clusters than the one-workgroup preparation handles (65536): the
    multi-kernel form runs; the first 60000 clusters alone take the
    one-workgroup form.  Both agree bit for bit on every shared output and a
    sample of clusters matches the oracle."""
    rng = np.random.default_rng(21)
    src_off, src = scenes.batched_clusters(seed=5, n_clusters=8, n_min=20_000, n_max=20_001)
    K, H = 70_000, 64
    sizes = rng.integers(0, 41, size=K)
    sizes[[17, 40_000, 65_600]] = [5000, 4097, 3000]
    parts = []
    for k, n in enumerate(sizes):
        j = k % 8
        a = int(src_off[j]) + int(rng.integers(0, 20_000 - int(n)))
        parts.append(src[a:a + int(n)])
    off = np.zeros(K + 1, np.uint32)
    off[1:] = np.cumsum(sizes)
    xyz = np.concatenate(parts).astype(np.float32)
    tag = (np.arange(K, dtype=np.uint64) * 2654435761 % (1 << 32)).astype(np.uint32)
    note(f"many clusters K={K} N={len(xyz)}")
    out = {}
    for kk in (K, 60_000):
        n = int(off[kk])
        T = cluster_tensors(off[:kk + 1], xyz[:n], tag[:kk])
        cl = vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"])
        pb, hb = run_planes_and_hulls(vm, cl, kk, n, H, 0.01, SEED, 2)
        out[kk] = (planes_np(pb), hulls_np(hb))
    (Pa, Ha), (Pb, Hb) = out[K], out[60_000]
    k2 = 60_000
    assert Pa["status"] == Pb["status"] == 0 and Ha["status"] == Hb["status"] == 0
    for key in ("plane", "best", "nin", "counts", "hyp"):
        assert np.array_equal(np.asarray(Pa[key][:k2]).view(np.uint8), np.asarray(Pb[key]).view(np.uint8)), key
    assert np.array_equal(Pa["in_off"][:k2 + 1], Pb["in_off"])
    assert np.array_equal(Pa["in_idx"][:Pb["in_off"][k2]], Pb["in_idx"][:Pb["in_off"][k2]])
    assert np.array_equal(Ha["v_off"][:k2 + 1], Hb["v_off"])
    assert np.array_equal(Ha["area"][:k2], Hb["area"])
    nv = int(Hb["v_off"][k2])
    assert np.array_equal(Ha["v_idx"][:nv], Hb["v_idx"][:nv])
    assert np.array_equal(bits(Ha["v_xyz"][:nv]), bits(Hb["v_xyz"][:nv]))
    sample = sorted(set(rng.choice(K, 120, replace=False).tolist()) | {0, 17, 40_000, 65_535, 65_536, 65_600, K - 1})
    for k in sample:
        a, b = int(off[k]), int(off[k + 1])
        r = oracle.plane_and_hull(xyz[a:b, 0], xyz[a:b, 1], xyz[a:b, 2], H, 0.01, SEED, int(tag[k]), 2)
        compare_cluster(k, Pa, Ha, r)


def test_hull_paths_by_survivor_count(vm):
    """The clusters of hull_path_clusters reach every hull path: one wave (at
    most 64 points or survivors), the workgroup chain with a one-wave sort (up
    to 256 survivors) and a workgroup sort (up to 2048), the 64-direction
    refinement of larger survivor sets, and the sort in global memory beyond
    that.  All against the oracle, vertex lists bit for bit."""
    off, xyz, tag = hull_path_clusters()
    parts = [xyz[off[k]:off[k + 1]] for k in range(len(tag))]
    T = cluster_tensors(off, xyz, tag)
    cl = vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"])
    H = 128
    note("hull paths")
    pb, hb = run_planes_and_hulls(vm, cl, len(parts), len(xyz), H, 0.01, SEED, 1)
    P, Hh = planes_np(pb), hulls_np(hb)
    assert P["status"] == 0 and Hh["status"] == 0
    for k in range(len(parts)):
        a, b = int(off[k]), int(off[k + 1])
        r = oracle.plane_and_hull(xyz[a:b, 0], xyz[a:b, 1], xyz[a:b, 2], H, 0.01, SEED, int(tag[k]), 1)
        compare_cluster(k, P, Hh, r, check_all_hyp=False)


def test_hull_mid_list_beyond_half_the_grid(vm):
    """More clusters with 65..256 hull survivors (thin rings: nearly every
    point is on the hull) than half of the small-cluster kernel's workgroups,
    so that its workgroup chains stride over the list, mixed with discs small
    enough for the one-wave path; every cluster against the oracle, vertex
    lists bit for bit."""
    import os
    rng = np.random.default_rng(71)
    nrm = np.array([0.3, 0.1, 1.0]) / np.linalg.norm([0.3, 0.1, 1.0])
    a = np.cross(nrm, [1.0, 0.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(nrm, a)
    parts = []
    for q in range(1300):
        n = int(rng.integers(80, 250))
        r = 0.2 + 0.1 * rng.random() + rng.normal(0, 1e-5, n)
        th = rng.random(n) * 2 * np.pi
        p = (r * np.cos(th))[:, None] * a + (r * np.sin(th))[:, None] * b + rng.random(3)
        parts.append(p.astype(np.float32))
        if q % 5 == 0:
            n = int(rng.integers(8, 60))
            r = 0.05 * np.sqrt(rng.random(n))
            th = rng.random(n) * 2 * np.pi
            p = (r * np.cos(th))[:, None] * a + (r * np.sin(th))[:, None] * b + rng.random(3)
            parts.append(p.astype(np.float32))
    off = np.zeros(len(parts) + 1, np.uint32)
    off[1:] = np.cumsum([len(p) for p in parts])
    xyz = np.concatenate(parts)
    K = len(parts)
    tag = np.arange(K, dtype=np.uint32) * 31 + 9
    T = cluster_tensors(off, xyz, tag)
    cl = vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"])
    H = 32
    note(f"hull mid list: {K} clusters, {len(xyz)} points")
    pb, hb = run_planes_and_hulls(vm, cl, K, len(xyz), H, 0.01, SEED, 3, with_all=False)
    P, Hh = planes_np(pb), hulls_np(hb)
    assert P["status"] == 0 and Hh["status"] == 0
    refs = oracle.planes_and_hulls(off, xyz, tag, H, 0.01, SEED, 3, threads=max(1, min(16, os.cpu_count() or 1)))
    survivors = 0
    for k, r in enumerate(refs):
        compare_cluster(k, P, Hh, r, check_all_hyp=False)
        survivors += int(Hh["v_off"][k + 1] - Hh["v_off"][k]) > 64
    # the rings' polygons keep more than a wave of vertices: they took the workgroup chain
    assert survivors > 1024, survivors

"""Whole-frame checks of the oracle (Sec. III-B then III-C on the map) on the
tiny stair scene: the three planes come out where the scene put them."""
import numpy as np

import oracle
import scenes


def _run(sc, n_hyp=256):
    g = sc.geom
    m = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    m.insert(scenes.frame_points(sc, sc.seed))
    return m, oracle.segment(m, sc.min_cluster, n_hyp, sc.eps, 0x5EED, 0)


def test_tiny_scene_planes():
    sc = scenes.scene_tiny(0)
    m, fr = _run(sc)
    cl = fr.clusters
    assert len(cl.tag) == 3
    sizes = np.diff(cl.off.astype(np.int64))
    assert np.all(sizes >= 30)
    # grouping: label = smallest key of the cluster, keys ascending within it
    for k in range(3):
        ks = cl.key[cl.off[k]:cl.off[k + 1]]
        assert ks[0] == cl.tag[k] and np.all(np.diff(ks.astype(np.int64)) > 0)
    assert np.all(np.diff(cl.tag.astype(np.int64)) > 0)
    heights = sorted(-float(r.ransac.plane[3]) for r in fr.results)
    assert abs(heights[0] - 0.0) < 0.01 and abs(heights[1] - 0.18) < 0.02 and abs(heights[2] - 0.36) < 0.03
    for r in fr.results:
        assert r.ransac.plane[2] > 0.99
    areas = sorted(r.hull.area for r in fr.results)
    assert abs(areas[0] - 0.18) < 0.01 and abs(areas[1] - 0.18) < 0.01 and abs(areas[2] - 1.6384) < 0.02


def test_tiny_exact_scene_recovers_treads():
    sc = scenes.scene_tiny_exact(0)
    m, fr = _run(sc)
    assert len(fr.clusters.tag) == 3
    for r in fr.results:
        # noise-free horizontal planes: every voxel mean of a cluster is on it
        assert np.allclose(r.ransac.plane[:3], [0, 0, 1], atol=1e-6)
        assert len(r.ransac.inliers) == r.ransac.counts.max()
    zs = sorted(-float(r.ransac.plane[3]) for r in fr.results)
    assert np.allclose(zs, [0.0, 0.18, 0.36], atol=1e-6)


def test_group_drops_small_and_counts_add_up():
    sc = scenes.scene_tiny(0)
    m, fr = _run(sc)
    lab = fr.labels
    u, c = np.unique(lab, return_counts=True)
    assert int(fr.clusters.off[-1]) == int(c[c >= 30].sum())
    assert len(fr.clusters.tag) == int((c >= 30).sum())


def test_threaded_oracle_is_identical():
    """The all-cores column of the CPU baseline: clusters spread over threads
    give exactly the single-threaded results (per-cluster frame numbers too)."""
    off, xyz = scenes.batched_clusters(seed=11, n_clusters=40, n_min=3, n_max=3000)
    tag = np.arange(40, dtype=np.uint32) * 13 + 1
    frames = np.arange(40, dtype=np.uint64) % 3
    a = oracle.planes_and_hulls(off, xyz, tag, 96, 0.01, 0x5EED, frames, threads=1)
    b = oracle.planes_and_hulls(off, xyz, tag, 96, 0.01, 0x5EED, frames, threads=8)
    assert len(a) == len(b) == 40
    for ra, rb in zip(a, b):
        assert ra.ransac.best_h == rb.ransac.best_h
        assert np.array_equal(ra.ransac.counts, rb.ransac.counts)
        assert np.array_equal(ra.ransac.plane.view(np.uint32), rb.ransac.plane.view(np.uint32))
        assert np.array_equal(ra.ransac.inliers, rb.ransac.inliers)
        if ra.hull is None:
            assert rb.hull is None
        else:
            assert np.array_equal(ra.hull_local, rb.hull_local) and ra.hull.area == rb.hull.area
    # a per-cluster frame number is the cluster's own RNG counter word
    c = oracle.planes_and_hulls(off, xyz, tag, 96, 0.01, 0x5EED, 2, ks=[5])
    r = oracle.plane_and_hull(xyz[off[5]:off[6], 0], xyz[off[5]:off[6], 1], xyz[off[5]:off[6], 2], 96, 0.01,
                              0x5EED, int(tag[5]), 2)
    assert np.array_equal(c[0].ransac.counts, r.ransac.counts)

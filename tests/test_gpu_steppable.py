"""The steppable path on the GPU against the oracle: Eq. (3)-(4) normals (bit
for bit) and steppable flags of every occupied voxel, the gated labels of
Alg. 1, the cluster layout, and the planes and polygons of the full Sec. III-C
path (vm_segment_frame_steppable), on a box standing on a floor, the tiny
stair scene, random voxel sets with scattered means (radius 1 and 2), and
the full 400x400x200 map."""
import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_util import bits, compare_cluster, hulls_np, note, planes_np

pytestmark = pytest.mark.gpu

SEED = 0x5EED


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check_map(vm, m, om, radius=1, min_cluster=30):
    import torch
    V = len(om.key)
    nrm = torch.zeros((V, 3), dtype=torch.float32, device="cuda")
    stp = torch.zeros(V, dtype=torch.uint8, device="cuda")
    lab = torch.zeros(V, dtype=torch.int32, device="cuda")
    cl = m.ccl_steppable(min_cluster, vm.step_params(radius=radius), normals=nrm, steppable=stp, labels=lab)
    torch.cuda.synchronize()
    got = vm.read_clusters(cl)
    mu = om.means()
    rn, rs, _ = oracle.classify(om.key, mu, om.dims, radius=radius)
    assert np.array_equal(bits(nrm.cpu().numpy()), bits(rn))
    assert np.array_equal(stp.cpu().numpy().astype(bool), rs)
    rl, _ = oracle.ccl_gated(om.key, mu, rn, rs, om.dims)
    assert np.array_equal(lab.cpu().numpy().view(np.uint32), rl)
    c = oracle.group(om.key, rl, mu, min_cluster)
    assert got["K"] == len(c.tag) and np.array_equal(got["off"], c.off) and np.array_equal(got["tag"], c.tag)
    assert np.array_equal(got["key"], c.key)
    assert np.array_equal(bits(np.c_[got["x"], got["y"], got["z"]]), bits(c.xyz))
    return c, rs


def test_box_on_floor_and_full_path():
    import torch
    import paper_2510_01592_amd as vm
    from tests.test_oracle_steppable import _box_on_floor
    om = _box_on_floor()
    m = vm.Map(tuple(om.origin), om.voxel_size, tuple(int(d) for d in om.dims), 16)
    m.import_(_t(om.key.view(np.int32)), _t(om.cnt.view(np.int32)), _t(om.sums.view(np.int64)))
    note("steppable: box on floor")
    c, _ = _check_map(vm, m, om)
    assert len(c.tag) == 2
    # the full path on a fresh map: insert a frame, classify, cluster, planes, polygons
    sc = scenes.scene_tiny(0)
    g = sc.geom
    pts = scenes.frame_points(sc, 0)
    m2 = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    pb = vm.PlaneBuffers.alloc(64, 1 << 17, sc.n_hyp)
    hb = vm.HullBuffers.alloc(64, 1 << 17)
    note("steppable: full path, tiny scene")
    cl = m2.segment_frame(_t(pts), pb, hb, min_cluster=30, n_hyp=sc.n_hyp, eps=sc.eps, seed=SEED, frame=3,
                          step=vm.step_params())
    torch.cuda.synchronize()
    om2 = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    om2.insert(pts)
    fr = oracle.segment(om2, 30, sc.n_hyp, sc.eps, SEED, 3, steppable={})
    got = vm.read_clusters(cl)
    assert got["K"] == len(fr.clusters.tag) >= 3
    assert np.array_equal(got["tag"], fr.clusters.tag)
    P, Hh = planes_np(pb), hulls_np(hb)
    for k, r in enumerate(fr.results):
        compare_cluster(k, P, Hh, r, check_all_hyp=False)
    m.close()
    m2.close()


@pytest.mark.parametrize("radius,seed", [(1, 0), (2, 1), (1, 2)])
def test_random_voxels(radius, seed):
    import paper_2510_01592_amd as vm
    rng = np.random.default_rng(200 + seed)
    dims = (37, 23, 19)
    s = 0.01
    # dense random blobs, so neighbourhoods are full and gates are exercised
    n = 20_000
    idx = np.clip(rng.normal([18, 11, 9], [6, 4, 3], size=(n, 3)).astype(int), 0, np.array(dims) - 1)
    pts = ((idx + rng.uniform(0, 1, (n, 3))) * s).astype(np.float32)
    om = oracle.OracleMap((0.0, 0.0, 0.0), s, dims)
    om.insert(pts)
    m = vm.Map((0.0, 0.0, 0.0), s, dims, 16)
    m.insert(_t(pts))
    note(f"steppable: random voxels radius {radius} seed {seed}")
    c, st = _check_map(vm, m, om, radius=radius, min_cluster=2)
    assert 0 < st.sum() < len(st)
    m.close()


def test_full_map():
    import paper_2510_01592_amd as vm
    sc = scenes.scene_full_map(1)
    g = sc.geom
    m = vm.Map(g.origin, g.voxel_size, g.dims, 23)
    om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    for f in range(4):
        pts = scenes.frame_points(sc, 2 + f)
        m.insert(_t(pts))
        om.insert(pts)
    note(f"steppable: full map, {len(om.key)} voxels")
    c, st = _check_map(vm, m, om)
    # the floor, treads, tabletop and the gentler patches are steppable clusters
    assert len(c.tag) >= 10
    m.close()

"""The persistent form (vm_planes_hulls): RANSAC planes and polygons of a
whole cluster set in one persistent launch.  Every output -- planes, every
hypothesis' count and plane, inlier CSR, polygons, areas, status flags -- is
bit-identical to vm_ransac_planes followed by vm_hulls, under every work
split, and matches the oracle; the sets cover ragged and degenerate sizes,
every hull path (one wave in the finisher; the tail launch for more than 64
survivors, with its LDS chain, its 64-direction refinement and its sort in
global memory), output capacity overflows and the 2000-cluster set."""
import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_util import (bits, cluster_tensors, compare_cluster, hull_path_clusters, hulls_np, note, planes_np,
                            ragged_clusters)

pytestmark = pytest.mark.gpu

SEED = 0x5EED


def _view(vm, off, xyz, tag):
    T = cluster_tensors(off, xyz, tag)
    return vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"]), T


def _run(vm, cl, H, frame, fused, k_cap=None, in_cap=None, v_cap=None, with_all=True):
    import torch
    k_cap = cl.k_cap if k_cap is None else k_cap
    in_cap = cl.n_cap if in_cap is None else in_cap
    v_cap = cl.n_cap if v_cap is None else v_cap
    kc = min(k_cap, cl.k_cap)
    work = torch.empty(vm.workspace_bytes(kc, cl.n_cap, H), dtype=torch.uint8, device="cuda")
    pb = vm.PlaneBuffers.alloc(k_cap, in_cap, H, with_all=with_all)
    hb = vm.HullBuffers.alloc(k_cap, v_cap)
    prm = vm.ransac_params(H, 0.01, SEED, frame)
    if fused:
        vm.planes_hulls(cl, prm, pb, hb, work)
    else:
        vm.ransac_planes(cl, prm, pb, work)
        vm.hulls(cl, pb, hb, work)
    torch.cuda.synchronize()
    return planes_np(pb), hulls_np(hb)


def _same(a, b, K):
    (P1, H1), (P2, H2) = a, b
    assert P1["status"] == P2["status"] and H1["status"] == H2["status"]
    for key in ("best", "nin"):
        assert np.array_equal(P1[key][:K], P2[key][:K]), key
    assert np.array_equal(bits(P1["plane"][:K]), bits(P2["plane"][:K]))
    if P1["counts"] is not None:
        assert np.array_equal(P1["counts"][:K], P2["counts"][:K])
        assert np.array_equal(bits(P1["hyp"][:K]), bits(P2["hyp"][:K]))
    assert np.array_equal(P1["in_off"][:K + 1], P2["in_off"][:K + 1])
    n = min(int(P1["in_off"][K]), len(P1["in_idx"]))
    assert np.array_equal(P1["in_idx"][:n], P2["in_idx"][:n])
    assert np.array_equal(H1["v_off"][:K + 1], H2["v_off"][:K + 1])
    v = min(int(H1["v_off"][K]), len(H1["v_idx"]))
    assert np.array_equal(H1["v_idx"][:v], H2["v_idx"][:v])
    assert np.array_equal(bits(H1["v_xyz"][:v]), bits(H2["v_xyz"][:v]))
    assert np.array_equal(H1["area"][:K].view(np.uint64), H2["area"][:K].view(np.uint64))


def test_fused_ragged_matches_oracle_and_two_pass():
    import paper_2510_01592_amd as vm
    off, xyz, tag = ragged_clusters()
    cl, _keep = _view(vm, off, xyz, tag)
    K, H = len(tag), 384
    note("fused: ragged clusters")
    got = _run(vm, cl, H, 5, True)
    ref = _run(vm, cl, H, 5, False)
    _same(got, ref, K)
    P, Hh = got
    for k in range(K):
        a, b = int(off[k]), int(off[k + 1])
        r = oracle.plane_and_hull(xyz[a:b, 0], xyz[a:b, 1], xyz[a:b, 2], H, 0.01, SEED, int(tag[k]), 5)
        compare_cluster(k, P, Hh, r)


def test_fused_hull_paths():
    import paper_2510_01592_amd as vm
    off, xyz, tag = hull_path_clusters()
    cl, _keep = _view(vm, off, xyz, tag)
    K, H = len(tag), 128
    note("fused: hull paths by survivor count")
    got = _run(vm, cl, H, 1, True, with_all=False)
    _same(got, _run(vm, cl, H, 1, False, with_all=False), K)
    P, Hh = got
    assert P["status"] == 0 and Hh["status"] == 0
    for k in range(K):
        a, b = int(off[k]), int(off[k + 1])
        r = oracle.plane_and_hull(xyz[a:b, 0], xyz[a:b, 1], xyz[a:b, 2], H, 0.01, SEED, int(tag[k]), 1)
        compare_cluster(k, P, Hh, r, check_all_hyp=False)


def test_fused_every_split_identical():
    import paper_2510_01592_amd as vm
    off, xyz, tag = ragged_clusters(seed=9, n_clusters=40, n_max=12_000)
    cl, _keep = _view(vm, off, xyz, tag)
    K, H = len(tag), 320
    try:
        vm.set_fused_config(None)
        base = _run(vm, cl, H, 2, True)
        for cfg in (dict(hyp_chunk=64, small_max=0, groups_per_cu=1), dict(hyp_chunk=128, small_max=64, groups_per_cu=2),
                    dict(hyp_chunk=512, small_max=256, groups_per_cu=8), dict(hyp_chunk=192, small_max=3, groups_per_cu=3)):
            note(f"fused split {cfg}")
            vm.set_fused_config(cfg)
            _same(_run(vm, cl, H, 2, True), base, K)
    finally:
        vm.set_fused_config(None)
    _same(base, _run(vm, cl, H, 2, False), K)


def test_fused_autotune_keeps_results():
    import torch
    import paper_2510_01592_amd as vm
    off, xyz, tag = ragged_clusters(seed=13, n_clusters=50, n_max=20_000)
    cl, _keep = _view(vm, off, xyz, tag)
    K, H = len(tag), 256
    work = torch.empty(vm.workspace_bytes(K, cl.n_cap, H), dtype=torch.uint8, device="cuda")
    pb = vm.PlaneBuffers.alloc(K, cl.n_cap, H, with_all=True)
    hb = vm.HullBuffers.alloc(K, cl.n_cap)
    try:
        note("fused autotune")
        best = vm.autotune_fused(cl, vm.ransac_params(H, 0.01, SEED, 4), pb, hb, work, reps=1)
        assert set(best) == {"hyp_chunk", "small_max", "groups_per_cu"}
        torch.cuda.synchronize()
        _same((planes_np(pb), hulls_np(hb)), _run(vm, cl, H, 4, False), K)
        # the tuned split serves later calls of the same shape, with the same results
        _same(_run(vm, cl, H, 4, True), _run(vm, cl, H, 4, False), K)
    finally:
        vm.set_fused_config(None)


def test_fused_capacity_overflows():
    import paper_2510_01592_amd as vm
    sc = scenes.scene_tiny(0)
    g = sc.geom
    m = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    import torch
    m.insert(torch.from_numpy(scenes.frame_points(sc, 0)).cuda())
    cl = m.ccl(30)
    torch.cuda.synchronize()
    K = vm.read_clusters(cl)["K"]
    assert K == 3
    for k_cap, in_cap, v_cap in ((2, 30000, 10), (4, 1000, 1 << 16), (8, 1 << 17, 5)):
        note(f"fused overflow k_cap={k_cap} in_cap={in_cap} v_cap={v_cap}")
        got = _run(vm, cl, 32, 0, True, k_cap=k_cap, in_cap=in_cap, v_cap=v_cap, with_all=False)
        ref = _run(vm, cl, 32, 0, False, k_cap=k_cap, in_cap=in_cap, v_cap=v_cap, with_all=False)
        _same(got, ref, min(K, k_cap))
        assert got[0]["status"] or got[1]["status"]
    m.close()


def test_fused_batched_2000():
    import paper_2510_01592_amd as vm
    off, xyz = scenes.batched_clusters(seed=3)
    K = len(off) - 1
    tag = np.arange(K, dtype=np.uint32)
    cl, _keep = _view(vm, off, xyz, tag)
    note(f"fused: 2000 clusters, {len(xyz)} points, H=1024")
    got = _run(vm, cl, 1024, 0, True, with_all=False)
    ref = _run(vm, cl, 1024, 0, False, with_all=False)
    assert got[0]["status"] == 0 and got[1]["status"] == 0
    _same(got, ref, K)


def test_multi_sets_equal_each_alone():
    """vm_planes_hulls_multi: several cluster sets with their own frame
    numbers in one pass give each set exactly its alone results; a set that
    does not fit the merged bounds is skipped and flagged."""
    import torch
    import paper_2510_01592_amd as vm
    H = 256
    data = [ragged_clusters(seed=s, n_clusters=n, n_max=m) for s, n, m in ((21, 30, 20_000), (22, 5, 3_000),
                                                                           (23, 45, 9_000))]
    views = [_view(vm, *d) for d in data]
    frames = [5, 9, 2]
    Ks = [len(d[2]) for d in data]
    Ns = [len(d[1]) for d in data]
    k_cap, n_cap = sum(Ks), sum(Ns)
    work = torch.empty(vm.multi_workspace_bytes(k_cap, n_cap, H), dtype=torch.uint8, device="cuda")
    pbs = [vm.PlaneBuffers.alloc(K, N, H, with_all=True) for K, N in zip(Ks, Ns)]
    hbs = [vm.HullBuffers.alloc(K, N) for K, N in zip(Ks, Ns)]
    note("multi: three sets in one pass")
    vm.planes_hulls_multi([v for v, _ in views], frames, vm.ransac_params(H, 0.01, SEED, 0), pbs, hbs, k_cap, n_cap,
                          work)
    torch.cuda.synchronize()
    for i, ((cl, _), f) in enumerate(zip(views, frames)):
        _same((planes_np(pbs[i]), hulls_np(hbs[i])), _run(vm, cl, H, f, True), Ks[i])
    # merged bounds that hold only the first two sets: the third is skipped
    pbs2 = [vm.PlaneBuffers.alloc(K, N, H) for K, N in zip(Ks, Ns)]
    hbs2 = [vm.HullBuffers.alloc(K, N) for K, N in zip(Ks, Ns)]
    k2 = Ks[0] + Ks[1]
    work2 = torch.empty(vm.multi_workspace_bytes(k2, n_cap, H), dtype=torch.uint8, device="cuda")
    note("multi: the third set does not fit")
    vm.planes_hulls_multi([v for v, _ in views], frames, vm.ransac_params(H, 0.01, SEED, 0), pbs2, hbs2, k2, n_cap,
                          work2)
    torch.cuda.synchronize()
    for i in range(2):
        _same((planes_np(pbs2[i]), hulls_np(hbs2[i])), _run(vm, views[i][0], H, frames[i], True, with_all=False), Ks[i])
    assert int(pbs2[2].status.cpu()[0]) & vm.FLAG_CLUSTERS_CAP
    assert int(hbs2[2].status.cpu()[0]) & vm.FLAG_CLUSTERS_CAP
    assert int(pbs2[2].in_off.cpu()[0]) == 0 and int(hbs2[2].v_off.cpu()[0]) == 0


def test_multi_sets_with_small_outputs_equal_each_alone():
    """Merged sets whose own outputs are too small: one set's inlier list
    holds a third of its inliers (later clusters lose their polygons), one
    set's vertex list holds 40 vertices, one set has more clusters than its
    outputs; each gets exactly what it gets alone with the same outputs
    (flags, offsets, the entries that fit)."""
    import torch
    import paper_2510_01592_amd as vm
    H = 256
    data = [ragged_clusters(seed=s, n_clusters=n, n_max=m) for s, n, m in ((31, 25, 20_000), (32, 20, 6_000),
                                                                           (33, 30, 9_000))]
    views = [_view(vm, *d) for d in data]
    frames = [3, 11, 7]
    Ks = [len(d[2]) for d in data]
    Ns = [len(d[1]) for d in data]
    k_cap, n_cap = sum(Ks), sum(Ns)
    caps = [(Ks[0], Ns[0] // 3, Ns[0]), (Ks[1], Ns[1], 40), (Ks[2] - 4, Ns[2], Ns[2])]
    work = torch.empty(vm.multi_workspace_bytes(k_cap, n_cap, H), dtype=torch.uint8, device="cuda")
    pbs = [vm.PlaneBuffers.alloc(kc, ic, H) for kc, ic, _ in caps]
    hbs = [vm.HullBuffers.alloc(kc, vc) for kc, _, vc in caps]
    note("multi: sets with small outputs")
    vm.planes_hulls_multi([v for v, _ in views], frames, vm.ransac_params(H, 0.01, SEED, 0), pbs, hbs, k_cap, n_cap,
                          work)
    torch.cuda.synchronize()
    for i, ((cl, _), f) in enumerate(zip(views, frames)):
        kc, ic, vc = caps[i]
        alone = _run(vm, cl, H, f, False, k_cap=kc, in_cap=ic, v_cap=vc, with_all=False)
        _same((planes_np(pbs[i]), hulls_np(hbs[i])), alone, min(kc, Ks[i]))
    assert int(pbs[0].status.cpu()[0]) & vm.FLAG_INLIERS_CAP
    assert int(hbs[1].status.cpu()[0]) & vm.FLAG_HULL_CAP
    assert int(pbs[2].status.cpu()[0]) & vm.FLAG_CLUSTERS_CAP

"""Graph capture and replay (vm_capture_begin/end, vm_graph_launch): a frame
captured once and replayed with new points in the same buffer and a device
frame counter gives, replay after replay, exactly what direct calls give.
Eager work and synchronisations run between the replays."""
import numpy as np
import pytest

import scenes
from tests.gpu_util import bits, hulls_np, note, planes_np

pytestmark = pytest.mark.gpu

SEED = 0x5EED


def test_segment_frame_graph_replays_match_direct_calls():
    import torch
    import paper_2510_01592_amd as vm
    sc = scenes.scene_tiny(0)
    g = sc.geom
    frames = [torch.from_numpy(scenes.frame_points(sc, 40 + i, n=30_000)).cuda() for i in range(6)]
    s = torch.cuda.Stream()
    ma = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    mb = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    pa, ha = vm.PlaneBuffers.alloc(64, 1 << 17, 64), vm.HullBuffers.alloc(64, 1 << 17)
    pb, hb = vm.PlaneBuffers.alloc(64, 1 << 17, 64), vm.HullBuffers.alloc(64, 1 << 17)
    buf = torch.empty_like(frames[0])
    frame_t = torch.zeros(1, dtype=torch.int32, device="cuda")
    kw = dict(min_cluster=30, n_hyp=64, eps=0.01, seed=SEED)
    with torch.cuda.stream(s):
        note("graph: warm-up call (allocates the map workspace)")
        ma.segment_frame(frames[0], pa, ha, frame=0, **kw, stream=s)
        mb.segment_frame(frames[0], pb, hb, frame=0, **kw, stream=s)
        s.synchronize()
        note("graph: capture")
        with vm.capture(s) as cap:
            ma.segment_frame(buf, pa, ha, d_frame=frame_t, **kw, stream=s)
        graph = cap.graph
    for i in range(1, 6):
        with torch.cuda.stream(s):
            buf.copy_(frames[i])
            frame_t.fill_(i)
            note(f"graph: replay {i}")
            graph.launch(s)
            mb.segment_frame(frames[i], pb, hb, frame=i, **kw, stream=s)
        s.synchronize()
        A, B = planes_np(pa), planes_np(pb)
        for key in ("plane", "best", "nin", "in_off", "in_idx"):
            assert np.array_equal(A[key], B[key]), (i, key)
        HA, HB = hulls_np(ha), hulls_np(hb)
        for key in ("v_off", "v_idx", "area"):
            assert np.array_equal(HA[key], HB[key]), (i, key)
        assert np.array_equal(bits(HA["v_xyz"]), bits(HB["v_xyz"]))
        assert ma.stats(s).occupied == mb.stats(s).occupied
    graph.close()


def test_batched_graph_with_frame_counter():
    import torch
    import paper_2510_01592_amd as vm
    from tests.gpu_util import cluster_tensors
    off, xyz = scenes.batched_clusters(seed=11, n_clusters=40, n_min=50, n_max=20_000)
    K, N = len(off) - 1, len(xyz)
    T = cluster_tensors(off, xyz, np.arange(K, dtype=np.uint32))
    cl = vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"])
    work = torch.empty(vm.workspace_bytes(K, N, 128), dtype=torch.uint8, device="cuda")
    pa, ha = vm.PlaneBuffers.alloc(K, N, 128, with_all=True), vm.HullBuffers.alloc(K, N)
    pb, hb = vm.PlaneBuffers.alloc(K, N, 128, with_all=True), vm.HullBuffers.alloc(K, N)
    frame_t = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        note("batched graph: capture")
        with vm.capture(s) as cap:
            vm.ransac_planes(cl, vm.ransac_params(128, 0.01, SEED, d_frame=frame_t), pa, work, stream=s)
            vm.hulls(cl, pa, ha, work, stream=s)
    for f in (0, 1, 7):
        with torch.cuda.stream(s):
            frame_t.fill_(f)
            note(f"batched graph: replay frame {f}")
            cap.graph.launch(s)
            vm.ransac_planes(cl, vm.ransac_params(128, 0.01, SEED, frame=f), pb, work, stream=s)
            vm.hulls(cl, pb, hb, work, stream=s)
        s.synchronize()
        A, B = planes_np(pa), planes_np(pb)
        for key in ("plane", "best", "in_idx", "counts", "hyp"):
            assert np.array_equal(A[key], B[key]), (f, key)
        assert np.array_equal(hulls_np(ha)["area"], hulls_np(hb)["area"])
    cap.graph.close()

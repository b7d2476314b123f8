"""The served form against the oracle: several robots' posed frames arrive
over time and are processed concurrently (one stream per robot, continuous
admission); every frame's labels, clusters, planes, inlier lists and
polygons equal what the oracle computes replaying that robot's frames alone
(map insert with the frame's pose, then the whole map segmented with the
robot's own frame number)."""
import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_util import bits, note

pytestmark = pytest.mark.gpu

N_HYP, EPS, SEED, MINC = 512, 0.01, 0x5EED, 30


def _robot(r, n_frames):
    import torch
    sc = scenes.scene_full_map(10 + r)
    pool = scenes.surface_pool(sc, 40 + r, 1_000_000)
    poses = scenes.random_walk_poses(60 + r, n_frames, sigma_t=0.01, sigma_rot_deg=0.5)
    rng = np.random.default_rng(80 + r)
    frames = []
    for k in range(n_frames):
        n = int(rng.integers(200_000, 400_001))
        pts = scenes.stream_frame(sc, pool, 500 * r + k, n, poses[k])
        frames.append((pts, poses[k]))
    return sc, frames


def _compare(r, k, got, fr, om):
    where = (r, k)
    assert got["status"].tolist() == [0, 0], where
    assert got["occupied"] == len(om.key), where
    assert np.array_equal(got["labels"], fr.labels), where
    cl = fr.clusters
    K = len(cl.tag)
    assert got["K"] == K and got["N"] == len(cl.key), where
    assert np.array_equal(got["off"], cl.off) and np.array_equal(got["tag"], cl.tag), where
    assert np.array_equal(got["key"], cl.key), where
    assert np.array_equal(bits(got["xyz"]), bits(cl.xyz)), where
    for c, res in enumerate(fr.results):
        rr = res.ransac
        assert got["best"][c] == rr.best_h, (where, c)
        assert np.array_equal(bits(got["plane"][c]), bits(rr.plane if rr.best_h >= 0 else np.zeros(4, np.float32))), \
            (where, c)
        a, b = int(got["in_off"][c]), int(got["in_off"][c + 1])
        assert got["nin"][c] == b - a == len(rr.inliers), (where, c)
        assert np.array_equal(got["in_idx"][a:b], rr.inliers), (where, c)
        va, vb = int(got["v_off"][c]), int(got["v_off"][c + 1])
        if res.hull is None:
            assert vb == va and got["area"][c] == 0.0, (where, c)
            continue
        assert np.array_equal(got["v_idx"][va:vb], res.hull_local), (where, c)
        assert np.array_equal(bits(got["v_xyz"][va:vb]), bits(res.hull.xyz)), (where, c)
        assert abs(got["area"][c] - res.hull.area) <= 1e-5 * max(abs(res.hull.area), 1e-30), (where, c)


@pytest.mark.parametrize("batch", [False, True], ids=["streams", "batched"])
def test_served_frames_equal_oracle_replay(batch):
    import torch

    import paper_2510_01592_amd as vm
    from paper_2510_01592_amd.serve import GpuBackend, Request, Scheduler
    robots, n_frames = 3, 5
    data = [_robot(r, n_frames) for r in range(robots)]
    maps = [vm.Map(sc.geom.origin, sc.geom.voxel_size, sc.geom.dims, 21) for sc, _ in data]
    be = GpuBackend(maps, n_slots=6, n_hyp=N_HYP, k_cap=4096, in_cap=1 << 21, v_cap=1 << 18, capture_cap=1 << 21,
                    batch=batch, batch_k_cap=8192, batch_n_cap=1 << 22)
    # every robot's first frame at t = 0, the rest over 60 ms: frames of
    # different robots overlap on the device
    reqs = []
    for r, (sc, frames) in enumerate(data):
        arr = np.sort(np.random.default_rng(90 + r).uniform(0, 0.06, n_frames))
        arr[0] = 0.0
        for k, (pts, (R, t)) in enumerate(frames):
            reqs.append(Request(r, k, float(arr[k]), len(pts), (torch.from_numpy(pts).pin_memory(), R, t)))
    note(f"served ({'batched' if batch else 'streams'}): 3 robots x 5 posed frames in the mix")
    sch = Scheduler(be, n_robots=robots, n_slots=6, budget_bytes=1 << 28)
    done = sch.run(reqs)
    assert len(done) == robots * n_frames and not sch.rejected
    assert sch.peak_inflight > 1
    if batch:
        assert sch.batched_frames == robots * n_frames and sch.batches < robots * n_frames
    got = {(c.request.robot, c.request.seq): c.result for c in done}
    for r, (sc, frames) in enumerate(data):
        g = sc.geom
        om = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
        for k, (pts, (R, t)) in enumerate(frames):
            om.insert(pts, R, t)
            fr = oracle.segment(om, MINC, N_HYP, EPS, SEED, k, threads=8)
            _compare(r, k, got[(r, k)], fr, om)
    for m in maps:
        m.close()

"""The served form on the GPU: frames of several robots, arriving over time
and processed concurrently (one stream per robot, continuous admission),
give for every robot exactly the results that robot gets alone."""
import numpy as np
import pytest

import scenes
from tests.gpu_util import note

pytestmark = pytest.mark.gpu


def _robot_inputs(r, n_frames):
    import torch
    sc = scenes.scene_tiny(r)
    poses = scenes.random_walk_poses(50 + r, n_frames, sigma_t=0.003, sigma_rot_deg=0.3)
    rng = np.random.default_rng(70 + r)
    frames = []
    for k in range(n_frames):
        n = int(rng.integers(20_000, 80_000))
        pts = scenes.frame_points(sc, 1000 * r + k, n=n, pose=poses[k])
        frames.append((torch.from_numpy(pts).pin_memory(), poses[k][0], poses[k][1]))
    return sc, frames


def _run(robots, inputs, arrivals, n_slots=6, budget=1 << 26):
    import paper_2510_01592_amd as vm
    from paper_2510_01592_amd.serve import GpuBackend, Request, Scheduler
    maps = {}
    for r in robots:
        g = inputs[r][0].geom
        maps[r] = vm.Map(g.origin, g.voxel_size, g.dims, 17)
    order = sorted(robots)
    idx = {r: i for i, r in enumerate(order)}
    be = GpuBackend([maps[r] for r in order], n_slots=n_slots, n_hyp=64, k_cap=256, in_cap=1 << 17, v_cap=1 << 15)
    reqs = []
    for r in order:
        for k, (pts, R, t) in enumerate(inputs[r][1]):
            reqs.append(Request(idx[r], k, float(arrivals[r][k]), int(pts.shape[0]), (pts, R, t)))
    sch = Scheduler(be, n_robots=len(order), n_slots=n_slots, budget_bytes=budget)
    done = sch.run(reqs)
    out = {(order[c.request.robot], c.request.seq): c.result for c in done}
    return out, sch


def test_results_alone_equal_results_in_the_mix():
    robots = [0, 1, 2, 3]
    n_frames = 5
    inputs = {r: _robot_inputs(r, n_frames) for r in robots}
    # every robot's first frame arrives at once (so frames of different
    # robots are in flight together however fast they run), the rest over
    # 50 ms
    arrivals = {r: np.sort(np.random.default_rng(90 + r).uniform(0, 0.05, n_frames)) for r in robots}
    for r in robots:
        arrivals[r][0] = 0.0
    note("serve: 4 robots in the mix")
    mix, sch = _run(robots, inputs, arrivals)
    assert len(mix) == len(robots) * n_frames and not sch.rejected
    assert sch.peak_inflight > 1
    for r in robots:
        note(f"serve: robot {r} alone")
        alone, _ = _run([r], inputs, arrivals)
        for k in range(n_frames):
            a, b = alone[(r, k)], mix[(r, k)]
            assert a["K"] == b["K"] and a["occupied"] == b["occupied"], (r, k)
            assert np.array_equal(a["best"], b["best"]), (r, k)
            assert np.array_equal(a["plane"].view(np.uint32), b["plane"].view(np.uint32)), (r, k)
            assert np.array_equal(a["area"].view(np.uint64), b["area"].view(np.uint64)), (r, k)
            assert np.array_equal(a["v_off"], b["v_off"]), (r, k)
            assert a["status"].tolist() == [0, 0]

"""Host logic of the served form, with a simulated device (no GPU): admission
by arrival, result slots and HBM budget; per-robot order; rejection of frames
larger than the whole budget; overlap of robots (continuous batching)."""
import numpy as np
import pytest

from paper_2510_01592_amd.serve import Backend, Request, Scheduler, latency_summary, poisson_arrivals


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class SimBackend(Backend):
    """Each robot's frames run one after another (its stream); robots overlap.
    Service time proportional to the point count."""

    def __init__(self, clock, per_point_s=1e-9, fixed_s=1e-3):
        self.clock = clock
        self.per_point_s, self.fixed_s = per_point_s, fixed_s
        self.robot_free = {}
        self.active = []          # (finish, slot, robot, seq)
        self.log = []

    def bytes_for(self, req):
        return 12 * req.n_points

    def submit(self, req, slot):
        now = self.clock()
        assert all(sl != slot for fin, sl, _r, _q in self.active if fin > now), "slot reused while in flight"
        start = max(now, self.robot_free.get(req.robot, 0.0))
        fin = start + self.fixed_s + self.per_point_s * req.n_points
        self.robot_free[req.robot] = fin
        self.active.append((fin, slot, req.robot, req.seq))
        self.log.append(("submit", now, req.robot, req.seq, slot))
        return fin

    def done(self, h):
        return self.clock() >= h

    def result(self, h, slot):
        return {"slot": slot}


def _requests(n_robots=4, rate=30.0, dur=1.0, seed=0, sizes=(200_000, 2_000_000)):
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_robots):
        for k, a in enumerate(poisson_arrivals(rate, dur, 100 + r)):
            reqs.append(Request(r, k, float(a), int(rng.integers(sizes[0], sizes[1] + 1))))
    return reqs


def test_all_served_in_order_within_budget():
    clk = Clock()
    be = SimBackend(clk)
    reqs = _requests()
    budget = 64 << 20
    sch = Scheduler(be, n_robots=4, n_slots=6, budget_bytes=budget, per_robot_inflight=2, clock=clk, sleep=clk.sleep)
    done = sch.run(reqs, t0=0.0)
    assert len(done) == len(reqs) and not sch.rejected
    assert sch.peak_used <= budget and sch.peak_inflight <= 6
    for r in range(4):
        seqs = [c.request.seq for c in sorted(done, key=lambda c: c.finished) if c.request.robot == r]
        assert seqs == sorted(seqs)
    for c in done:
        assert c.admitted >= c.request.arrival and c.finished >= c.admitted
        assert c.latency >= be.fixed_s
    s = latency_summary(done, 1.0)
    assert s["frames"] == len(reqs) and s["p99_ms"] >= s["p50_ms"]


def test_robots_overlap_and_late_arrivals_are_admitted_while_others_run():
    clk = Clock()
    be = SimBackend(clk, per_point_s=5e-9, fixed_s=2e-3)
    reqs = _requests(n_robots=8, rate=30.0, dur=0.5, seed=1)
    sch = Scheduler(be, n_robots=8, n_slots=16, budget_bytes=1 << 30, clock=clk, sleep=clk.sleep)
    done = sch.run(reqs, t0=0.0)
    assert len(done) == len(reqs)
    assert sch.peak_inflight > 1
    # some frame was admitted while another robot's earlier frame was still running
    spans = [(c.admitted, c.finished, c.request.robot) for c in done]
    assert any(a2 > a1 and a2 < f1 and r2 != r1 for (a1, f1, r1) in spans for (a2, f2, r2) in spans)


def test_budget_limits_concurrency_and_rejects_oversized():
    clk = Clock()
    be = SimBackend(clk)
    reqs = [Request(0, 0, 0.0, 1000), Request(1, 0, 0.0, 1000), Request(2, 0, 0.0, 10_000_000),
            Request(3, 0, 0.001, 1000)]
    sch = Scheduler(be, n_robots=4, n_slots=4, budget_bytes=12 * 1000, clock=clk, sleep=clk.sleep)
    done = sch.run(reqs, t0=0.0)
    assert [r.robot for r in sch.rejected] == [2]
    assert len(done) == 3
    assert sch.peak_used <= 12 * 1000 and sch.peak_inflight == 1


def test_slot_and_per_robot_limits():
    clk = Clock()
    be = SimBackend(clk)
    reqs = [Request(0, k, 0.0, 1000) for k in range(5)]
    sch = Scheduler(be, n_robots=1, n_slots=8, budget_bytes=1 << 30, per_robot_inflight=2, clock=clk,
                    sleep=clk.sleep)
    done = sch.run(reqs, t0=0.0)
    assert len(done) == 5 and sch.peak_inflight <= 2
    with pytest.raises(ValueError):
        Scheduler(be, 1, 0, 1 << 20)


class SimBatchBackend(SimBackend):
    """Frames admitted together form one batch: it starts when its slowest
    robot is free and all of its frames finish together."""

    batching = True

    def __init__(self, clock, **kw):
        super().__init__(clock, **kw)
        self.batches = []

    def submit_batch(self, items):
        now = self.clock()
        robots = [req.robot for req, _ in items]
        assert len(set(robots)) == len(robots), "one frame per robot per batch"
        start = max([now] + [self.robot_free.get(r, 0.0) for r in robots])
        fin = start + self.fixed_s + self.per_point_s * sum(req.n_points for req, _ in items)
        for req, slot in items:
            assert all(sl != slot for f, sl, _r, _q in self.active if f > now), "slot reused while in flight"
            self.robot_free[req.robot] = fin
            self.active.append((fin, slot, req.robot, req.seq))
            self.log.append(("submit", now, req.robot, req.seq, slot))
        self.batches.append(len(items))
        return [fin] * len(items)


def test_batching_admission_rounds():
    clock = Clock()
    be = SimBatchBackend(clock, per_point_s=2e-10, fixed_s=2e-3)
    reqs = _requests(n_robots=6, rate=60.0, dur=0.5, seed=3)
    sch = Scheduler(be, 6, n_slots=8, budget_bytes=1 << 30, clock=clock, sleep=clock.sleep)
    done = sch.run(reqs)
    assert len(done) == len(reqs) and not sch.rejected
    assert sch.batches == len(be.batches) and sch.batched_frames == len(reqs)
    assert max(be.batches) > 1          # robots do share batches
    # per-robot order is kept
    for r in range(6):
        seqs = [e[3] for e in be.log if e[2] == r]
        assert seqs == sorted(seqs)

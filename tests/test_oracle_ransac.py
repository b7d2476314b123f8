"""Pins for the oracle's cluster RANSAC (Sec. III-C, "Multi-plane estimation").

(a) each hypothesis samples three distinct points and takes their plane,
(b) counts the cluster's points closer than eps = 0.01 m to it,
(c) the hypothesis with the most inliers wins and its inliers are extracted.
The pins use exact rational distances, brute force over every triple of a
small cluster, exact recovery of noise-free planes (cross-checked with an
SVD fit), and the degenerate cases."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

EPS = np.float32(0.01)


def _exact_dist(plane, p):
    nx, ny, nz, d = (Fraction(float(v)) for v in plane)
    return abs(nx * Fraction(float(p[0])) + ny * Fraction(float(p[1])) + nz * Fraction(float(p[2])) + d)


def test_draw3_distinct_in_range_and_uniform():
    for n in (3, 4, 5, 17, 1000, 2 ** 31 + 7):
        for h in range(300):
            a, b, c = oracle.draw3(0x5EED, 99, 4, h, n)
            assert len({a, b, c}) == 3 and max(a, b, c) < n
    # every ordered triple of 5 points is about equally likely
    hist = {}
    N = 60000
    for h in range(N):
        t = oracle.draw3(1, 2, 3, h, 5)
        hist[t] = hist.get(t, 0) + 1
    assert len(hist) == 60
    expect = N / 60
    chi2 = sum((v - expect) ** 2 / expect for v in hist.values())
    assert chi2 < 120            # 59 dof; p ~ 1e-5 bound


def test_hypothesis_planes_pass_through_their_triples():
    rng = np.random.default_rng(0)
    pts = rng.normal(size=(50, 3)).astype(np.float32)
    r = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], 64, EPS, 7, 123, 0)
    for h in range(64):
        pl = r.hyp[h]
        a, b, c = oracle.draw3(7, 123, 0, h, 50)
        nrm = math.sqrt(sum(float(v) ** 2 for v in pl[:3]))
        assert abs(nrm - 1) < 1e-6
        # fixed orientation: +z, then +y, then +x
        assert pl[2] > 0 or (pl[2] == 0 and (pl[1] > 0 or (pl[1] == 0 and pl[0] > 0)))
        for i in (a, b, c):
            assert float(_exact_dist(pl, pts[i])) < 1e-5
        # independent plane through the triple (numpy float64) agrees
        n = np.cross(pts[b].astype(np.float64) - pts[a], pts[c].astype(np.float64) - pts[a])
        n /= np.linalg.norm(n)
        n *= np.sign(n[2])
        assert np.allclose(n, pl[:3], atol=1e-6)


def test_counts_match_exact_distance():
    rng = np.random.default_rng(1)
    pts = np.concatenate([
        np.c_[rng.uniform(-1, 1, (400, 2)), rng.normal(0, 0.006, 400)],
        rng.uniform(-1, 1, (100, 3))]).astype(np.float32)
    r = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], 32, EPS, 3, 5, 1)
    epsq = Fraction(float(EPS))
    for h in range(32):
        if r.counts[h] < 0:
            continue
        exact = 0
        ambiguous = 0
        for p in pts:
            dd = _exact_dist(r.hyp[h], p)
            exact += dd < epsq
            ambiguous += abs(dd - epsq) < Fraction(1, 10 ** 6)
        assert abs(int(r.counts[h]) - exact) <= ambiguous


def test_best_is_first_maximum_and_inliers_are_its_points():
    rng = np.random.default_rng(2)
    pts = np.concatenate([np.c_[rng.uniform(-1, 1, (300, 2)), rng.normal(0, 0.005, 300)],
                          rng.uniform(-1, 1, (300, 3))]).astype(np.float32)
    r = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], 128, EPS, 9, 1, 0)
    assert r.best_h == int(np.argmax(r.counts))          # argmax returns the first maximum
    assert np.array_equal(r.plane, r.hyp[r.best_h])
    assert len(r.inliers) == r.counts[r.best_h]
    assert np.all(np.diff(r.inliers.astype(np.int64)) > 0)
    d = [float(_exact_dist(r.plane, pts[i])) for i in r.inliers]
    assert max(d) < 0.01 + 1e-6


def _two_planes(rng, n1, n2, n_out):
    # points on z = 0 and on x = 0.5 (far apart), outliers far from both
    a = np.c_[rng.uniform(-1, 0, (n1, 2)), np.zeros(n1)]
    b = np.c_[np.full(n2, 0.5), rng.uniform(0.2, 1.0, (n2, 2))]
    o = np.c_[rng.uniform(1.5, 2.5, (n_out, 2)), rng.uniform(1.5, 2.5, n_out)]
    return np.concatenate([a, b, o]).astype(np.float32)


def test_brute_force_all_triples():
    rng = np.random.default_rng(4)
    for trial in range(6):
        pts = _two_planes(rng, 9, 6, 5)          # n = 20, C(20,3) = 1140 triples
        pts = pts[rng.permutation(len(pts))]
        n = len(pts)
        H = 4000
        r = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], H, EPS, 100 + trial, trial, 0)
        epsq = Fraction(float(EPS))

        def count_for(triple):
            a, b, c = (pts[i].astype(np.float64) for i in triple)
            nrm = np.cross(b - a, c - a)
            if np.dot(nrm, nrm) < 1e-24:
                return -1
            nrm /= np.linalg.norm(nrm)
            pl = np.r_[nrm, -np.dot(nrm, a)].astype(np.float32)
            return sum(_exact_dist(pl, p) < epsq for p in pts)

        all_counts = {t: count_for(t) for t in itertools.combinations(range(n), 3)}
        drawn = {tuple(sorted(oracle.draw3(100 + trial, trial, 0, h, n))) for h in range(H)}
        best_drawn = max(all_counts[t] for t in drawn)
        assert r.counts[r.best_h] == best_drawn
        best_all = max(all_counts.values())
        if any(all_counts[t] == best_all for t in drawn):
            assert r.counts[r.best_h] == best_all == 9


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_exact_recovery_noise_free(seed):
    rng = np.random.default_rng(seed)
    nrm = rng.normal(size=3)
    nrm[2] = abs(nrm[2]) + 0.5
    nrm /= np.linalg.norm(nrm)
    d = rng.uniform(-0.5, 0.5)
    u = np.cross(nrm, [1.0, 0.0, 0.0]); u /= np.linalg.norm(u)
    v = np.cross(nrm, u)
    s = rng.uniform(-0.5, 0.5, size=(2000, 2))
    pts = (-d * nrm[None, :] + s[:, :1] * u + s[:, 1:] * v).astype(np.float32)
    r = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], 256, EPS, seed, 17, 2)
    valid = r.counts >= 0
    assert np.all(r.counts[valid] == 2000)
    assert r.best_h == int(np.argmax(valid))
    assert np.allclose(r.plane[:3], nrm, atol=1e-6) and abs(r.plane[3] - d) < 1e-6
    # an SVD fit of the centred points agrees
    c = pts.astype(np.float64).mean(axis=0)
    _, _, vt = np.linalg.svd(pts.astype(np.float64) - c)
    n_svd = vt[-1] * np.sign(vt[-1][2])
    assert np.allclose(n_svd, r.plane[:3], atol=1e-5)
    assert abs(-np.dot(n_svd, c) - r.plane[3]) < 1e-5


def test_far_outliers_are_never_counted():
    rng = np.random.default_rng(8)
    plane_pts = np.c_[rng.uniform(-1, 1, (600, 2)), rng.normal(0, 0.001, 600)]
    out = np.c_[rng.uniform(-1, 1, (400, 2)), rng.choice([-1, 1], 400) * rng.uniform(0.03, 0.5, 400)]
    pts = np.concatenate([plane_pts, out]).astype(np.float32)
    pts = pts[rng.permutation(1000)]
    r = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], 256, EPS, 1, 1, 0)
    # P(no hypothesis drew three plane points) = (1 - 0.6^3)^256 < 1e-26
    assert r.counts[r.best_h] == 600
    assert np.all(np.abs(pts[r.inliers, 2]) < 0.01)


def test_degenerate_cases():
    t = np.linspace(0, 1, 50)
    line = np.c_[t, 2 * t, -t].astype(np.float32)
    r = oracle.ransac(line[:, 0], line[:, 1], line[:, 2], 64, EPS, 0, 0, 0)
    assert r.best_h == -1 and np.all(r.counts == -1) and len(r.inliers) == 0
    same = np.ones((10, 3), np.float32)
    assert oracle.ransac(same[:, 0], same[:, 1], same[:, 2], 16, EPS, 0, 0, 0).best_h == -1
    two = np.eye(3, dtype=np.float32)[:2]
    assert oracle.ransac(two[:, 0], two[:, 1], two[:, 2], 16, EPS, 0, 0, 0).best_h == -1
    three = np.eye(3, dtype=np.float32)
    r = oracle.ransac(three[:, 0], three[:, 1], three[:, 2], 16, EPS, 0, 0, 0)
    assert r.best_h == 0 and list(r.inliers) == [0, 1, 2]
    assert np.allclose(r.plane[:3], np.ones(3) / math.sqrt(3), atol=1e-7)


def test_streams_differ_by_tag_and_frame():
    rng = np.random.default_rng(3)
    pts = rng.normal(size=(100, 3)).astype(np.float32)
    a = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], 32, EPS, 5, 1, 0)
    b = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], 32, EPS, 5, 2, 0)
    c = oracle.ransac(pts[:, 0], pts[:, 1], pts[:, 2], 32, EPS, 5, 1, 1)
    assert not np.array_equal(a.hyp, b.hyp) and not np.array_equal(a.hyp, c.hyp)

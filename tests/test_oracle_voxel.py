"""Pins for the oracle's voxel update (Sec. III-B, Eq. (1)).

Eq. (1) keeps a running mean: mu <- (c mu + p)/(c + 1), c <- c + 1.  By
induction that recurrence equals the arithmetic mean of the voxel's points.
The oracle stores the mean exactly as integer sums of fixed-point offsets
(quantum s/2^20), so its result is checked here against exact rational
arithmetic, against cell-membership properties that any voxelisation must
satisfy, and against order independence."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenes
from tests.exact import round_to_f32


def _mean_by_recurrence(ps):
    mu, c = None, 0
    for p in ps:
        mu = p if c == 0 else (c * mu + p) / (c + 1)       # Eq. (1)
        c += 1
    return mu


def _ulp32(x: float) -> float:
    return float(np.spacing(np.float32(abs(x)) if x != 0 else np.float32(1e-38)))


def test_recurrence_equals_arithmetic_mean():
    rng = np.random.default_rng(0)
    for _ in range(50):
        ps = [Fraction(float(v)) for v in rng.normal(size=rng.integers(1, 40))]
        assert _mean_by_recurrence(ps) == sum(ps) / len(ps)


def _random_pose(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    return R, rng.uniform(-0.02, 0.02, size=3)


@pytest.mark.parametrize("posed", [False, True])
def test_mean_matches_exact_rational_mean(posed):
    rng = np.random.default_rng(11 if posed else 10)
    origin, s, dims = (-0.24, -0.24, -0.24), 0.01, (48, 48, 48)
    # clumps of points so that many voxels hold several points
    centres = rng.uniform(-0.1, 0.1, size=(40, 3))
    pts = (centres[rng.integers(0, 40, size=3000)] + rng.normal(0, 0.004, size=(3000, 3))).astype(np.float32)
    R, t = _random_pose(rng) if posed else (np.eye(3), np.zeros(3))
    m = oracle.OracleMap(origin, s, dims)
    m.insert(pts, R, t)
    mu = m.means()
    key, frac, kept = oracle.voxelize(pts, R, t, origin, s, dims)
    q = s / 2 ** 20
    checked = 0
    for vi in rng.choice(len(m.key), size=min(200, len(m.key)), replace=False):
        members = np.nonzero(key == m.key[vi])[0]
        assert len(members) == m.cnt[vi]
        for a in range(3):
            # exact rational position of each member after the pose
            ex = [sum(Fraction(float(R[a, b])) * Fraction(float(pts[i, b])) for b in range(3))
                  + Fraction(float(t[a])) for i in members]
            mean = sum(ex) / len(ex)
            err = abs(Fraction(float(mu[vi, a])) - mean)
            assert err <= Fraction(2 * q) + Fraction(_ulp32(float(mu[vi, a])) / 2) + Fraction(1, 10 ** 12)
        checked += 1
    assert checked > 50


def test_cell_membership_and_offsets():
    rng = np.random.default_rng(3)
    origin, s, dims = np.array([-0.5, -0.25, 0.125]), 0.01, np.array([100, 50, 20])
    pts = rng.uniform(origin - 0.05, origin + s * dims + 0.05, size=(20000, 3)).astype(np.float32)
    key, frac, kept = oracle.voxelize(pts, np.eye(3), np.zeros(3), origin, s, dims)
    lo_ok = np.all((pts >= origin) & (pts < origin + s * dims), axis=1)
    # points clearly inside are kept, clearly outside are dropped
    margin = 1e-6
    inside = np.all((pts > origin + margin) & (pts < origin + s * dims - margin), axis=1)
    outside = ~np.all((pts > origin - margin) & (pts < origin + s * dims + margin), axis=1)
    assert np.all(key[inside] != oracle.NO_KEY)
    assert np.all(key[outside] == oracle.NO_KEY)
    assert kept == int(np.sum(key != oracle.NO_KEY))
    ok = np.nonzero(key != oracle.NO_KEY)[0]
    k = key[ok].astype(np.int64)
    idx = np.stack([k % dims[0], (k // dims[0]) % dims[1], k // (dims[0] * dims[1])], axis=1)
    for j in rng.choice(len(ok), size=500, replace=False):
        i = ok[j]
        for a in range(3):
            p = Fraction(float(pts[i, a]))
            o = Fraction(float(origin[a]))
            S = Fraction(s)
            lo = o + (idx[j, a] + Fraction(int(frac[i, a]), 2 ** 20)) * S
            hi = o + (idx[j, a] + Fraction(int(frac[i, a]) + 1, 2 ** 20)) * S
            tol = Fraction(1, 10 ** 13)
            assert lo - tol <= p < hi + tol
    assert np.all(lo_ok[inside])


def test_faces_belong_to_upper_voxel():
    # exactly representable geometry: s = 0.25, origin 0
    origin, s, dims = (0.0, 0.0, 0.0), 0.25, (8, 8, 8)
    pts = np.array([[0.25, 0.5, 0.75], [0.0, 0.0, 0.0], [1.0, 1.25, 1.5]], np.float32)
    key, frac, kept = oracle.voxelize(pts, np.eye(3), np.zeros(3), origin, s, dims)
    assert list(key) == [1 + 8 * (2 + 8 * 3), 0, 4 + 8 * (5 + 8 * 6)]
    assert np.all(frac == 0)
    # the upper face of the grid is outside (half-open cells)
    key2, _, kept2 = oracle.voxelize(np.array([[2.0, 0.1, 0.1], [1.999, 0.1, 0.1]], np.float32),
                                     np.eye(3), np.zeros(3), origin, s, dims)
    assert key2[0] == oracle.NO_KEY and key2[1] == 7 + 8 * 0 and kept2 == 1


def test_non_finite_points_dropped():
    pts = np.array([[np.nan, 0.1, 0.1], [0.1, np.inf, 0.1], [0.1, 0.1, -np.inf], [0.1, 0.1, 0.1]], np.float32)
    m = oracle.OracleMap((0, 0, 0), 0.01, (64, 64, 64))
    m.insert(pts)
    assert m.points_dropped == 3 and m.points_in == 1 and len(m.key) == 1


def test_identity_pose_is_exact():
    rng = np.random.default_rng(5)
    pts = rng.uniform(0, 1, size=(1000, 3)).astype(np.float32)
    origin, s, dims = (0.0, 0.0, 0.0), 1.0 / 64, (64, 64, 64)      # binary-exact grid
    key, frac, _ = oracle.voxelize(pts, np.eye(3), np.zeros(3), origin, s, dims)
    # with a power-of-two voxel the fixed point is the exact binary expansion
    q = np.floor(pts.astype(np.float64) * 64 * 2 ** 20).astype(np.int64)
    k = (q[:, 0] >> 20) + 64 * ((q[:, 1] >> 20) + 64 * (q[:, 2] >> 20))
    assert np.array_equal(key.astype(np.int64), k)
    assert np.array_equal(frac.astype(np.int64), q & 0xFFFFF)


def test_order_and_batching_independence():
    sc = scenes.scene_tiny(0)
    pts = scenes.frame_points(sc, 0)[:20000]
    g = sc.geom
    a = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    a.insert(pts)
    b = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    perm = np.random.default_rng(1).permutation(len(pts))
    b.insert(pts[perm][:7000])
    b.insert(pts[perm][7000:])
    assert np.array_equal(a.key, b.key) and np.array_equal(a.cnt, b.cnt) and np.array_equal(a.sums, b.sums)
    assert np.array_equal(a.means().view(np.uint32), b.means().view(np.uint32))


def test_noise_free_floor_mean_is_zero():
    sc = scenes.scene_tiny_exact(0)
    pts = scenes.frame_points(sc, 0)
    g = sc.geom
    floor = pts[np.abs(pts[:, 2]) < 1e-6]
    m = oracle.OracleMap(g.origin, g.voxel_size, g.dims)
    m.insert(floor)
    assert np.max(np.abs(m.means()[:, 2])) <= 1e-9


def test_round_to_f32_helper():
    rng = np.random.default_rng(0)
    for v in rng.normal(size=200) * 10.0 ** rng.integers(-30, 30, size=200):
        assert round_to_f32(Fraction(float(v))) == float(np.float32(v)) or \
            abs(float(np.float32(v)) - v) == abs(round_to_f32(Fraction(float(v))) - v)

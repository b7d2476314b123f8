"""Pins of the oracle's voxel clearing (Sec. III-B, Eq. (2)): the rays'
voxel paths against the properties that define a 3D Bresenham line (length,
26-connected unit steps on the driving axis, every minor coordinate within
half a voxel of the ideal line, exact axis-aligned and diagonal paths, the
cut at the grid's faces), and the clearing rule (voxels passed through are
removed, voxels holding a point of the frame are kept, the result does not
depend on the point order, a moved object disappears)."""
import numpy as np
import pytest

import oracle

DIMS = (50, 40, 30)


@pytest.mark.parametrize("seed", range(4))
def test_ray_paths_are_bresenham_lines(seed):
    rng = np.random.default_rng(seed)
    for _ in range(300):
        a = rng.integers(0, DIMS)
        b = rng.integers(0, DIMS)
        p = oracle.ray_voxels(a, b, DIMS)
        d = b - a
        dm = int(np.abs(d).max())
        assert len(p) == dm
        if dm == 0:
            continue
        assert np.array_equal(p[0], a)
        m = int(np.argmax(np.abs(d)))                 # first axis of the largest extent
        steps = np.diff(np.vstack([p, b]), axis=0)
        assert np.all(np.abs(steps) <= 1)              # 26-connected
        assert np.all(steps[:, m] == np.sign(d[m]))    # the driving axis moves every step
        for k in range(3):                             # minor axes: within half a voxel of the line
            ideal = a[k] + d[k] * np.arange(dm) / dm
            assert np.all(np.abs(p[:, k] - ideal) <= 0.5 + 1e-12)


def test_axis_and_diagonal_rays():
    p = oracle.ray_voxels([3, 5, 7], [10, 5, 7], DIMS)
    assert np.array_equal(p, np.c_[np.arange(3, 10), np.full(7, 5), np.full(7, 7)])
    p = oracle.ray_voxels([20, 20, 20], [14, 14, 14], DIMS)
    assert np.array_equal(p, np.repeat(np.arange(20, 14, -1)[:, None], 3, axis=1))
    # a ray to a point outside the grid stops at the grid's face
    p = oracle.ray_voxels([45, 20, 10], [70, 20, 10], DIMS)
    assert np.array_equal(p[:, 0], np.arange(45, 50))


def _map_with(cells, s=0.01):
    om = oracle.OracleMap((0.0, 0.0, 0.0), s, DIMS)
    om.insert(((np.asarray(cells, np.float64) + 0.5) * s).astype(np.float32))
    return om


def _key(c):
    return int(c[0] + DIMS[0] * (c[1] + DIMS[1] * c[2]))


def _clear(om, pts_map, sensor):
    """clear with the sensor at `sensor` (identity rotation): the points are
    handed over in the sensor frame, as a frame arrives"""
    return om.clear_rays((np.asarray(pts_map, np.float64) - sensor).astype(np.float32), np.eye(3), sensor)


def test_wall_between_sensor_and_point_is_cleared():
    s = 0.01
    wall = [[20, y, z] for y in range(10, 30) for z in range(5, 25)]
    om = _map_with(wall)
    sensor = np.array([5.5, 20.5, 15.5]) * s
    target = np.array([[40.5, 20.5, 15.5], [40.5, 12.5, 8.5]]) * s
    removed = _clear(om, target, sensor)
    # each ray crosses the wall in exactly one voxel
    assert removed == 2
    assert _key([20, 20, 15]) not in set(om.key.tolist())
    # the same rays with a point inside the wall: its voxel holds a point, kept
    om2 = _map_with(wall)
    pts = np.vstack([target, np.array([[20.5, 20.5, 15.5]]) * s])
    removed2 = _clear(om2, pts, sensor)
    assert removed2 == 1 and _key([20, 20, 15]) in set(om2.key.tolist())


def test_clearing_does_not_depend_on_point_order():
    rng = np.random.default_rng(5)
    cells = rng.integers(0, DIMS, size=(3000, 3))
    pts = (rng.uniform(0, 1, (2000, 3)) * np.array(DIMS) * 0.01).astype(np.float32)
    sensor = np.array([0.25, 0.2, 0.15])
    a, b = _map_with(cells), _map_with(cells)
    na = _clear(a, pts, sensor)
    nb = _clear(b, pts[rng.permutation(len(pts))], sensor)
    assert na == nb > 0
    assert np.array_equal(a.key, b.key) and np.array_equal(a.cnt, b.cnt) and np.array_equal(a.sums, b.sums)
    # what is left: exactly the voxels not on any ray, or holding a point
    kept = set(a.key.tolist())
    # (the voxels of the points as the map sees them: sensor frame + t, in float32 then fp64)
    sens = (pts.astype(np.float64) - sensor).astype(np.float32).astype(np.float64) + sensor
    vox = np.floor(sens / 0.01).astype(np.int64)
    own = {_key(v) for v in vox}
    on_ray = set()
    sv = np.floor(sensor / 0.01).astype(np.int64)
    for v in vox:
        for c in oracle.ray_voxels(sv, v, DIMS):
            on_ray.add(_key(c))
    before = set(_map_with(cells).key.tolist())
    assert kept == {k for k in before if k not in on_ray or k in own}


def test_moved_object_is_removed():
    s = 0.01
    # frame 1: a box at x = 25; frame 2: the box has gone, the wall behind it at x = 40 is seen
    box = [[x, y, z] for x in range(24, 27) for y in range(18, 23) for z in range(13, 18)]
    om = _map_with(box)
    wall_pts = np.array([[40.5, y + 0.5, z + 0.5] for y in range(10, 30) for z in range(5, 25)]) * s
    sensor = np.array([5.5, 20.5, 15.5]) * s
    _clear(om, wall_pts, sensor)
    om.insert(wall_pts.astype(np.float32))
    keys = set(om.key.tolist())
    # the box's voxels facing the sensor are gone
    assert _key([24, 20, 15]) not in keys
    assert all(_key([40, y, z]) in keys for y in range(10, 30) for z in range(5, 25))
    with pytest.raises(ValueError):
        _clear(om, wall_pts, np.array([-1.0, 0.2, 0.1]))

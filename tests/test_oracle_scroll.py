"""Pins of the oracle's map scrolling (Sec. III-B, the robot-centric local
map): on a dyadic grid, where voxelisation is exact, shifting a map equals
building it with the shifted origin from the points that stay inside;
shifting there and back keeps exactly the voxels that never left; a voxel
lands on the key its coordinates give."""
import numpy as np

import oracle

S = 2.0 ** -6            # voxel edge 1/64 m: every quantity below is exact in float32 and fp64
DIMS = (40, 32, 24)


def _points(rng, n):
    # multiples of 2^-12 m inside a slightly larger box than the grid
    q = rng.integers(-200, np.array(DIMS) * 64 + 200, size=(n, 3))
    return (q * 2.0 ** -12).astype(np.float32)


def test_shift_equals_rebuilding_with_the_shifted_origin():
    """the points stored before the shift (those inside the original grid),
    inserted into a grid whose origin is already shifted, give the same map"""
    rng = np.random.default_rng(1)
    pts = _points(rng, 20_000)
    inside = np.all((pts >= 0) & (pts < np.array(DIMS, np.float32) * np.float32(S)), axis=1)
    for d in ((3, -2, 1), (-7, 0, 0), (0, 0, 5), (40, 0, 0), (1, 1, 1)):
        a = oracle.OracleMap((0.0, 0.0, 0.0), S, DIMS)
        a.insert(pts)
        n0 = len(a.key)
        dropped = a.shift(*d)
        b = oracle.OracleMap(tuple(np.array(d) * S), S, DIMS)
        b.insert(pts[inside])
        assert np.array_equal(a.origin, b.origin)
        assert np.array_equal(a.key, b.key) and np.array_equal(a.cnt, b.cnt) and np.array_equal(a.sums, b.sums)
        assert np.array_equal(a.means(), b.means())
        assert dropped == n0 - len(a.key) and dropped > 0
        if d[0] == DIMS[0]:   # a shift by the whole width of the grid empties it
            assert len(a.key) == 0


def test_there_and_back_keeps_the_voxels_that_stayed():
    rng = np.random.default_rng(2)
    a = oracle.OracleMap((0.25, -0.5, 0.125), S, DIMS)
    a.insert(_points(rng, 20_000) + np.float32(0.25))
    before = (a.key.copy(), a.cnt.copy(), a.sums.copy())
    NX, NY = DIMS[0], DIMS[1]
    x, y, z = before[0] % NX, (before[0] // NX) % NY, before[0] // (NX * NY)
    stays = (x >= 5) & (y < NY - 3)
    a.shift(5, -3, 0)
    a.shift(-5, 3, 0)
    assert np.array_equal(a.key, before[0][stays])
    assert np.array_equal(a.cnt, before[1][stays]) and np.array_equal(a.sums, before[2][stays])


def test_a_voxel_lands_where_its_coordinates_say():
    a = oracle.OracleMap((0.0, 0.0, 0.0), S, DIMS)
    p = ((np.array([[10, 7, 3]]) + 0.25) * S).astype(np.float32)
    a.insert(p)
    a.shift(4, -2, 1)
    assert a.key.tolist() == [(10 - 4) + DIMS[0] * ((7 + 2) + DIMS[1] * (3 - 1))]
    assert np.allclose(a.means(), p)

"""Pins for the oracle's clustering (Sec. III-C, Alg. 1).

Alg. 1 propagates the smaller label across every adjacency until nothing
changes; from initial labels L_i = i its fixed point gives every voxel the
smallest initial label in its connected component.  The oracle computes that
fixed point by breadth-first search over 26-neighbours.  It is pinned here
against (i) Alg. 1's own propagation loop run to convergence on tiny grids,
(ii) an independent union-find, (iii) scipy.ndimage.label, and (iv) special
cases with known component counts."""
import itertools

import numpy as np
import pytest
from scipy import ndimage

import oracle

OFFS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def _keys_of(grid):
    # grid indexed [z, y, x]; key = x + NX (y + NY z) is the C-order flat index
    return np.flatnonzero(grid.ravel()).astype(np.uint32)


def _dims_of(grid):
    nz, ny, nx = grid.shape
    return (nx, ny, nz)


def _label_propagation(grid):
    """Alg. 1, run sequentially: repeat 'both ends take the smaller label' over
    all adjacent pairs until no label changes."""
    nz, ny, nx = grid.shape
    occ = [tuple(p) for p in np.argwhere(grid)]
    lab = {p: p[2] + nx * (p[1] + ny * p[0]) for p in occ}
    changed = True
    while changed:
        changed = False
        for p in occ:
            for dz, dy, dx in OFFS:
                q = (p[0] + dz, p[1] + dy, p[2] + dx)
                if q in lab and lab[q] != lab[p]:
                    m = min(lab[p], lab[q])
                    changed = changed or lab[p] != m or lab[q] != m
                    lab[p] = lab[q] = m
    return np.array([lab[p] for p in occ], dtype=np.uint32)


def _union_find(grid):
    nz, ny, nx = grid.shape
    keys = _keys_of(grid)
    pos = {int(k): i for i, k in enumerate(keys)}
    parent = list(range(len(keys)))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i, k in enumerate(keys):
        x, y, z = int(k) % nx, (int(k) // nx) % ny, int(k) // (nx * ny)
        for dz, dy, dx in OFFS:
            xx, yy, zz = x + dx, y + dy, z + dz
            if 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                j = pos.get(xx + nx * (yy + ny * zz))
                if j is not None:
                    a, b = find(i), find(j)
                    if a != b:
                        parent[max(a, b)] = min(a, b)
    return np.array([keys[find(i)] for i in range(len(keys))], dtype=np.uint32)


def test_against_label_propagation_tiny():
    rng = np.random.default_rng(0)
    for _ in range(60):
        shape = tuple(int(v) for v in rng.integers(1, 6, size=3))
        grid = rng.random(shape) < rng.uniform(0.1, 0.6)
        lab, _ = oracle.ccl26(_keys_of(grid), _dims_of(grid))
        assert np.array_equal(lab, _label_propagation(grid))


def test_against_union_find_many():
    rng = np.random.default_rng(1)
    for _ in range(1500):
        shape = tuple(int(v) for v in rng.integers(1, 7, size=3))
        grid = rng.random(shape) < rng.uniform(0.1, 0.6)
        lab, nc = oracle.ccl26(_keys_of(grid), _dims_of(grid))
        ref = _union_find(grid)
        assert np.array_equal(lab, ref)
        assert nc == len(np.unique(ref))


@pytest.mark.parametrize("shape,p,seed", [((40, 64, 64), 0.08, 0), ((60, 80, 100), 0.03, 1),
                                          ((20, 200, 200), 0.12, 2), ((30, 30, 30), 0.3, 3)])
def test_against_scipy(shape, p, seed):
    grid = np.random.default_rng(seed).random(shape) < p
    keys = _keys_of(grid)
    lab, nc = oracle.ccl26(keys, _dims_of(grid))
    sl, n = ndimage.label(grid, structure=np.ones((3, 3, 3), dtype=int))
    s = sl.ravel()[keys]
    assert nc == n
    # same partition: map scipy labels to the smallest key of each component
    mins = np.full(n + 1, np.iinfo(np.uint64).max, dtype=np.uint64)
    np.minimum.at(mins, s, keys.astype(np.uint64))
    assert np.array_equal(lab.astype(np.uint64), mins[s])


def test_full_map_size_against_scipy():
    # a dense grid of the 4x4x2 m map's size (400x400x200) with planar slabs and noise
    rng = np.random.default_rng(7)
    grid = rng.random((200, 400, 400)) < 0.01
    grid[10:12, :, :] = True
    grid[40, 50:150, 20:300] = True
    grid[100:102, 300:380, 100:200] = True
    keys = _keys_of(grid)
    lab, nc = oracle.ccl26(keys, _dims_of(grid))
    sl, n = ndimage.label(grid, structure=np.ones((3, 3, 3), dtype=int))
    assert nc == n
    s = sl.ravel()[keys]
    mins = np.full(n + 1, np.iinfo(np.uint64).max, dtype=np.uint64)
    np.minimum.at(mins, s, keys.astype(np.uint64))
    assert np.array_equal(lab.astype(np.uint64), mins[s])


def test_checkerboard_is_one_component():
    z, y, x = np.indices((6, 6, 6))
    grid = (x + y + z) % 2 == 0
    lab, nc = oracle.ccl26(_keys_of(grid), _dims_of(grid))
    assert nc == 1 and np.all(lab == 0)
    # with 6-connectivity the same grid falls apart into single voxels
    assert ndimage.label(grid)[1] == grid.sum()


def test_slabs_gap():
    grid = np.zeros((5, 8, 8), bool)
    grid[0] = True
    grid[2] = True
    lab, nc = oracle.ccl26(_keys_of(grid), _dims_of(grid))
    assert nc == 2 and set(lab.tolist()) == {0, 2 * 64}
    grid[1, 3, 3] = True
    lab, nc = oracle.ccl26(_keys_of(grid), _dims_of(grid))
    assert nc == 1 and np.all(lab == 0)


def test_diagonal_corner_touch_and_singletons():
    grid = np.zeros((4, 4, 4), bool)
    grid[0, 0, 0] = grid[1, 1, 1] = True       # corner neighbours: joined
    grid[3, 3, 3] = True                       # alone
    lab, nc = oracle.ccl26(_keys_of(grid), _dims_of(grid))
    assert nc == 2 and list(lab) == [0, 0, 63]


def test_row_wrap_is_not_adjacency():
    # x = NX-1 in one row and x = 0 in the next row are not neighbours
    grid = np.zeros((1, 3, 5), bool)
    grid[0, 0, 4] = True
    grid[0, 2, 0] = True
    lab, nc = oracle.ccl26(_keys_of(grid), _dims_of(grid))
    assert nc == 2


def test_empty():
    lab, nc = oracle.ccl26(np.zeros(0, np.uint32), (4, 4, 4))
    assert nc == 0 and len(lab) == 0

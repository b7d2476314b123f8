"""Pins of the oracle's steppable classification (Sec. III-C, Eq. (3)-(4))
and of its gated clustering (Alg. 1 with the distance and normal-angle
gates): the Jacobi eigen-decomposition against LAPACK (numpy.linalg.eigh),
normals of exact planes against their true normals, the 15-degree and
N_th boundaries, the gated components against a brute-force union-find
over the explicitly enumerated gated edges, the reduction to the plain
26-connected labelling when the gates are open, and a box standing on a
floor, which the ungated labelling merges and the gated one separates."""
import math

import numpy as np
import pytest

import oracle

DIMS = (40, 40, 40)


def _keys(xyz_idx, dims=DIMS):
    x, y, z = np.asarray(xyz_idx, np.int64).T
    return (x + dims[0] * (y + dims[1] * z)).astype(np.uint32)


def test_jacobi_against_lapack():
    rng = np.random.default_rng(0)
    for trial in range(400):
        B = rng.normal(size=(3, 3)) * (10.0 ** rng.uniform(-6, 2))
        if trial % 4 == 0:                       # nearly rank 2 (points on a plane)
            B[:, 2] *= 1e-4
        A = B @ B.T if trial % 2 else (B + B.T) / 2
        d, V = oracle.jacobi3(A)
        w, U = np.linalg.eigh(A)
        scale = max(np.abs(w).max(), 1e-300)
        assert np.allclose(np.sort(d), w, rtol=0, atol=1e-12 * scale)
        assert np.allclose(V.T @ V, np.eye(3), atol=1e-13)
        assert np.allclose(A @ V, V * d[None, :], rtol=0, atol=1e-11 * scale)
        # the eigenvector of the smallest eigenvalue, when it is well separated
        m = int(np.argmin(d))
        gap = (w[1] - w[0]) / scale
        if gap > 1e-6:
            assert abs(abs(float(V[:, m] @ U[:, 0])) - 1.0) < 1e-9 / gap
    # nothing to rotate: diagonal and zero matrices keep V = I
    for A in (np.diag([3.0, 1.0, 2.0]), np.zeros((3, 3))):
        d, V = oracle.jacobi3(A)
        assert np.array_equal(V, np.eye(3)) and np.array_equal(d, np.diag(A))


def _plane_voxels(normal, centre, half, spacing=0.002, dims=DIMS, s=0.01):
    """Noise-free points of a square patch (voxelised by the oracle map):
    (keys, means)."""
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    a = np.cross(n, [0.0, 1.0, 0.0] if abs(n[1]) < 0.9 else [1.0, 0.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    g = np.arange(-half, half + 1e-12, spacing)
    u, v = np.meshgrid(g, g, indexing="ij")
    p = np.asarray(centre)[None, :] + u.reshape(-1, 1) * a[None, :] + v.reshape(-1, 1) * b[None, :]
    om = oracle.OracleMap((0.0, 0.0, 0.0), s, dims)
    om.insert(p.astype(np.float32))
    return om.key, om.means()


@pytest.mark.parametrize("tilt_deg", [0.0, 5.0, 14.0, 16.0, 40.0, 90.0])
def test_plane_normals_and_the_angle_threshold(tilt_deg):
    t = math.radians(tilt_deg)
    true_n = np.array([math.sin(t), 0.0, math.cos(t)])
    keys, mu = _plane_voxels(true_n, (0.2, 0.2, 0.2), 0.08)
    nrm, st, nb = oracle.classify(keys, mu, DIMS)
    # interior voxels (full neighbourhoods): the normal of the plane
    inner = nb >= 8
    assert inner.sum() > 50
    ang = np.degrees(np.arccos(np.clip(np.abs(nrm[inner].astype(np.float64) @ true_n), -1, 1)))
    assert ang.max() < 0.05, ang.max()
    assert np.all(nrm[:, 2] >= 0)
    assert np.all(st[inner] == (tilt_deg <= 15.0))


def test_normals_against_numpy_scatter_and_eigh():
    rng = np.random.default_rng(4)
    idx = rng.integers(0, 12, size=(500, 3))
    keys = np.unique(_keys(idx))
    mu = (np.stack([keys % 40, (keys // 40) % 40, keys // 1600], 1) * 0.01 + rng.uniform(0, 0.01, (len(keys), 3)))
    mu = mu.astype(np.float32)
    nrm, st, nb = oracle.classify(keys, mu, DIMS, radius=1)
    pos = {int(k): i for i, k in enumerate(keys)}
    for i in rng.choice(len(keys), 120, replace=False):
        k = int(keys[i])
        x, y, z = k % 40, (k // 40) % 40, k // 1600
        nbrs = [pos[kk] for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if (kk := (x + dx) + 40 * ((y + dy) + 40 * (z + dz))) in pos
                and 0 <= x + dx < 40 and 0 <= y + dy < 40 and 0 <= z + dz < 40]
        assert nb[i] == len(nbrs)
        P = mu[nbrs].astype(np.float64)
        C = (P - P.mean(0)).T @ (P - P.mean(0))
        w, U = np.linalg.eigh(C)
        if len(nbrs) < 3 or (w[1] - w[0]) < 1e-6 * max(w[2], 1e-30):
            continue
        u = U[:, 0] * (1 if U[2, 0] >= 0 else -1)
        assert np.allclose(nrm[i], u, atol=1e-6), (i, nrm[i], u)


def test_neighbour_count_threshold():
    # a lone voxel, a pair and a flat 2x2 square: N = 1, 2, 4 at radius 1
    keys = np.sort(np.concatenate([_keys([[5, 5, 5]]), _keys([[20, 5, 5], [21, 5, 5]]),
                                   _keys([[30, 30, 5], [31, 30, 5], [30, 31, 5], [31, 31, 5]])]))
    cells = np.stack([keys % 40, (keys // 40) % 40, keys // 1600], 1)
    mu = ((cells + 0.5) * 0.01).astype(np.float32)
    nrm, st, nb = oracle.classify(keys, mu, DIMS)
    by = {int(k): (bool(s), int(n)) for k, s, n in zip(keys, st, nb)}
    assert by[int(_keys([[5, 5, 5]])[0])] == (False, 1)
    assert by[int(_keys([[20, 5, 5]])[0])] == (False, 2)
    for c in ([30, 30, 5], [31, 31, 5]):
        assert by[int(_keys([c])[0])] == (True, 4)
    # and with N_th = 5 the square is no longer steppable
    _, st5, _ = oracle.classify(keys, mu, DIMS, n_th=5)
    assert not st5.any()


def _brute_gated(keys, mu, nrm, st, dims, d_th, cos_th):
    """Union-find over the explicitly enumerated gated edges; labels = the
    smallest key of each component."""
    n = len(keys)
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    pos = {int(k): i for i, k in enumerate(keys)}
    nx, ny = dims[0], dims[1]
    for i in range(n):
        if not st[i]:
            continue
        k = int(keys[i])
        x, y, z = k % nx, (k // nx) % ny, k // (nx * ny)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dx, dy, dz) == (0, 0, 0):
                        continue
                    xx, yy, zz = x + dx, y + dy, z + dz
                    if not (0 <= xx < dims[0] and 0 <= yy < dims[1] and 0 <= zz < dims[2]):
                        continue
                    j = pos.get(xx + nx * (yy + ny * zz))
                    if j is None or not st[j]:
                        continue
                    d = mu[i].astype(np.float64) - mu[j].astype(np.float64)
                    if not (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < d_th * d_th):
                        continue
                    a, b = nrm[i].astype(np.float64), nrm[j].astype(np.float64)
                    if not (a[0] * b[0] + a[1] * b[1] + a[2] * b[2] > cos_th):
                        continue
                    ri, rj = find(i), find(j)
                    if ri != rj:
                        parent[max(ri, rj)] = min(ri, rj)
    lab = np.full(n, oracle.NO_KEY, np.uint32)
    for i in range(n):
        if st[i]:
            lab[i] = keys[find(i)]
    return lab


@pytest.mark.parametrize("seed", range(6))
def test_gated_ccl_against_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    dims = (9, 8, 7)
    cells = rng.integers(0, [9, 8, 7], size=(rng.integers(30, 250), 3))
    keys = np.unique(_keys(cells, dims))
    c = np.stack([keys % 9, (keys // 9) % 8, keys // 72], 1)
    mu = ((c + rng.uniform(0, 1, c.shape)) * 0.01).astype(np.float32)
    v = rng.normal(size=(len(keys), 3)) * [0.2, 0.2, 1.0]
    nrm = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    nrm[nrm[:, 2] < 0] *= -1
    st = rng.random(len(keys)) < 0.8
    for d_th, cos_th in ((0.05, oracle.COS_15), (0.012, oracle.COS_15), (0.05, 0.5), (1e9, -2.0)):
        lab, nc = oracle.ccl_gated(keys, mu, nrm, st, dims, d_th, cos_th)
        ref = _brute_gated(keys, mu, nrm, st, dims, d_th, cos_th)
        assert np.array_equal(lab, ref), (d_th, cos_th)
        assert nc == len(np.unique(ref[ref != oracle.NO_KEY]))


def test_open_gates_reduce_to_plain_labelling():
    rng = np.random.default_rng(7)
    dims = (20, 18, 16)
    keys = np.unique(_keys(rng.integers(0, [20, 18, 16], size=(1500, 3)), dims))
    mu = np.zeros((len(keys), 3), np.float32)
    nrm = np.tile(np.array([0, 0, 1], np.float32), (len(keys), 1))
    lab, _ = oracle.ccl_gated(keys, mu, nrm, np.ones(len(keys), bool), dims, 1.0, 0.5)
    ref, _ = oracle.ccl26(keys, dims)
    assert np.array_equal(lab, ref)


def _box_on_floor():
    """A 0.6 m floor patch and a 0.2 x 0.2 x 0.15 m box standing on it (top and
    four sides), noise-free, 1 cm voxels."""
    s = 0.01
    pts = []
    g = np.arange(0.0, 0.6, 0.002)
    u, v = np.meshgrid(g, g, indexing="ij")
    fl = np.c_[u.ravel() + 0.05, v.ravel() + 0.05, np.full(u.size, 0.105)]
    # (no floor under the box: a scan does not see it)
    under = (fl[:, 0] > 0.25) & (fl[:, 0] < 0.45) & (fl[:, 1] > 0.25) & (fl[:, 1] < 0.45)
    pts.append(fl[~under])
    g2 = np.arange(0.0, 0.2, 0.002)
    h = np.arange(0.0, 0.15, 0.002)
    u, v = np.meshgrid(g2, g2, indexing="ij")
    pts.append(np.c_[u.ravel() + 0.25, v.ravel() + 0.25, np.full(u.size, 0.255)])          # top
    a, b = np.meshgrid(g2, h, indexing="ij")
    for fixed, axis in ((0.25, 0), (0.45, 0), (0.25, 1), (0.45, 1)):
        side = np.zeros((a.size, 3))
        side[:, axis] = fixed
        side[:, 1 - axis] = a.ravel() + 0.25
        side[:, 2] = b.ravel() + 0.105
        pts.append(side)
    om = oracle.OracleMap((0.0, 0.0, 0.0), s, (80, 80, 40))
    om.insert(np.concatenate(pts).astype(np.float32))
    return om


def test_box_on_floor_separates_only_with_the_gates():
    om = _box_on_floor()
    plain = oracle.segment(om, 30, 64, 0.01, 1, 0)
    assert len(plain.clusters.tag) == 1                      # floor, sides and top touch
    fr = oracle.segment(om, 30, 64, 0.01, 1, 0, steppable={})
    sizes = np.diff(fr.clusters.off.astype(np.int64))
    assert len(fr.clusters.tag) == 2, sizes                  # the floor, then the top
    zs = [fr.clusters.xyz[fr.clusters.off[k]:fr.clusters.off[k + 1], 2].mean() for k in range(2)]
    assert abs(zs[0] - 0.105) < 0.006 and abs(zs[1] - 0.255) < 0.006
    for r in fr.results:                                     # each a horizontal plane
        assert r.ransac.best_h >= 0 and abs(r.ransac.plane[2]) > 0.999
    # the box sides are not steppable, the floor away from the box is
    st = fr.steppable.steppable
    z = om.means()[:, 2]
    assert not st[(z > 0.13) & (z < 0.23)].any()
    assert st[(z < 0.11)].mean() > 0.9

"""Pins for the oracle's boundary polygon (Sec. III-C, "Boundary polygon
generation"): the convex hull of a plane's inliers, in the plane.

Checked against an O(n^3) brute-force edge test in exact rational
arithmetic, scipy's Qhull, closed-form areas, and the invariants every convex
hull satisfies (strict convexity, containment, vertices drawn from the input,
independence from input order and from the in-plane basis)."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import ConvexHull

import oracle


def _embed(uv, normal=(0.0, 0.0, 1.0), d=0.0, jitter=0.0, rng=None):
    n = np.asarray(normal, np.float64)
    n /= np.linalg.norm(n)
    a = np.cross(n, [1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.cross(n, [0.0, 1.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    p = -d * n[None, :] + uv[:, :1] * a[None, :] + uv[:, 1:] * b[None, :]
    if jitter:
        p += rng.normal(0, jitter, size=(len(uv), 1)) * n[None, :]
    p = p.astype(np.float32)
    plane = np.r_[n, d].astype(np.float32)
    return p, plane


def _hull(p, plane):
    return oracle.hull(p[:, 0], p[:, 1], p[:, 2], plane)


def _brute_vertices(u, v):
    P = [(Fraction(float(a)), Fraction(float(b))) for a, b in zip(u, v)]
    n = len(P)
    verts = set()
    for i in range(n):
        for j in range(n):
            if i == j or P[i] == P[j]:
                continue
            ok = True
            for k in range(n):
                if k in (i, j):
                    continue
                cr = (P[j][0] - P[i][0]) * (P[k][1] - P[i][1]) - (P[j][1] - P[i][1]) * (P[k][0] - P[i][0])
                if cr < 0:
                    ok = False
                    break
                if cr == 0:
                    # collinear: must lie strictly between i and j
                    t = ((P[k][0] - P[i][0]) * (P[j][0] - P[i][0]) + (P[k][1] - P[i][1]) * (P[j][1] - P[i][1]))
                    L = (P[j][0] - P[i][0]) ** 2 + (P[j][1] - P[i][1]) ** 2
                    if not (0 < t < L):
                        ok = False
                        break
            if ok:
                verts.add(i)
                verts.add(j)
    return verts


@pytest.mark.parametrize("seed", range(12))
def test_against_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 40))
    uv = rng.uniform(-1, 1, size=(n, 2)) * rng.uniform(0.05, 2.0)
    p, plane = _embed(uv, rng.normal(size=3) * [1, 1, 3] + [0, 0, 2], rng.uniform(-1, 1))
    h = _hull(p, plane)
    u, v = oracle.hull_project(p[:, 0], p[:, 1], p[:, 2], plane)
    assert set(h.idx.tolist()) == _brute_vertices(u, v)


@pytest.mark.parametrize("seed", range(6))
def test_area_against_qhull(seed):
    rng = np.random.default_rng(100 + seed)
    uv = rng.normal(size=(5000, 2)) * [0.8, 0.3]
    p, plane = _embed(uv, rng.normal(size=3) + [0, 0, 3], 0.2, jitter=0.003, rng=rng)
    h = _hull(p, plane)
    u, v = oracle.hull_project(p[:, 0], p[:, 1], p[:, 2], plane)
    qh = ConvexHull(np.c_[u, v])
    assert abs(h.area - qh.volume) <= 1e-12 * qh.volume
    assert set(h.idx.tolist()) == set(qh.vertices.tolist())


def test_unit_square_with_interior_point():
    uv = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], np.float64)
    p, plane = _embed(uv)
    h = _hull(p, plane)
    assert len(h.idx) == 4 and 4 not in h.idx.tolist()
    assert h.area == pytest.approx(1.0, rel=1e-7)


def test_rectangle_tread_area():
    # a 0.30 m x 0.60 m stair tread: corners plus interior points
    rng = np.random.default_rng(0)
    corners = np.array([[0, 0], [0.3, 0], [0.3, 0.6], [0, 0.6]])
    inner = rng.uniform([0.001, 0.001], [0.299, 0.599], size=(3000, 2))
    uv = np.concatenate([inner, corners])
    p, plane = _embed(uv, (0, 0, 1), -0.18)
    h = _hull(p, plane)
    assert sorted(h.idx.tolist()) == [3000, 3001, 3002, 3003]
    assert h.area == pytest.approx(0.18, rel=1e-6)


@pytest.mark.parametrize("k", [3, 5, 8, 31, 100])
def test_regular_polygon(k):
    r = 0.7
    th = 2 * math.pi * np.arange(k) / k + 0.1
    uv = np.c_[r * np.cos(th), r * np.sin(th)]
    uv = np.concatenate([uv, 0.3 * uv[::2]])
    p, plane = _embed(uv, (0.2, -0.1, 1.0), 0.4)
    h = _hull(p, plane)
    assert len(h.idx) == k
    assert h.area == pytest.approx(0.5 * k * r * r * math.sin(2 * math.pi / k), rel=1e-5)


def test_invariants_convex_containment_order():
    rng = np.random.default_rng(9)
    uv = rng.uniform(-1, 1, size=(4000, 2)) * [1.5, 0.4]
    p, plane = _embed(uv, (0.1, 0.3, 1.0), -0.5, jitter=0.002, rng=rng)
    h = _hull(p, plane)
    u, v = oracle.hull_project(p[:, 0], p[:, 1], p[:, 2], plane)
    H = np.c_[u[h.idx], v[h.idx]]
    m = len(H)
    # counter-clockwise, strictly convex, starting at the lexicographic minimum
    for i in range(m):
        a, b, c = H[i], H[(i + 1) % m], H[(i + 2) % m]
        assert (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]) > 0
    assert tuple(H[0]) == min(map(tuple, np.c_[u, v]))
    # every point inside (left of every edge, up to 1e-9 m)
    for i in range(m):
        a, b = H[i], H[(i + 1) % m]
        L = math.hypot(*(b - a))
        cr = (b[0] - a[0]) * (v - a[1]) - (b[1] - a[1]) * (u - a[0])
        assert np.all(cr / L >= -1e-9)
    # vertices lie on the plane
    dist = h.xyz.astype(np.float64) @ plane[:3].astype(np.float64) + plane[3]
    assert np.max(np.abs(dist)) < 1e-6
    # order independence (same vertex set and area)
    perm = rng.permutation(len(p))
    h2 = _hull(p[perm], plane)
    assert set(perm[h2.idx].tolist()) == set(h.idx.tolist())
    assert h2.area == pytest.approx(h.area, rel=1e-12)


def test_area_independent_of_in_plane_rotation():
    rng = np.random.default_rng(10)
    uv = rng.uniform(-1, 1, size=(2000, 2)) * [0.9, 0.2]
    areas = []
    for ang in (0.0, 0.3, 1.1, 2.5):
        c, s = math.cos(ang), math.sin(ang)
        p, plane = _embed(uv @ np.array([[c, -s], [s, c]]).T, (0.0, 0.0, 1.0), 0.0)
        areas.append(_hull(p, plane).area)
    assert max(areas) - min(areas) <= 1e-6 * max(areas)


def test_degenerate_hulls():
    t = np.linspace(0, 1, 20)
    p, plane = _embed(np.c_[t, 0.5 * t])
    h = _hull(p, plane)
    assert len(h.idx) == 2 and h.area == 0.0
    assert set(h.idx.tolist()) == {0, 19}
    one, plane1 = _embed(np.array([[0.2, 0.3]]))
    h1 = _hull(one, plane1)
    assert list(h1.idx) == [0] and h1.area == 0.0
    dup, plane2 = _embed(np.array([[0.2, 0.3]] * 5))
    assert _hull(dup, plane2).area == 0.0

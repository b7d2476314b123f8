"""CPU oracle for the voxel-map plane-segmentation path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the library.  It shares no code
with the HIP path; both only take their inputs from ``scenes``.

The arithmetic lives in ``vm_oracle.c`` (plain C, fp64 where the method is
floating point).  This wrapper adds the steps whose definition is a library
primitive: grouping voxels by label is a stable sort (Sec. III-C,
"Clustering of steppable points", last sentence).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
NO_KEY = 0xFFFFFFFF
# Eq. (4) and Alg. 1 thresholds of the paper: N_th = 3 neighbour points,
# theta_th = 15 degrees (cos 15 deg = (sqrt 6 + sqrt 2) / 4, rounded to fp64),
# d_th = 0.05 m
N_TH = 3
COS_15 = float.fromhex("0x1.ee8dd4748bf15p-1")
D_TH = 0.05


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, u32, u64, f32, f64 = ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float, ctypes.c_double
        L.vo_philox4x64_10.argtypes = [P, P, P]
        L.vo_philox4x64_10.restype = None
        L.vo_draw3.argtypes = [u64, u64, u64, u64, u64, P]
        L.vo_draw3.restype = None
        L.vo_voxelize.argtypes = [P, i64, P, P, P, f64, P, P, P]
        L.vo_voxelize.restype = i64
        L.vo_map_accumulate.argtypes = [P, P, P, i64, P, P, i64, P, P, P, i64]
        L.vo_map_accumulate.restype = i64
        L.vo_voxel_mean.argtypes = [P, P, P, i64, P, f64, P, P]
        L.vo_voxel_mean.restype = None
        L.vo_ccl26.argtypes = [P, i64, P, P]
        L.vo_ccl26.restype = i64
        L.vo_ransac.argtypes = [P, P, P, i64, u32, f32, u64, u64, u64, P, P, P, P, P]
        L.vo_ransac.restype = ctypes.c_int32
        L.vo_hull.argtypes = [P, P, P, i64, P, P, P, P]
        L.vo_hull.restype = i64
        L.vo_hull_project.argtypes = [P, P, P, i64, P, P, P]
        L.vo_hull_project.restype = None
        L.vo_ray_voxels.argtypes = [P, P, P, P, i64]
        L.vo_ray_voxels.restype = i64
        L.vo_clear_rays.argtypes = [P, P, P, i64, P, i64, P, P, P, f64, P]
        L.vo_clear_rays.restype = i64
        L.vo_jacobi3.argtypes = [P, P]
        L.vo_jacobi3.restype = None
        L.vo_classify.argtypes = [P, P, i64, P, ctypes.c_int32, u32, f64, P, P, P]
        L.vo_classify.restype = None
        L.vo_ccl_gated.argtypes = [P, P, P, P, i64, P, f64, f64, P]
        L.vo_ccl_gated.restype = i64
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=dtype))


# --------------------------------------------------------------------------
# primitives
# --------------------------------------------------------------------------
def philox4x64_10(ctr, key) -> np.ndarray:
    c, k, out = _c(ctr, np.uint64), _c(key, np.uint64), np.zeros(4, np.uint64)
    lib().vo_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def draw3(seed: int, tag: int, frame: int, h: int, n: int) -> Tuple[int, int, int]:
    out = np.zeros(3, np.uint64)
    lib().vo_draw3(seed & (2**64 - 1), tag & (2**64 - 1), frame & (2**64 - 1), h, n, _p(out))
    return int(out[0]), int(out[1]), int(out[2])


def voxelize(xyz: np.ndarray, R, t, origin, voxel_size: float, dims) -> Tuple[np.ndarray, np.ndarray, int]:
    xyz = _c(xyz, np.float32).reshape(-1, 3)
    n = len(xyz)
    key = np.empty(n, np.uint32)
    frac = np.empty((n, 3), np.uint64)
    kept = lib().vo_voxelize(_p(xyz), n, _p(_c(R, np.float64)), _p(_c(t, np.float64)),
                             _p(_c(origin, np.float64)), float(voxel_size), _p(_c(dims, np.int32)),
                             _p(key), _p(frac))
    return key, frac, int(kept)


def voxel_mean(key, cnt, sums, origin, voxel_size, dims) -> np.ndarray:
    key, cnt, sums = _c(key, np.uint32), _c(cnt, np.uint32), _c(sums, np.uint64).reshape(-1, 3)
    mu = np.empty((len(key), 3), np.float32)
    lib().vo_voxel_mean(_p(key), _p(cnt), _p(sums), len(key), _p(_c(origin, np.float64)),
                        float(voxel_size), _p(_c(dims, np.int32)), _p(mu))
    return mu


def ccl26(keys: np.ndarray, dims) -> Tuple[np.ndarray, int]:
    keys = _c(keys, np.uint32)
    if len(keys) > 1 and not np.all(keys[1:] > keys[:-1]):
        raise ValueError("keys must be strictly ascending")
    lab = np.empty(len(keys), np.uint32)
    nc = lib().vo_ccl26(_p(keys), len(keys), _p(_c(dims, np.int32)), _p(lab))
    if nc < 0:
        raise MemoryError("oracle CCL allocation failed")
    return lab, int(nc)


@dataclasses.dataclass
class RansacResult:
    best_h: int
    plane: np.ndarray          # float32[4]
    counts: np.ndarray         # int32[H]
    hyp: np.ndarray            # float32[H, 4]
    inliers: np.ndarray        # uint32[m], cluster-local ascending


def ransac(x, y, z, n_hyp: int, eps: float, seed: int, tag: int, frame: int) -> RansacResult:
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    n = len(x)
    counts = np.empty(n_hyp, np.int32)
    hyp = np.empty((n_hyp, 4), np.float32)
    best = np.empty(4, np.float32)
    inl = np.empty(max(n, 1), np.uint32)
    nin = np.zeros(1, np.int64)
    h = lib().vo_ransac(_p(x), _p(y), _p(z), n, n_hyp, ctypes.c_float(eps), seed & (2**64 - 1),
                        tag & (2**64 - 1), frame & (2**64 - 1), _p(counts), _p(hyp), _p(best),
                        _p(inl), _p(nin))
    return RansacResult(int(h), best, counts, hyp, inl[: int(nin[0])].copy())


@dataclasses.dataclass
class HullResult:
    idx: np.ndarray            # uint32[h], indices into the hull's input points
    xyz: np.ndarray            # float32[h, 3]
    area: float


def hull(x, y, z, plane) -> HullResult:
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    m = len(x)
    idx = np.empty(max(m, 1), np.uint32)
    xyz = np.empty((max(m, 1), 3), np.float32)
    area = np.zeros(1, np.float64)
    h = lib().vo_hull(_p(x), _p(y), _p(z), m, _p(_c(plane, np.float32)), _p(idx), _p(xyz), _p(area))
    if h < 0:
        raise MemoryError("oracle hull allocation failed")
    return HullResult(idx[:h].copy(), xyz[:h].copy(), float(area[0]))


def hull_project(x, y, z, plane) -> Tuple[np.ndarray, np.ndarray]:
    x, y, z = _c(x, np.float32), _c(y, np.float32), _c(z, np.float32)
    u = np.empty(len(x), np.float64)
    v = np.empty(len(x), np.float64)
    lib().vo_hull_project(_p(x), _p(y), _p(z), len(x), _p(_c(plane, np.float32)), _p(u), _p(v))
    return u, v


def ray_voxels(a, b, dims) -> np.ndarray:
    """Voxel coordinates [m, 3] of the ray from voxel a to voxel b (Bresenham,
    a included, b excluded, cut at the grid's faces)."""
    a, b = _c(a, np.int64), _c(b, np.int64)
    cap = int(np.abs(b - a).max()) + 1
    out = np.empty((cap, 3), np.int64)
    m = lib().vo_ray_voxels(_p(a), _p(b), _p(_c(dims, np.int32)), _p(out), cap)
    return out[:m].copy()


def jacobi3(A) -> Tuple[np.ndarray, np.ndarray]:
    """(diagonal after the cyclic Jacobi sweeps, eigenvectors as columns)."""
    a = np.array(A, dtype=np.float64).reshape(3, 3).copy(order="C")
    v = np.empty((3, 3), np.float64)
    lib().vo_jacobi3(_p(a), _p(v))
    return np.diag(a).copy(), v


def classify(keys, mu, dims, radius: int = 1, n_th: int = N_TH, cos_th: float = COS_15):
    """Eq. (3)-(4) for every occupied voxel: (normal float32[n,3], steppable
    bool[n], neighbour count uint32[n])."""
    keys, mu = _c(keys, np.uint32), _c(mu, np.float32).reshape(-1, 3)
    n = len(keys)
    nrm = np.empty((n, 3), np.float32)
    st = np.empty(n, np.uint8)
    nb = np.empty(n, np.uint32)
    lib().vo_classify(_p(keys), _p(mu), n, _p(_c(dims, np.int32)), int(radius), int(n_th), float(cos_th), _p(nrm),
                      _p(st), _p(nb))
    return nrm, st.astype(bool), nb


def ccl_gated(keys, mu, normal, steppable, dims, d_th: float = D_TH, cos_th: float = COS_15):
    """Alg. 1 with its gates: (labels uint32[n], NO_KEY for voxels that are not
    steppable; number of components)."""
    keys, mu = _c(keys, np.uint32), _c(mu, np.float32).reshape(-1, 3)
    normal = _c(normal, np.float32).reshape(-1, 3)
    st = _c(np.asarray(steppable).astype(np.uint8), np.uint8)
    lab = np.empty(len(keys), np.uint32)
    nc = lib().vo_ccl_gated(_p(keys), _p(mu), _p(normal), _p(st), len(keys), _p(_c(dims, np.int32)), float(d_th),
                            float(cos_th), _p(lab))
    if nc < 0:
        raise MemoryError("oracle gated CCL allocation failed")
    return lab, int(nc)


# --------------------------------------------------------------------------
# the map and the per-frame path
# --------------------------------------------------------------------------
class OracleMap:
    """Sparse voxel map as arrays sorted by key (Sec. III-B): per occupied
    voxel its point count and the integer sums of its fixed-point offsets."""

    def __init__(self, origin, voxel_size: float, dims):
        self.origin = np.asarray(origin, np.float64)
        self.voxel_size = float(voxel_size)
        self.dims = np.asarray(dims, np.int32)
        self.key = np.zeros(0, np.uint32)
        self.cnt = np.zeros(0, np.uint32)
        self.sums = np.zeros((0, 3), np.uint64)
        self.points_in = 0
        self.points_dropped = 0

    def insert(self, xyz: np.ndarray, R=None, t=None) -> None:
        R = np.eye(3) if R is None else R
        t = np.zeros(3) if t is None else t
        pk, pf, kept = voxelize(xyz, R, t, self.origin, self.voxel_size, self.dims)
        cap = len(self.key) + kept
        ok = np.empty(max(cap, 1), np.uint32)
        oc = np.empty(max(cap, 1), np.uint32)
        osum = np.empty((max(cap, 1), 3), np.uint64)
        n = lib().vo_map_accumulate(_p(self.key), _p(self.cnt), _p(self.sums), len(self.key),
                                    _p(pk), _p(pf), len(pk), _p(ok), _p(oc), _p(osum), cap)
        if n < 0:
            raise MemoryError("oracle map accumulate failed")
        self.key, self.cnt, self.sums = ok[:n].copy(), oc[:n].copy(), osum[:n].copy()
        self.points_in += kept
        self.points_dropped += len(pk) - kept

    def means(self) -> np.ndarray:
        return voxel_mean(self.key, self.cnt, self.sums, self.origin, self.voxel_size, self.dims)

    def shift(self, dx: int, dy: int, dz: int) -> int:
        """Sec. III-B's robot-centric map: the grid moves by (dx, dy, dz) whole
        voxels.  The origin becomes origin + s * shift (fp64); voxel (x, y, z)
        becomes (x - dx, y - dy, z - dz) with its count and sums unchanged;
        voxels leaving the grid are dropped.  Returns how many were dropped."""
        d = np.array([dx, dy, dz], np.int64)
        NX, NY, NZ = (int(v) for v in self.dims)
        k = self.key.astype(np.int64)
        x, y, z = k % NX - d[0], (k // NX) % NY - d[1], k // (NX * NY) - d[2]
        keep = (x >= 0) & (y >= 0) & (z >= 0) & (x < NX) & (y < NY) & (z < NZ)
        nk = (x + NX * (y + NY * z))[keep]
        order = np.argsort(nk, kind="stable")    # the order is kept anyway: a constant offset
        self.key = nk[order].astype(np.uint32)
        self.cnt = self.cnt[keep][order].copy()
        self.sums = self.sums[keep][order].copy()
        self.origin = np.array([self.origin[i] + float(d[i]) * self.voxel_size for i in range(3)], np.float64)
        return int((~keep).sum())

    def clear_rays(self, xyz: np.ndarray, R=None, t=None) -> int:
        """Eq. (2) for one frame: remove the occupied voxels the frame's rays
        pass through (the sensor at the pose's translation), except those
        holding one of its points.  Returns the number removed."""
        R = np.eye(3) if R is None else R
        t = np.zeros(3) if t is None else t
        xyz = _c(xyz, np.float32).reshape(-1, 3)
        n0 = len(self.key)
        key, cnt, sums = self.key.copy(), self.cnt.copy(), self.sums.copy()
        n = lib().vo_clear_rays(_p(key), _p(cnt), _p(sums), n0, _p(xyz), len(xyz), _p(_c(R, np.float64)),
                                _p(_c(t, np.float64)), _p(self.origin), self.voxel_size, _p(self.dims))
        if n < 0:
            raise ValueError("sensor outside the grid (or no memory)")
        self.key, self.cnt, self.sums = key[:n].copy(), cnt[:n].copy(), sums[:n].copy()
        return n0 - int(n)


@dataclasses.dataclass
class Clusters:
    off: np.ndarray            # uint32[K+1]
    key: np.ndarray            # uint32[sum]: voxel keys, ascending inside a cluster
    xyz: np.ndarray            # float32[sum, 3]: voxel means
    tag: np.ndarray            # uint32[K]: cluster label = smallest key


def group(keys: np.ndarray, labels: np.ndarray, mu: np.ndarray, min_cluster: int) -> Clusters:
    """Voxels sharing a label form a cluster (Sec. III-C, clustering); clusters
    below ``min_cluster`` voxels are dropped; clusters are ordered by label and
    the voxels of a cluster by key (both inputs are in ascending key order).
    Voxels labelled NO_KEY (not steppable) belong to no cluster."""
    sel0 = np.nonzero(labels != NO_KEY)[0]
    if len(sel0) != len(labels):
        keys, labels, mu = keys[sel0], labels[sel0], mu[sel0]
    uniq, inv, counts = np.unique(labels, return_inverse=True, return_counts=True)
    keep = counts[inv] >= min_cluster
    sel = np.nonzero(keep)[0]
    order = sel[np.argsort(labels[sel], kind="stable")]
    kept_labels = uniq[counts >= min_cluster]
    sizes = counts[counts >= min_cluster]
    off = np.zeros(len(kept_labels) + 1, np.uint32)
    off[1:] = np.cumsum(sizes)
    return Clusters(off, keys[order].astype(np.uint32), mu[order].astype(np.float32),
                    kept_labels.astype(np.uint32))


@dataclasses.dataclass
class ClusterResult:
    tag: int
    ransac: RansacResult
    hull: Optional[HullResult]          # hull vertices indexed cluster-locally
    hull_local: Optional[np.ndarray]    # uint32 cluster-local point indices of the vertices


def plane_and_hull(x, y, z, n_hyp: int, eps: float, seed: int, tag: int, frame: int) -> ClusterResult:
    r = ransac(x, y, z, n_hyp, eps, seed, tag, frame)
    if r.best_h < 0:
        return ClusterResult(tag, r, None, None)
    inl = r.inliers
    hres = hull(np.asarray(x)[inl], np.asarray(y)[inl], np.asarray(z)[inl], r.plane)
    return ClusterResult(tag, r, hres, inl[hres.idx].astype(np.uint32))


@dataclasses.dataclass
class FrameResult:
    labels: np.ndarray
    clusters: Clusters
    results: List[ClusterResult]


def planes_and_hulls(off, xyz, tag, n_hyp: int, eps: float, seed: int, frame, ks=None,
                     threads: int = 1) -> List[ClusterResult]:
    """:func:`plane_and_hull` for the clusters ``ks`` (default: all) of a CSR
    (off[K+1], xyz[N,3], tag[K]); ``frame`` is one number or one per cluster.
    With threads > 1 the clusters are spread over a thread pool (the C calls
    release the interpreter lock); every cluster is computed by the same
    single-threaded code, so the results do not depend on ``threads``."""
    ks = range(len(tag)) if ks is None else list(ks)
    fr = np.broadcast_to(np.asarray(frame, dtype=np.uint64), (len(tag),))

    def one(k):
        a, b = int(off[k]), int(off[k + 1])
        p = xyz[a:b]
        return plane_and_hull(p[:, 0], p[:, 1], p[:, 2], n_hyp, eps, seed, int(tag[k]), int(fr[k]))

    if threads <= 1:
        return [one(k) for k in ks]
    import concurrent.futures
    # largest clusters first, so a big one does not start last
    order = sorted(ks, key=lambda k: -(int(off[k + 1]) - int(off[k])))
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        done = dict(zip(order, ex.map(one, order)))
    return [done[k] for k in ks]


@dataclasses.dataclass
class Steppable:
    normal: np.ndarray       # float32[n, 3] per occupied voxel
    steppable: np.ndarray    # bool[n]
    n_nb: np.ndarray         # uint32[n] neighbour points


def segment(m: OracleMap, min_cluster: int, n_hyp: int, eps: float, seed: int, frame: int,
            cluster_subset: Optional[List[int]] = None, threads: int = 1,
            steppable: Optional[dict] = None) -> FrameResult:
    """Sec. III-C on the whole accumulated map: label, group, then one plane
    and one hull per kept cluster (optionally only for ``cluster_subset``).
    With ``steppable`` (dict of radius, n_th, cos_th, d_th) the voxels are
    classified first (Eq. (3)-(4)) and only steppable voxels are clustered,
    with Alg. 1's distance and normal-angle gates; the classification is
    returned in the result's ``steppable`` field."""
    if steppable is not None:
        mu = m.means()
        nrm, st, nb = classify(m.key, mu, m.dims, steppable.get("radius", 1), steppable.get("n_th", N_TH),
                               steppable.get("cos_th", COS_15))
        labels, _ = ccl_gated(m.key, mu, nrm, st, m.dims, steppable.get("d_th", D_TH), steppable.get("cos_th", COS_15))
        cl = group(m.key, labels, mu, min_cluster)
        res = planes_and_hulls(cl.off, cl.xyz, cl.tag, n_hyp, eps, seed, frame, cluster_subset, threads)
        fr = FrameResult(labels, cl, res)
        fr.steppable = Steppable(nrm, st, nb)
        return fr
    labels, _ = ccl26(m.key, m.dims)
    cl = group(m.key, labels, m.means(), min_cluster)
    res = planes_and_hulls(cl.off, cl.xyz, cl.tag, n_hyp, eps, seed, frame, cluster_subset, threads)
    return FrameResult(labels, cl, res)

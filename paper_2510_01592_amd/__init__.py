"""Python binding of ``libvm.so`` (include/vm.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; this module only
turns torch tensors into device pointers and the current HIP stream, and
mirrors the C structs with ctypes.  Importing it loads the library and fails
loudly if it has not been built (``python paper_2510_01592_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvm.so")

VM_OK, VM_E_ARG, VM_E_OOM, VM_E_CAPACITY, VM_E_DEVICE, VM_E_STATE = 0, -1, -2, -3, -4, -5
FLAG_HASH_FULL, FLAG_CLUSTERS_CAP, FLAG_INLIERS_CAP, FLAG_HULL_CAP = 0x1, 0x2, 0x4, 0x8
STAGES = ["insert", "rank", "ccl", "ccl_link", "group", "hypotheses", "count", "select", "hull", "clear"]

EXPORTED = [
    "vm_status_string", "vm_version", "vm_map_create", "vm_map_destroy", "vm_map_clear", "vm_map_stats",
    "vm_map_stats_async",
    "vm_insert", "vm_map_export", "vm_map_import", "vm_ccl", "vm_workspace_bytes", "vm_ransac_planes",
    "vm_ransac_planes_noalloc", "vm_planes_hulls", "vm_set_fused_config", "vm_get_fused_config",
    "vm_autotune_fused", "vm_planes_hulls_multi", "vm_multi_workspace_bytes", "vm_ccl_steppable",
    "vm_segment_frame_steppable", "vm_clear_rays", "vm_ccl_propagate", "vm_map_shift", "vm_map_recenter",
    "vm_map_origin",
    "vm_hulls", "vm_segment_frame", "vm_set_stage_timing", "vm_stage_times",
    "vm_set_count_config", "vm_get_count_config", "vm_autotune_count",
    "vm_capture_begin", "vm_capture_end", "vm_graph_launch", "vm_graph_destroy",
]

_P = ctypes.c_void_p


class MapDesc(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("voxel_size", ctypes.c_double),
                ("dims", ctypes.c_int32 * 3), ("hash_capacity_log2", ctypes.c_uint32),
                ("insert_batch_log2", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class Pose(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3)]


class MapStats(ctypes.Structure):
    _fields_ = [("occupied", ctypes.c_uint64), ("points_in", ctypes.c_uint64),
                ("points_dropped", ctypes.c_uint64), ("points_lost", ctypes.c_uint64),
                ("status_flags", ctypes.c_uint32), ("hash_capacity_log2", ctypes.c_uint32),
                ("last_touched", ctypes.c_uint64), ("voxels_cleared", ctypes.c_uint64),
                ("voxels_shifted_out", ctypes.c_uint64)]


# vm_map_stats_t in 64-bit words (the size of a device buffer for Map.stats_async)
STATS_WORDS = ctypes.sizeof(MapStats) // 8


class Clusters(ctypes.Structure):
    _fields_ = [("k_cap", ctypes.c_uint32), ("n_cap", ctypes.c_uint32), ("d_meta", _P), ("d_off", _P),
                ("d_x", _P), ("d_y", _P), ("d_z", _P), ("d_key", _P), ("d_tag", _P)]


class RansacParams(ctypes.Structure):
    _fields_ = [("n_hyp", ctypes.c_uint32), ("eps", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("frame", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("d_frame", _P)]


class Planes(ctypes.Structure):
    _fields_ = [("k_cap", ctypes.c_uint32), ("in_cap", ctypes.c_uint32), ("d_plane", _P), ("d_best_h", _P),
                ("d_n_inliers", _P), ("d_in_off", _P), ("d_in_idx", _P), ("d_counts", _P), ("d_hyp", _P),
                ("d_status", _P)]


class HullsOut(ctypes.Structure):
    _fields_ = [("k_cap", ctypes.c_uint32), ("v_cap", ctypes.c_uint32), ("d_v_off", _P), ("d_v_idx", _P),
                ("d_v_xyz", _P), ("d_area", _P), ("d_status", _P)]


class SegParams(ctypes.Structure):
    _fields_ = [("min_cluster", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("ransac", RansacParams)]


SEG_CLEAR_RAYS = 0x1


class CountConfig(ctypes.Structure):
    _fields_ = [("count_grid", ctypes.c_uint32), ("chunk_mult", ctypes.c_uint32),
                ("wave_max_points", ctypes.c_uint32), ("plane_max_points", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class StepParams(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_uint32), ("n_th", ctypes.c_uint32), ("cos_th", ctypes.c_double),
                ("d_th", ctypes.c_double)]


# the paper's thresholds: N_th = 3, theta_th = 15 deg (cos = (sqrt 6 + sqrt 2) / 4 in fp64), d_th = 0.05 m
COS_15 = float.fromhex("0x1.ee8dd4748bf15p-1")


def step_params(radius: int = 1, n_th: int = 3, cos_th: float = COS_15, d_th: float = 0.05) -> StepParams:
    return StepParams(int(radius), int(n_th), float(cos_th), float(d_th))


class FusedConfig(ctypes.Structure):
    _fields_ = [("hyp_chunk", ctypes.c_uint32), ("small_max", ctypes.c_uint32), ("groups_per_cu", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_ if f != "reserved"}


class VMError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libvm.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch already
        # loaded (same SONAME), so both share one runtime and one device context
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python paper_2510_01592_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        i32, u32, u64, i64, sz = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_size_t
        sig = {
            "vm_status_string": ([i32], ctypes.c_char_p),
            "vm_version": ([], i32),
            "vm_map_create": ([ctypes.POINTER(MapDesc), ctypes.POINTER(_P)], i32),
            "vm_map_destroy": ([_P], i32),
            "vm_map_clear": ([_P, _P], i32),
            "vm_map_stats": ([_P, _P, ctypes.POINTER(MapStats)], i32),
            "vm_map_stats_async": ([_P, _P, _P], i32),
            "vm_insert": ([_P, _P, i64, ctypes.POINTER(Pose), _P], i32),
            "vm_clear_rays": ([_P, _P, i64, ctypes.POINTER(Pose), _P], i32),
            "vm_map_shift": ([_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P], i32),
            "vm_map_recenter": ([_P, _P, _P, _P], i32),
            "vm_map_origin": ([_P, _P], i32),
            "vm_ccl_propagate": ([_P, u32, _P, ctypes.POINTER(Clusters), ctypes.POINTER(u32), _P], i32),
            "vm_map_export": ([_P, _P, _P, _P, _P, u64, ctypes.POINTER(u64), _P], i32),
            "vm_map_import": ([_P, _P, _P, _P, u64, _P], i32),
            "vm_ccl": ([_P, u32, _P, ctypes.POINTER(Clusters), _P], i32),
            "vm_workspace_bytes": ([u32, u32, u32], sz),
            "vm_ransac_planes": ([ctypes.POINTER(Clusters), ctypes.POINTER(RansacParams), ctypes.POINTER(Planes),
                                  _P, sz, _P], i32),
            "vm_ransac_planes_noalloc": ([ctypes.POINTER(Clusters), ctypes.POINTER(RansacParams),
                                          ctypes.POINTER(Planes), _P], i32),
            "vm_planes_hulls": ([ctypes.POINTER(Clusters), ctypes.POINTER(RansacParams), ctypes.POINTER(Planes),
                                 ctypes.POINTER(HullsOut), _P, sz, _P], i32),
            "vm_planes_hulls_multi": ([u32, ctypes.POINTER(Clusters), ctypes.POINTER(u32), ctypes.POINTER(RansacParams),
                                       ctypes.POINTER(Planes), ctypes.POINTER(HullsOut), u32, u32, _P, sz, _P], i32),
            "vm_multi_workspace_bytes": ([u32, u32, u32], sz),
            "vm_set_fused_config": ([ctypes.POINTER(FusedConfig)], i32),
            "vm_get_fused_config": ([ctypes.POINTER(FusedConfig)], i32),
            "vm_autotune_fused": ([ctypes.POINTER(Clusters), ctypes.POINTER(RansacParams), ctypes.POINTER(Planes),
                                   ctypes.POINTER(HullsOut), _P, sz, _P, u32, ctypes.POINTER(FusedConfig)], i32),
            "vm_hulls": ([ctypes.POINTER(Clusters), ctypes.POINTER(Planes), ctypes.POINTER(HullsOut), _P, sz, _P],
                         i32),
            "vm_segment_frame": ([_P, _P, i64, ctypes.POINTER(Pose), ctypes.POINTER(SegParams),
                                  ctypes.POINTER(Planes), ctypes.POINTER(HullsOut), _P, ctypes.POINTER(Clusters), _P],
                                 i32),
            "vm_ccl_steppable": ([_P, ctypes.POINTER(StepParams), u32, _P, _P, _P, ctypes.POINTER(Clusters), _P], i32),
            "vm_segment_frame_steppable": ([_P, _P, i64, ctypes.POINTER(Pose), ctypes.POINTER(SegParams),
                                            ctypes.POINTER(StepParams), ctypes.POINTER(Planes), ctypes.POINTER(HullsOut),
                                            _P, ctypes.POINTER(Clusters), _P], i32),
            "vm_capture_begin": ([_P], i32),
            "vm_capture_end": ([_P, ctypes.POINTER(_P)], i32),
            "vm_graph_launch": ([_P, _P], i32),
            "vm_graph_destroy": ([_P], i32),
            "vm_set_count_config": ([ctypes.POINTER(CountConfig)], i32),
            "vm_get_count_config": ([ctypes.POINTER(CountConfig)], i32),
            "vm_autotune_count": ([ctypes.POINTER(Clusters), ctypes.POINTER(RansacParams), ctypes.POINTER(Planes),
                                   _P, sz, _P, u32, ctypes.POINTER(CountConfig)], i32),
            "vm_set_stage_timing": ([i32], i32),
            "vm_stage_times": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64), i32], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().vm_status_string(s).decode()


def _check(st: int, what: str) -> None:
    if st != VM_OK:
        raise VMError(st, what)


def _stream(stream=None) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def make_pose(R=None, t=None) -> Pose:
    p = Pose()
    R = np.eye(3) if R is None else np.asarray(R, np.float64).reshape(3, 3)
    t = np.zeros(3) if t is None else np.asarray(t, np.float64).reshape(3)
    for i in range(9):
        p.R[i] = float(R.reshape(-1)[i])
    for i in range(3):
        p.t[i] = float(t[i])
    return p


def version() -> int:
    return int(lib().vm_version())


# --------------------------------------------------------------------------
# outputs
# --------------------------------------------------------------------------
@dataclasses.dataclass
class PlaneBuffers:
    """Device buffers of vm_planes (allocated with torch)."""
    k_cap: int
    in_cap: int
    n_hyp: int
    plane: "torch.Tensor"
    best_h: "torch.Tensor"
    n_inliers: "torch.Tensor"
    in_off: "torch.Tensor"
    in_idx: "torch.Tensor"
    status: "torch.Tensor"
    counts: Optional["torch.Tensor"] = None
    hyp: Optional["torch.Tensor"] = None

    @staticmethod
    def alloc(k_cap: int, in_cap: int, n_hyp: int, with_all: bool = False, device="cuda") -> "PlaneBuffers":
        import torch
        z = dict(device=device)
        return PlaneBuffers(
            k_cap, in_cap, n_hyp,
            torch.zeros((k_cap, 4), dtype=torch.float32, **z),
            torch.zeros(k_cap, dtype=torch.int32, **z),
            torch.zeros(k_cap, dtype=torch.int32, **z),
            torch.zeros(k_cap + 1, dtype=torch.int32, **z),
            torch.zeros(max(in_cap, 1), dtype=torch.int32, **z),
            torch.zeros(1, dtype=torch.int32, **z),
            torch.zeros((k_cap, n_hyp), dtype=torch.int32, **z) if with_all else None,
            torch.zeros((k_cap, n_hyp, 4), dtype=torch.float32, **z) if with_all else None,
        )

    def c(self) -> Planes:
        return Planes(self.k_cap, self.in_cap, _ptr(self.plane), _ptr(self.best_h), _ptr(self.n_inliers),
                      _ptr(self.in_off), _ptr(self.in_idx), _ptr(self.counts), _ptr(self.hyp), _ptr(self.status))


@dataclasses.dataclass
class HullBuffers:
    k_cap: int
    v_cap: int
    v_off: "torch.Tensor"
    v_idx: "torch.Tensor"
    v_xyz: "torch.Tensor"
    area: "torch.Tensor"
    status: "torch.Tensor"

    @staticmethod
    def alloc(k_cap: int, v_cap: int, device="cuda") -> "HullBuffers":
        import torch
        z = dict(device=device)
        return HullBuffers(k_cap, v_cap, torch.zeros(k_cap + 1, dtype=torch.int32, **z),
                           torch.zeros(max(v_cap, 1), dtype=torch.int32, **z),
                           torch.zeros((max(v_cap, 1), 3), dtype=torch.float32, **z),
                           torch.zeros(k_cap, dtype=torch.float64, **z), torch.zeros(1, dtype=torch.int32, **z))

    def c(self) -> HullsOut:
        return HullsOut(self.k_cap, self.v_cap, _ptr(self.v_off), _ptr(self.v_idx), _ptr(self.v_xyz),
                        _ptr(self.area), _ptr(self.status))


def ransac_params(n_hyp: int, eps: float = 0.01, seed: int = 0x5EED, frame: int = 0, d_frame=None) -> RansacParams:
    """``d_frame``: optional int32 device tensor holding the frame number (read when the work runs)."""
    return RansacParams(int(n_hyp), float(eps), int(seed) & (2 ** 64 - 1), int(frame) & 0xFFFFFFFF, 0,
                        _ptr(d_frame))


# --------------------------------------------------------------------------
# the map
# --------------------------------------------------------------------------
class Map:
    """A device-resident sparse voxel map (vm_map)."""

    def __init__(self, origin: Sequence[float], voxel_size: float, dims: Sequence[int], hash_capacity_log2: int,
                 insert_batch_log2: int = 0):
        d = MapDesc()
        d.insert_batch_log2 = int(insert_batch_log2)
        for i in range(3):
            d.origin[i] = float(origin[i])
            d.dims[i] = int(dims[i])
        d.voxel_size = float(voxel_size)
        d.hash_capacity_log2 = int(hash_capacity_log2)
        h = _P()
        _check(lib().vm_map_create(ctypes.byref(d), ctypes.byref(h)), "vm_map_create")
        self._h = h
        self.voxel_size = float(voxel_size)
        self.dims = tuple(int(v) for v in dims)

    @property
    def handle(self) -> int:
        return self._h.value

    def close(self) -> None:
        if self._h is not None and self._h.value:
            lib().vm_map_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clear(self, stream=None) -> None:
        _check(lib().vm_map_clear(self._h, _stream(stream)), "vm_map_clear")

    def stats(self, stream=None) -> MapStats:
        s = MapStats()
        _check(lib().vm_map_stats(self._h, _stream(stream), ctypes.byref(s)), "vm_map_stats")
        return s

    def stats_async(self, out, stream=None) -> None:
        """Enqueue the counters into ``out`` (device int64 tensor of >= STATS_WORDS entries)."""
        if out.numel() * out.element_size() < ctypes.sizeof(MapStats):
            raise ValueError("stats buffer too small")
        _check(lib().vm_map_stats_async(self._h, _ptr(out), _stream(stream)), "vm_map_stats_async")

    def insert(self, xyz, R=None, t=None, stream=None) -> None:
        if xyz.dtype.__str__() != "torch.float32" or xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("float32 [N, 3] tensor expected")
        pose = make_pose(R, t)
        _check(lib().vm_insert(self._h, _ptr(xyz), int(xyz.shape[0]), ctypes.byref(pose), _stream(stream)),
               "vm_insert")

    def shift(self, dx: int, dy: int, dz: int, stream=None) -> None:
        """vm_map_shift: move the grid by whole voxels (the robot-centric map)."""
        _check(lib().vm_map_shift(self._h, int(dx), int(dy), int(dz), _stream(stream)), "vm_map_shift")

    def recenter(self, center, stream=None) -> Tuple[int, int, int]:
        """vm_map_recenter: shift so that ``center`` lies in the grid's middle voxel; returns the shift."""
        c = (ctypes.c_double * 3)(*[float(v) for v in center])
        d = (ctypes.c_int32 * 3)()
        _check(lib().vm_map_recenter(self._h, c, d, _stream(stream)), "vm_map_recenter")
        return int(d[0]), int(d[1]), int(d[2])

    @property
    def origin(self) -> Tuple[float, float, float]:
        o = (ctypes.c_double * 3)()
        _check(lib().vm_map_origin(self._h, o), "vm_map_origin")
        return float(o[0]), float(o[1]), float(o[2])

    def clear_rays(self, xyz, R=None, t=None, stream=None) -> None:
        """vm_clear_rays: free the occupied voxels the frame's rays pass through
        (the sensor at t), except those holding one of its points."""
        if xyz.dtype.__str__() != "torch.float32" or xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("float32 [N, 3] tensor expected")
        pose = make_pose(R, t)
        _check(lib().vm_clear_rays(self._h, _ptr(xyz), int(xyz.shape[0]), ctypes.byref(pose), _stream(stream)),
               "vm_clear_rays")

    def export(self, cap: Optional[int] = None, stream=None):
        """(key, count, sums, mean) of every occupied voxel, ascending keys (torch, device)."""
        import torch
        if cap is None:
            cap = int(self.stats(stream).occupied)
        cap = max(int(cap), 1)
        key = torch.empty(cap, dtype=torch.int32, device="cuda")
        cnt = torch.empty(cap, dtype=torch.int32, device="cuda")
        sums = torch.empty((cap, 3), dtype=torch.int64, device="cuda")
        mean = torch.empty((cap, 3), dtype=torch.float32, device="cuda")
        n = ctypes.c_uint64()
        st = lib().vm_map_export(self._h, _ptr(key), _ptr(cnt), _ptr(sums), _ptr(mean), cap, ctypes.byref(n),
                                 _stream(stream))
        _check(st, "vm_map_export")
        m = int(n.value)
        return key[:m], cnt[:m], sums[:m], mean[:m]

    def import_(self, key, cnt, sums, stream=None) -> None:
        _check(lib().vm_map_import(self._h, _ptr(key), _ptr(cnt), _ptr(sums), int(key.shape[0]), _stream(stream)),
               "vm_map_import")

    def ccl(self, min_cluster: int = 30, labels=None, stream=None) -> Clusters:
        cl = Clusters()
        _check(lib().vm_ccl(self._h, int(min_cluster), _ptr(labels), ctypes.byref(cl), _stream(stream)), "vm_ccl")
        return cl

    def ccl_propagate(self, min_cluster: int = 30, labels=None, stream=None):
        """vm_ccl_propagate (Alg. 1's label propagation, the union-find's baseline):
        (clusters, sweeps run).  Synchronises the stream."""
        cl = Clusters()
        n = ctypes.c_uint32()
        _check(lib().vm_ccl_propagate(self._h, int(min_cluster), _ptr(labels), ctypes.byref(cl), ctypes.byref(n),
                                      _stream(stream)), "vm_ccl_propagate")
        return cl, int(n.value)

    def ccl_steppable(self, min_cluster: int = 30, step: Optional[StepParams] = None, normals=None, steppable=None,
                      labels=None, stream=None) -> Clusters:
        """vm_ccl_steppable: classification, gated clustering, grouping.  normals (float32 [V, 3]),
        steppable (uint8 [V]) and labels (int32 [V]) are optional device outputs."""
        cl = Clusters()
        stp = step_params() if step is None else step
        _check(lib().vm_ccl_steppable(self._h, ctypes.byref(stp), int(min_cluster), _ptr(normals), _ptr(steppable),
                                      _ptr(labels), ctypes.byref(cl), _stream(stream)), "vm_ccl_steppable")
        return cl

    def segment_frame(self, xyz, planes: PlaneBuffers, hulls: HullBuffers, R=None, t=None, min_cluster: int = 30,
                      n_hyp: int = 256, eps: float = 0.01, seed: int = 0x5EED, frame: int = 0, labels=None,
                      stream=None, d_frame=None, step: Optional[StepParams] = None,
                      clear: bool = False) -> Clusters:
        """vm_segment_frame, or vm_segment_frame_steppable when ``step`` is given;
        ``clear`` casts the frame's rays first (VM_SEG_CLEAR_RAYS)."""
        pose = make_pose(R, t)
        sp = SegParams(int(min_cluster), SEG_CLEAR_RAYS if clear else 0,
                       ransac_params(n_hyp, eps, seed, frame, d_frame))
        cl = Clusters()
        pc, hc = planes.c(), hulls.c()
        n = 0 if xyz is None else int(xyz.shape[0])
        if step is None:
            st = lib().vm_segment_frame(self._h, _ptr(xyz) if n else None, n, ctypes.byref(pose), ctypes.byref(sp),
                                        ctypes.byref(pc), ctypes.byref(hc), _ptr(labels), ctypes.byref(cl),
                                        _stream(stream))
            _check(st, "vm_segment_frame")
        else:
            st = lib().vm_segment_frame_steppable(self._h, _ptr(xyz) if n else None, n, ctypes.byref(pose),
                                                  ctypes.byref(sp), ctypes.byref(step), ctypes.byref(pc),
                                                  ctypes.byref(hc), _ptr(labels), ctypes.byref(cl), _stream(stream))
            _check(st, "vm_segment_frame_steppable")
        return cl


def cluster_view(off, x, y, z, tag, meta, key=None) -> Clusters:
    """vm_clusters over caller-owned device tensors (off int32[K+1], x/y/z
    float32[N], tag int32[K], meta int32[2] = (K, N))."""
    K = int(tag.shape[0])
    N = int(x.shape[0])
    return Clusters(K, N, _ptr(meta), _ptr(off), _ptr(x), _ptr(y), _ptr(z), _ptr(key), _ptr(tag))


def clusters_from_host(off, xyz, tag):
    """Upload a host CSR (off uint32[K+1], xyz float32[N,3], tag uint32[K]) to
    device tensors and return (vm_clusters view, dict of the owning tensors;
    keep it alive while the view is used)."""
    import torch
    off = np.ascontiguousarray(np.asarray(off, np.uint32))
    xyz = np.asarray(xyz, np.float32).reshape(-1, 3)
    tag = np.ascontiguousarray(np.asarray(tag, np.uint32))
    t = dict(off=torch.from_numpy(off.view(np.int32)).cuda(),
             x=torch.from_numpy(np.ascontiguousarray(xyz[:, 0])).cuda(),
             y=torch.from_numpy(np.ascontiguousarray(xyz[:, 1])).cuda(),
             z=torch.from_numpy(np.ascontiguousarray(xyz[:, 2])).cuda(),
             tag=torch.from_numpy(tag.view(np.int32)).cuda(),
             meta=torch.tensor([len(tag), len(xyz)], dtype=torch.int32).cuda())
    return cluster_view(t["off"], t["x"], t["y"], t["z"], t["tag"], t["meta"]), t


def workspace_bytes(k_cap: int, n_cap: int, n_hyp: int) -> int:
    return int(lib().vm_workspace_bytes(int(k_cap), int(n_cap), int(n_hyp)))


def ransac_planes(cl: Clusters, params: RansacParams, out: PlaneBuffers, work, stream=None) -> None:
    pc = out.c()
    _check(lib().vm_ransac_planes(ctypes.byref(cl), ctypes.byref(params), ctypes.byref(pc), _ptr(work),
                                  int(work.numel() * work.element_size()), _stream(stream)), "vm_ransac_planes")


NOALLOC_WORK_BYTES = 64 << 20   # VM_NOALLOC_WORK_BYTES


def ransac_planes_noalloc(cl: Clusters, params: RansacParams, out: PlaneBuffers, stream=None) -> None:
    """vm_ransac_planes with the library's fixed per-GPU workspace (allocates nothing)."""
    pc = out.c()
    _check(lib().vm_ransac_planes_noalloc(ctypes.byref(cl), ctypes.byref(params), ctypes.byref(pc), _stream(stream)),
           "vm_ransac_planes_noalloc")


def set_count_config(cfg: Optional[dict] = None) -> None:
    """Set the counting decomposition (None: the defaults); keys as CountConfig."""
    if cfg is None:
        _check(lib().vm_set_count_config(None), "vm_set_count_config")
        return
    c = get_count_config()
    for k, v in cfg.items():
        if k not in c:
            raise KeyError(k)
        c[k] = int(v)
    _check(lib().vm_set_count_config(ctypes.byref(CountConfig(**c))), "vm_set_count_config")


def get_count_config() -> dict:
    c = CountConfig()
    _check(lib().vm_get_count_config(ctypes.byref(c)), "vm_get_count_config")
    return c.as_dict()


def autotune_count(cl: Clusters, params: RansacParams, out: PlaneBuffers, work, stream=None, reps: int = 3) -> dict:
    """Time the counting decompositions on this workload, keep and return the fastest."""
    pc, best = out.c(), CountConfig()
    _check(lib().vm_autotune_count(ctypes.byref(cl), ctypes.byref(params), ctypes.byref(pc), _ptr(work),
                                   int(work.numel() * work.element_size()), _stream(stream), int(reps),
                                   ctypes.byref(best)), "vm_autotune_count")
    return best.as_dict()


def hulls(cl: Clusters, planes: PlaneBuffers, out: HullBuffers, work, stream=None) -> None:
    pc, hc = planes.c(), out.c()
    _check(lib().vm_hulls(ctypes.byref(cl), ctypes.byref(pc), ctypes.byref(hc), _ptr(work),
                          int(work.numel() * work.element_size()), _stream(stream)), "vm_hulls")


def planes_hulls(cl: Clusters, params: RansacParams, planes: PlaneBuffers, hulls_out: "HullBuffers", work,
                 stream=None) -> None:
    """vm_planes_hulls: RANSAC planes and polygons of every cluster in one persistent launch."""
    pc, hc = planes.c(), hulls_out.c()
    _check(lib().vm_planes_hulls(ctypes.byref(cl), ctypes.byref(params), ctypes.byref(pc), ctypes.byref(hc),
                                 _ptr(work), int(work.numel() * work.element_size()), _stream(stream)),
           "vm_planes_hulls")


def multi_workspace_bytes(k_cap: int, n_cap: int, n_hyp: int) -> int:
    return int(lib().vm_multi_workspace_bytes(int(k_cap), int(n_cap), int(n_hyp)))


def planes_hulls_multi(sets, frames, params: RansacParams, planes, hulls_out, k_cap: int, n_cap: int, work,
                       stream=None) -> None:
    """vm_planes_hulls_multi: several cluster sets (vm_clusters views) in one persistent pass; set i uses
    RNG frame word frames[i] and writes planes[i] / hulls_out[i]."""
    n = len(sets)
    cs = (Clusters * n)(*sets)
    fr = (ctypes.c_uint32 * n)(*[int(f) & 0xFFFFFFFF for f in frames])
    ps = (Planes * n)(*[p.c() for p in planes])
    hs = (HullsOut * n)(*[h.c() for h in hulls_out])
    _check(lib().vm_planes_hulls_multi(n, cs, fr, ctypes.byref(params), ps, hs, int(k_cap), int(n_cap), _ptr(work),
                                       int(work.numel() * work.element_size()), _stream(stream)),
           "vm_planes_hulls_multi")


def set_fused_config(cfg: Optional[dict] = None) -> None:
    """Set the persistent pass's work split (None: the defaults, and forget autotuned entries)."""
    if cfg is None:
        _check(lib().vm_set_fused_config(None), "vm_set_fused_config")
        return
    c = get_fused_config()
    for k, v in cfg.items():
        if k not in c:
            raise KeyError(k)
        c[k] = int(v)
    _check(lib().vm_set_fused_config(ctypes.byref(FusedConfig(**c))), "vm_set_fused_config")


def get_fused_config() -> dict:
    c = FusedConfig()
    _check(lib().vm_get_fused_config(ctypes.byref(c)), "vm_get_fused_config")
    return c.as_dict()


def autotune_fused(cl: Clusters, params: RansacParams, planes: PlaneBuffers, hulls_out: "HullBuffers", work,
                   stream=None, reps: int = 2) -> dict:
    """Time the persistent pass's splits on this workload; the fastest is kept for the call's shape bucket."""
    pc, hc, best = planes.c(), hulls_out.c(), FusedConfig()
    _check(lib().vm_autotune_fused(ctypes.byref(cl), ctypes.byref(params), ctypes.byref(pc), ctypes.byref(hc),
                                   _ptr(work), int(work.numel() * work.element_size()), _stream(stream), int(reps),
                                   ctypes.byref(best)), "vm_autotune_fused")
    return best.as_dict()


class Graph:
    """A captured sequence of library calls (vm_capture_begin/end), replayed with launch()."""

    def __init__(self, handle):
        self._h = handle

    def launch(self, stream=None) -> None:
        _check(lib().vm_graph_launch(self._h, _stream(stream)), "vm_graph_launch")

    def close(self) -> None:
        if self._h is not None and self._h.value:
            lib().vm_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class capture:
    """``with vm.capture(stream) as cap: ...library calls...`` then ``cap.graph.launch()``.
    The stream must not be the null stream (use a torch.cuda.Stream)."""

    def __init__(self, stream):
        self.stream = stream
        self.graph = None

    def __enter__(self):
        _check(lib().vm_capture_begin(_stream(self.stream)), "vm_capture_begin")
        return self

    def __exit__(self, exc_type, exc, tb):
        h = _P()
        st = lib().vm_capture_end(_stream(self.stream), ctypes.byref(h))
        if exc_type is None:
            _check(st, "vm_capture_end")
            self.graph = Graph(h)
        elif h.value:
            lib().vm_graph_destroy(h)
        return False


def set_stage_timing(enable: bool) -> None:
    _check(lib().vm_set_stage_timing(1 if enable else 0), "vm_set_stage_timing")


def stage_times() -> Tuple[np.ndarray, np.ndarray]:
    """(milliseconds, launches) per stage since the last call (synchronises)."""
    ms = (ctypes.c_double * len(STAGES))()
    n = (ctypes.c_uint64 * len(STAGES))()
    _check(lib().vm_stage_times(ms, n, len(STAGES)), "vm_stage_times")
    return np.array(ms[:]), np.array(n[:], dtype=np.int64)


class _DevArray:
    """Zero-copy view of library-owned device memory for torch."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False), "version": 2}


def device_view(ptr: int, n: int, dtype):
    """torch tensor aliasing n elements at a device pointer owned by the library."""
    import torch
    ts = {np.uint32: "<i4", np.int32: "<i4", np.float32: "<f4"}[dtype]   # uint32 travels as int32 bits
    if n == 0 or not ptr:
        return torch.zeros(0, dtype={np.uint32: torch.int32, np.int32: torch.int32, np.float32: torch.float32}[dtype],
                           device="cuda")
    return torch.as_tensor(_DevArray(ptr, n, ts), device="cuda")


def read_clusters(cl: Clusters):
    """Copy a device cluster view to host numpy arrays (synchronises)."""
    import torch
    torch.cuda.synchronize()

    def dev(ptr, n, dtype):
        return device_view(ptr, n, dtype).cpu().numpy().view(dtype).copy()

    meta = dev(cl.d_meta, 2, np.uint32)
    K, N = int(meta[0]), int(meta[1])
    return dict(K=K, N=N, off=dev(cl.d_off, K + 1, np.uint32), tag=dev(cl.d_tag, K, np.uint32),
                x=dev(cl.d_x, N, np.float32), y=dev(cl.d_y, N, np.float32), z=dev(cl.d_z, N, np.float32),
                key=dev(cl.d_key, N, np.uint32) if cl.d_key else None)


lib()

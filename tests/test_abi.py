"""The C ABI: the library loads and exports every function include/vm.h
declares; host-side argument checks reject bad input before any device work
(no GPU needed for these)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+(vm_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_parses():
    names = _declared()
    for n in ("vm_insert", "vm_ccl", "vm_ransac_planes", "vm_hulls", "vm_segment_frame", "vm_map_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2510_01592_amd as vm
    L = vm.lib()
    for n in _declared():
        assert hasattr(L, n), n
    assert sorted(vm.EXPORTED) == _declared()


def test_status_strings_and_version():
    import paper_2510_01592_amd as vm
    assert vm.version() >= 100
    assert vm.status_string(0) == "ok"
    assert vm.status_string(-1) == "invalid argument"
    assert "unknown" in vm.status_string(-99)


def test_workspace_bytes_monotone():
    import paper_2510_01592_amd as vm
    a = vm.workspace_bytes(10, 1000, 64)
    assert a > 0
    assert vm.workspace_bytes(20, 1000, 64) > a
    assert vm.workspace_bytes(10, 2000, 64) > a
    assert vm.workspace_bytes(10, 1000, 128) > a


def test_argument_errors_without_device_work():
    import paper_2510_01592_amd as vm
    L = vm.lib()
    h = ctypes.c_void_p()
    # null descriptor / out pointer
    assert L.vm_map_create(None, ctypes.byref(h)) == vm.VM_E_ARG
    d = vm.MapDesc()
    d.voxel_size = 0.0
    assert L.vm_map_create(ctypes.byref(d), ctypes.byref(h)) == vm.VM_E_ARG
    d.voxel_size = 0.01
    for i in range(3):
        d.dims[i] = 4096
    d.hash_capacity_log2 = 12
    assert L.vm_map_create(ctypes.byref(d), ctypes.byref(h)) == vm.VM_E_ARG     # 2^36 cells
    for i in range(3):
        d.dims[i] = 8
    d.hash_capacity_log2 = 40
    assert L.vm_map_create(ctypes.byref(d), ctypes.byref(h)) == vm.VM_E_ARG
    # null map handles
    assert L.vm_insert(None, None, 0, None, None) == vm.VM_E_ARG
    assert L.vm_clear_rays(None, None, 0, None, None) == vm.VM_E_ARG
    assert L.vm_map_shift(None, 1, 0, 0, None) == vm.VM_E_ARG
    assert L.vm_map_recenter(None, None, None, None) == vm.VM_E_ARG
    assert L.vm_map_origin(None, None) == vm.VM_E_ARG
    assert L.vm_map_destroy(None) == vm.VM_E_ARG
    assert L.vm_ccl(None, 30, None, None, None) == vm.VM_E_ARG
    assert L.vm_ccl_propagate(None, 30, None, None, None, None) == vm.VM_E_ARG
    # bad RANSAC parameters are rejected before any device pointer is touched
    cl = vm.Clusters(1, 1, 8, 8, 8, 8, 8, None, 8)
    pl = vm.Planes(1, 1, 8, 8, 8, 8, 8, None, None, 8)
    assert L.vm_capture_begin(None) == vm.VM_E_ARG
    assert L.vm_graph_launch(None, None) == vm.VM_E_ARG
    assert L.vm_graph_destroy(None) == vm.VM_E_ARG
    bad = vm.RansacParams(0, 0.01, 1, 0, 0)
    assert L.vm_ransac_planes(ctypes.byref(cl), ctypes.byref(bad), ctypes.byref(pl), 8, 1 << 20, None) == vm.VM_E_ARG
    bad = vm.RansacParams(16, -1.0, 1, 0, 0, None)
    assert L.vm_ransac_planes(ctypes.byref(cl), ctypes.byref(bad), ctypes.byref(pl), 8, 1 << 20, None) == vm.VM_E_ARG
    bad = vm.RansacParams(16, 0.01, 1, 0, 7)
    assert L.vm_ransac_planes(ctypes.byref(cl), ctypes.byref(bad), ctypes.byref(pl), 8, 1 << 20, None) == vm.VM_E_ARG
    ok = vm.RansacParams(16, 0.01, 1, 0, 0)
    assert L.vm_ransac_planes(ctypes.byref(cl), ctypes.byref(ok), ctypes.byref(pl), 8, 16, None) == vm.VM_E_CAPACITY
    # the allocation-free form: the same argument checks, and a workspace
    # beyond its fixed size is refused before any device work
    bad = vm.RansacParams(0, 0.01, 1, 0, 0)
    assert L.vm_ransac_planes_noalloc(ctypes.byref(cl), ctypes.byref(bad), ctypes.byref(pl), None) == vm.VM_E_ARG
    assert L.vm_ransac_planes_noalloc(None, ctypes.byref(ok), ctypes.byref(pl), None) == vm.VM_E_ARG
    huge = vm.Clusters(1, 1 << 30, 8, 8, 8, 8, 8, None, 8)
    assert vm.workspace_bytes(1, 1 << 30, 16) > vm.NOALLOC_WORK_BYTES
    assert L.vm_ransac_planes_noalloc(ctypes.byref(huge), ctypes.byref(ok), ctypes.byref(pl), None) == vm.VM_E_CAPACITY
    # the persistent form: argument checks and its cluster bound, before any device work
    hl = vm.HullsOut(1, 1, 8, 8, 8, 8, 8)
    assert L.vm_planes_hulls(ctypes.byref(cl), ctypes.byref(bad), ctypes.byref(pl), ctypes.byref(hl), 8, 1 << 20,
                             None) == vm.VM_E_ARG
    assert L.vm_planes_hulls(ctypes.byref(cl), ctypes.byref(ok), ctypes.byref(pl), None, 8, 1 << 20, None) == vm.VM_E_ARG
    many = vm.Clusters(70000, 1000, 8, 8, 8, 8, 8, None, 8)
    plm = vm.Planes(70000, 1, 8, 8, 8, 8, 8, None, None, 8)
    hlm = vm.HullsOut(70000, 1, 8, 8, 8, 8, 8)
    assert L.vm_planes_hulls(ctypes.byref(many), ctypes.byref(ok), ctypes.byref(plm), ctypes.byref(hlm), 8, 1 << 40,
                             None) == vm.VM_E_CAPACITY
    assert L.vm_planes_hulls(ctypes.byref(cl), ctypes.byref(ok), ctypes.byref(pl), ctypes.byref(hl), 8, 16,
                             None) == vm.VM_E_CAPACITY
    # steppable path: parameter checks before anything else
    for bad_sp in (vm.StepParams(0, 3, 0.9, 0.05), vm.StepParams(3, 3, 0.9, 0.05), vm.StepParams(1, 3, 1.5, 0.05),
                   vm.StepParams(1, 3, 0.9, 0.0)):
        assert L.vm_ccl_steppable(8, ctypes.byref(bad_sp), 30, None, None, None, None, None) == vm.VM_E_ARG
    assert L.vm_ccl_steppable(None, ctypes.byref(vm.step_params()), 30, None, None, None, None, None) == vm.VM_E_ARG
    ms = (ctypes.c_double * 8)()
    n = (ctypes.c_uint64 * 8)()
    assert L.vm_stage_times(ms, n, -1) == vm.VM_E_ARG


def test_struct_layouts_match_header_sizes():
    import paper_2510_01592_amd as vm
    # natural C alignment on x86-64 / amdgcn host ABI
    assert ctypes.sizeof(vm.MapDesc) == 3 * 8 + 8 + 3 * 4 + 4 + 4 + 4
    assert ctypes.sizeof(vm.MapStats) == 4 * 8 + 2 * 4 + 8 + 8 + 8
    assert ctypes.sizeof(vm.Pose) == 12 * 8
    assert ctypes.sizeof(vm.RansacParams) == 32
    assert ctypes.sizeof(vm.SegParams) == 40
    assert ctypes.sizeof(vm.Clusters) == 8 + 7 * 8
    assert ctypes.sizeof(vm.Planes) == 8 + 8 * 8
    assert ctypes.sizeof(vm.HullsOut) == 8 + 5 * 8
    assert ctypes.sizeof(vm.StepParams) == 8 + 2 * 8
    assert vm.COS_15 == float.fromhex("0x1.ee8dd4748bf15p-1")


def test_count_config_set_get_and_validation():
    """The counting decomposition is host state: set/get round-trip, out-of-range
    fields are rejected with nothing changed, NULL restores the defaults."""
    import paper_2510_01592_amd as vm
    L = vm.lib()
    vm.set_count_config(None)
    d = vm.get_count_config()
    assert d == {"count_grid": 16384, "chunk_mult": 2, "wave_max_points": 256, "plane_max_points": 256}
    try:
        vm.set_count_config({"count_grid": 1024, "chunk_mult": 4, "wave_max_points": 512, "plane_max_points": 64})
        assert vm.get_count_config() == {"count_grid": 1024, "chunk_mult": 4, "wave_max_points": 512,
                                         "plane_max_points": 64}
        cur = vm.get_count_config()
        bad = [dict(count_grid=0), dict(count_grid=12), dict(count_grid=65544), dict(chunk_mult=0),
               dict(chunk_mult=17), dict(wave_max_points=1025), dict(plane_max_points=257),
               dict(wave_max_points=32, plane_max_points=64)]
        for b in bad:
            c = dict(cur)
            c.update(b)
            assert L.vm_set_count_config(ctypes.byref(vm.CountConfig(**c))) == vm.VM_E_ARG, b
            assert vm.get_count_config() == cur
        # the extremes of the ranges are accepted
        for c in (dict(count_grid=8, chunk_mult=1, wave_max_points=0, plane_max_points=0),
                  dict(count_grid=65536, chunk_mult=16, wave_max_points=1024, plane_max_points=256)):
            vm.set_count_config(c)
            assert vm.get_count_config() == c
        assert L.vm_get_count_config(None) == vm.VM_E_ARG
        # the autotuner rejects a bad repeat count before any device work
        assert L.vm_autotune_count(None, None, None, None, 0, None, 0, None) == vm.VM_E_ARG
        assert L.vm_autotune_count(None, None, None, None, 0, None, 17, None) == vm.VM_E_ARG
    finally:
        vm.set_count_config(None)
    assert vm.get_count_config() == d


def test_fused_config_set_get_and_validation():
    import paper_2510_01592_amd as vm
    L = vm.lib()
    vm.set_fused_config(None)
    d = vm.get_fused_config()
    assert d == {"hyp_chunk": 512, "small_max": 0, "groups_per_cu": 5}
    try:
        for b in (dict(hyp_chunk=32), dict(hyp_chunk=96), dict(hyp_chunk=576), dict(small_max=257),
                  dict(groups_per_cu=0), dict(groups_per_cu=9)):
            c = dict(d)
            c.update(b)
            assert L.vm_set_fused_config(ctypes.byref(vm.FusedConfig(**c))) == vm.VM_E_ARG, b
            assert vm.get_fused_config() == d
        vm.set_fused_config(dict(hyp_chunk=512, small_max=0, groups_per_cu=8))
        assert vm.get_fused_config() == {"hyp_chunk": 512, "small_max": 0, "groups_per_cu": 8}
        assert L.vm_get_fused_config(None) == vm.VM_E_ARG
        assert L.vm_autotune_fused(None, None, None, None, None, 0, None, 0, None) == vm.VM_E_ARG
    finally:
        vm.set_fused_config(None)
    assert vm.get_fused_config() == d

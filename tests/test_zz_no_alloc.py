"""The allocation-free RANSAC entry point (vm_ransac_planes_noalloc) against
vm_ransac_planes with a caller workspace: identical results, bit for bit, on
two calls in a row, the second smaller (the shared per-GPU workspace keeps the
first call's contents)."""
import ctypes

import numpy as np
import pytest

import scenes
from tests.gpu_util import cluster_tensors, note, planes_np

pytestmark = pytest.mark.gpu

SEED = 0x5EED


def _clusters(seed, n_clusters, n_min, n_max, degenerate):
    off, xyz = scenes.batched_clusters(seed=seed, n_clusters=n_clusters, n_min=n_min, n_max=n_max)
    parts = [xyz[off[i]:off[i + 1]] for i in range(n_clusters)]
    if degenerate:
        t = np.linspace(0, 1, 40)
        parts += [np.zeros((0, 3), np.float32), xyz[:1], xyz[:2], xyz[:3], np.c_[t, 2 * t, t].astype(np.float32)]
    off = np.zeros(len(parts) + 1, np.uint32)
    off[1:] = np.cumsum([len(p) for p in parts])
    xyz = np.concatenate(parts).astype(np.float32)
    tag = np.arange(len(parts), dtype=np.uint32) * 7919 + 11
    return off, xyz, tag


def _view(vm, off, xyz, tag):
    T = cluster_tensors(off, xyz, tag)
    return vm.cluster_view(T["off"], T["x"], T["y"], T["z"], T["tag"], T["meta"]), T


def _same(a, b):
    for k in ("plane", "best", "nin", "in_off", "counts", "hyp"):
        assert np.array_equal(np.ascontiguousarray(a[k]).view(np.uint8), np.ascontiguousarray(b[k]).view(np.uint8)), k
    n = int(a["in_off"][len(a["best"])])
    assert np.array_equal(a["in_idx"][:n], b["in_idx"][:n])
    assert a["status"] == b["status"] == 0


def test_noalloc_matches_workspace_form_two_calls():
    import torch
    import paper_2510_01592_amd as vm
    cases = [(_clusters(7, 60, 3, 30_000, True), 384, 5), (_clusters(9, 17, 40, 5_000, False), 256, 2)]
    views = [_view(vm, *c[0]) for c in cases]
    for (c, H, frame), (cl, _) in zip(cases, views):
        assert vm.workspace_bytes(cl.k_cap, cl.n_cap, H) <= vm.NOALLOC_WORK_BYTES
    outs = []
    # the allocation-free calls back to back: the second (smaller) call sees
    # the first call's leftovers in the shared workspace
    for i, ((c, H, frame), (cl, _)) in enumerate(zip(cases, views)):
        note(f"noalloc call {i}: K={cl.k_cap} N={cl.n_cap} H={H}")
        pb = vm.PlaneBuffers.alloc(cl.k_cap, cl.n_cap, H, with_all=True)
        vm.ransac_planes_noalloc(cl, vm.ransac_params(H, 0.01, SEED, frame), pb)
        outs.append(pb)
    torch.cuda.synchronize()
    for i, ((c, H, frame), (cl, _)) in enumerate(zip(cases, views)):
        note(f"workspace call {i}")
        ref = vm.PlaneBuffers.alloc(cl.k_cap, cl.n_cap, H, with_all=True)
        work = torch.empty(vm.workspace_bytes(cl.k_cap, cl.n_cap, H), dtype=torch.uint8, device="cuda")
        vm.ransac_planes(cl, vm.ransac_params(H, 0.01, SEED, frame), ref, work)
        torch.cuda.synchronize()
        _same(planes_np(outs[i]), planes_np(ref))
        assert int((ref.best_h >= 0).sum()) > 0


def test_noalloc_rejects_oversized_workspace():
    import paper_2510_01592_amd as vm
    off, xyz, tag = _clusters(9, 4, 40, 400, False)
    cl, _keep = _view(vm, off, xyz, tag)
    big = vm.Clusters(cl.k_cap, 1 << 26, cl.d_meta, cl.d_off, cl.d_x, cl.d_y, cl.d_z, None, cl.d_tag)
    pb = vm.PlaneBuffers.alloc(cl.k_cap, 1024, 64)
    pc = pb.c()
    st = vm.lib().vm_ransac_planes_noalloc(ctypes.byref(big), ctypes.byref(vm.ransac_params(64)), ctypes.byref(pc),
                                           None)
    assert st == vm.VM_E_CAPACITY

"""Helpers shared by the GPU parity tests: run the library through its C ABI
and the oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def note(msg: str) -> None:
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def bits(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a.view(np.uint64)


def export_np(m):
    key, cnt, sums, mean = m.export()
    return (key.cpu().numpy().view(np.uint32), cnt.cpu().numpy().view(np.uint32),
            sums.cpu().numpy().view(np.uint64), mean.cpu().numpy())


def assert_map_equal(m, om: oracle.OracleMap) -> None:
    key, cnt, sums, mean = export_np(m)
    assert len(key) == len(om.key), (len(key), len(om.key))
    assert np.array_equal(key, om.key)
    assert np.array_equal(cnt, om.cnt)
    assert np.array_equal(sums, om.sums)
    assert np.array_equal(bits(mean), bits(om.means()))


def cluster_tensors(off: np.ndarray, xyz: np.ndarray, tag: np.ndarray):
    import torch
    d = dict(device="cuda")
    t = dict(
        off=torch.from_numpy(off.astype(np.int32)).to(**d),
        x=torch.from_numpy(np.ascontiguousarray(xyz[:, 0])).to(**d),
        y=torch.from_numpy(np.ascontiguousarray(xyz[:, 1])).to(**d),
        z=torch.from_numpy(np.ascontiguousarray(xyz[:, 2])).to(**d),
        tag=torch.from_numpy(tag.astype(np.int64).astype(np.uint32).view(np.int32)).to(**d),
        meta=torch.tensor([len(tag), len(xyz)], dtype=torch.int32, **d),
    )
    return t


def run_planes_and_hulls(vm, cl, k_cap, n_cap, n_hyp, eps, seed, frame, with_all=True):
    import torch
    work = torch.empty(vm.workspace_bytes(min(k_cap, cl.k_cap), cl.n_cap, n_hyp), dtype=torch.uint8, device="cuda")
    pb = vm.PlaneBuffers.alloc(k_cap, n_cap, n_hyp, with_all=with_all)
    hb = vm.HullBuffers.alloc(k_cap, n_cap)
    vm.ransac_planes(cl, vm.ransac_params(n_hyp, eps, seed, frame), pb, work)
    vm.hulls(cl, pb, hb, work)
    torch.cuda.synchronize()
    return pb, hb


def planes_np(pb):
    return dict(plane=pb.plane.cpu().numpy(), best=pb.best_h.cpu().numpy(), nin=pb.n_inliers.cpu().numpy(),
                in_off=pb.in_off.cpu().numpy().view(np.uint32), in_idx=pb.in_idx.cpu().numpy().view(np.uint32),
                counts=None if pb.counts is None else pb.counts.cpu().numpy(),
                hyp=None if pb.hyp is None else pb.hyp.cpu().numpy(), status=int(pb.status.cpu()[0]))


def hulls_np(hb):
    return dict(v_off=hb.v_off.cpu().numpy().view(np.uint32), v_idx=hb.v_idx.cpu().numpy().view(np.uint32),
                v_xyz=hb.v_xyz.cpu().numpy(), area=hb.area.cpu().numpy(), status=int(hb.status.cpu()[0]))


def compare_cluster(k: int, P: dict, Hh: dict, ref: oracle.ClusterResult, check_all_hyp: bool = True) -> None:
    r = ref.ransac
    assert P["best"][k] == r.best_h, (k, P["best"][k], r.best_h)
    if check_all_hyp and P["counts"] is not None:
        assert np.array_equal(P["counts"][k], r.counts), (k, np.nonzero(P["counts"][k] != r.counts)[0][:10])
        assert np.array_equal(bits(P["hyp"][k]), bits(r.hyp)), k
    assert np.array_equal(bits(P["plane"][k]), bits(r.plane)), (k, P["plane"][k], r.plane)
    a, b = int(P["in_off"][k]), int(P["in_off"][k + 1])
    assert np.array_equal(P["in_idx"][a:b], r.inliers), k
    assert P["nin"][k] == len(r.inliers)
    va, vb = int(Hh["v_off"][k]), int(Hh["v_off"][k + 1])
    if ref.hull is None:
        assert vb == va and Hh["area"][k] == 0.0
        return
    assert abs(Hh["area"][k] - ref.hull.area) <= 1e-5 * abs(ref.hull.area) + 1e-12, (k, Hh["area"][k], ref.hull.area)
    assert np.array_equal(Hh["v_idx"][va:vb], ref.hull_local), (k, Hh["v_idx"][va:vb], ref.hull_local)
    assert np.array_equal(bits(Hh["v_xyz"][va:vb]), bits(ref.hull.xyz)), k


def hull_path_clusters():
    """Discs (about a tenth of their inliers survive the octagon filter),
    rotated squares (few survivors) and thin rings (nearly every point on the
    hull) whose hulls reach every path: one wave, the workgroup chain, the
    64-direction refinement of survivor sets above 512 (the larger discs drop
    far below the workgroup sort's size with it; the 1500-point ring stays
    large and is sorted in LDS), and the sort in global memory (the larger
    rings stay above 2048); (off, xyz, tag)."""
    rng = np.random.default_rng(33)
    parts = []
    nrm = np.array([0.1, -0.2, 1.0]) / np.linalg.norm([0.1, -0.2, 1.0])
    a = np.cross(nrm, [1.0, 0.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(nrm, a)
    for n in (40, 200, 700, 1500, 3000, 8000, 30000, 60000):
        rad = 0.0056 * np.sqrt(n)
        r = rad * np.sqrt(rng.random(n))
        th = rng.random(n) * 2 * np.pi
        p = (r * np.cos(th))[:, None] * a + (r * np.sin(th))[:, None] * b + rng.normal(0, 0.002, n)[:, None] * nrm
        parts.append((p + [0.5, 0.5, 1.0]).astype(np.float32))
    for n in (1500, 3000, 6000):
        r = 0.3 + rng.normal(0, 1e-5, n)
        th = rng.random(n) * 2 * np.pi
        p = (r * np.cos(th))[:, None] * a + (r * np.sin(th))[:, None] * b
        parts.append((p + [0.5, 0.5, 1.0]).astype(np.float32))
    for n, ang in ((500, 0.3), (5000, 1.1)):
        s = (rng.random((n, 2)) - 0.5) * 0.01 * np.sqrt(n)
        c, si = np.cos(ang), np.sin(ang)
        uv = s @ np.array([[c, -si], [si, c]])
        parts.append(np.c_[uv, rng.normal(0, 0.002, n)].astype(np.float32))
    off = np.zeros(len(parts) + 1, np.uint32)
    off[1:] = np.cumsum([len(p) for p in parts])
    xyz = np.concatenate(parts)
    tag = np.arange(len(parts), dtype=np.uint32) * 7717 + 5
    return off, xyz, tag


def ragged_clusters(seed=7, n_clusters=60, n_max=30_000):
    """Log-uniform cluster sizes plus the degenerate sizes 0, 1, 2, 3 and a
    collinear cluster; (off, xyz, tag)."""
    import scenes
    off, xyz = scenes.batched_clusters(seed=seed, n_clusters=n_clusters, n_min=3, n_max=n_max)
    parts = [xyz[off[i]:off[i + 1]] for i in range(n_clusters)]
    t = np.linspace(0, 1, 40)
    parts += [np.zeros((0, 3), np.float32), xyz[:1], xyz[:2], xyz[:3], np.c_[t, 2 * t, t].astype(np.float32)]
    off = np.zeros(len(parts) + 1, np.uint32)
    off[1:] = np.cumsum([len(p) for p in parts])
    xyz = np.concatenate(parts).astype(np.float32)
    tag = np.arange(len(parts), dtype=np.uint32) * 7919 + 3
    return off, xyz, tag

// vm_propagate.hip -- Alg. 1 as the paper runs it: minimum-label propagation
// over the 26-adjacency of the occupied voxels, sweep after sweep until a
// sweep changes no label.  It reaches the same fixed point as the union-find
// labelling (every voxel takes the smallest key of its component) and serves
// as its comparison baseline.
//
//   k_lp_init:   L_i = key of voxel i (Alg. 1's L_i <- i, with keys as ids);
//   k_lp_sweep:  a thread per voxel visits its 13 neighbours of smaller key
//                (so every edge once); when the two labels differ, both ends
//                take the smaller one with atomicMin.  Whether anything
//                changed is reduced hierarchically: a lane flag, a wave
//                ballot, a workgroup flag in LDS, then one atomicOr per
//                workgroup into a device word the host reads between sweeps;
//   k_lp_finish: the labels as a forest for the grouping step (every voxel's
//                parent is its label's rank, the root counts its component).
#include "vm_common.h"

namespace vm {
namespace {

__device__ __forceinline__ bool lp_occupied(const uint32_t* __restrict__ bits, uint32_t key)
{
    return (bits[key >> 5] >> (key & 31)) & 1u;
}

__device__ __forceinline__ uint32_t lp_rank(const uint32_t* __restrict__ bits, const uint32_t* __restrict__ wrank,
                                            uint32_t key)
{
    return wrank[key >> 5] + __popc(bits[key >> 5] & ((1u << (key & 31)) - 1u));
}

__global__ void __launch_bounds__(kBlock) k_lp_init(const DevCounters* __restrict__ ctr,
                                                    const uint32_t* __restrict__ occ_key, uint32_t* __restrict__ label)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) label[r] = occ_key[r];
}

__global__ void __launch_bounds__(kBlock) k_lp_flags_clear(uint32_t* flag, uint32_t n)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) flag[i] = 0u;
}

__global__ void __launch_bounds__(kBlock) k_lp_sweep(Geom g, const DevCounters* __restrict__ ctr,
                                                     const uint32_t* __restrict__ bits,
                                                     const uint32_t* __restrict__ wrank,
                                                     const uint32_t* __restrict__ occ_key, uint32_t* label,
                                                     uint32_t* changed)
{
    __shared__ uint32_t s_changed;
    if (threadIdx.x == 0) s_changed = 0u;
    __syncthreads();
    const uint32_t V = ctr->n_occ;
    const int32_t NX = g.dims[0], NY = g.dims[1], NZ = g.dims[2];
    bool mine = false;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t key = occ_key[r];
        const int32_t x = (int32_t)(key % (uint32_t)NX), y = (int32_t)((key / (uint32_t)NX) % (uint32_t)NY),
                      z = (int32_t)(key / ((uint32_t)NX * (uint32_t)NY));
        uint32_t li = __hip_atomic_load(&label[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the 13 neighbours with smaller keys: dz = -1 (any dy, dx); dz = 0,
        // dy = -1 (any dx); dz = dy = 0, dx = -1
        for (int q = 0; q < 13; ++q) {
            const int dz = q < 9 ? -1 : 0;
            const int dy = q < 9 ? q / 3 - 1 : (q < 12 ? -1 : 0);
            const int dx = q < 12 ? q % 3 - 1 : -1;
            const int32_t xx = x + dx, yy = y + dy, zz = z + dz;
            if (xx < 0 || yy < 0 || zz < 0 || xx >= NX || yy >= NY || zz >= NZ) continue;
            const uint32_t k2 = (uint32_t)xx + (uint32_t)NX * ((uint32_t)yy + (uint32_t)NY * (uint32_t)zz);
            if (!lp_occupied(bits, k2)) continue;
            const uint32_t r2 = lp_rank(bits, wrank, k2);
            const uint32_t lj = __hip_atomic_load(&label[r2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (lj == li) continue;
            const uint32_t m = li < lj ? li : lj;
            // both ends take the smaller label; a change either way is reported
            if (lj > m && atomicMin(&label[r2], m) > m) mine = true;
            if (li > m) {
                if (atomicMin(&label[r], m) > m) mine = true;
                li = m;
            }
        }
    }
    if (__ballot(mine) && (threadIdx.x & (kWave - 1)) == 0) s_changed = 1u;
    __syncthreads();
    if (threadIdx.x == 0 && s_changed) atomicOr(changed, 1u);
}

// parent = rank of the label's voxel; each root counts its component (one
// atomic per distinct root per wave)
__global__ void __launch_bounds__(kBlock) k_lp_finish(const DevCounters* __restrict__ ctr,
                                                      const uint32_t* __restrict__ bits,
                                                      const uint32_t* __restrict__ wrank,
                                                      const uint32_t* __restrict__ label, uint32_t* __restrict__ parent,
                                                      uint32_t* __restrict__ csize)
{
    const uint32_t V = ctr->n_occ;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t b0 = blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); b0 < V; b0 += stride) {
        const uint32_t r = b0 + (uint32_t)lane;
        uint32_t root = 0;
        const bool v = r < V;
        if (v) {
            root = lp_rank(bits, wrank, label[r]);
            parent[r] = root;
        }
        uint64_t pending = __ballot(v);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const uint32_t lr = __shfl(root, leader, kWave);
            const bool same = v && root == lr;
            const uint32_t cnt = (uint32_t)__popcll(__ballot(same));
            if (lane == leader) atomicAdd(&csize[lr], cnt);
            pending &= ~__ballot(same);
        }
    }
}

}  // namespace

hipError_t launch_lp_init(const SegBuffers& b, uint32_t cap, uint32_t* label, DevCounters* ctr, hipStream_t s)
{
    k_lp_init<<<grid_for(cap), kBlock, 0, s>>>(ctr, b.occ_key, label);
    return hipGetLastError();
}

hipError_t launch_lp_sweeps(const Geom& g, const uint32_t* bits, const SegBuffers& b, uint32_t cap, uint32_t* label,
                            uint32_t* changed, uint32_t sweeps, DevCounters* ctr, hipStream_t s)
{
    // sweep i of the batch reports into changed[i]
    k_lp_flags_clear<<<1, kBlock, 0, s>>>(changed, sweeps);
    for (uint32_t i = 0; i < sweeps; ++i)
        k_lp_sweep<<<grid_for(cap), kBlock, 0, s>>>(g, ctr, bits, b.wrank, b.occ_key, label, changed + i);
    return hipGetLastError();
}

hipError_t launch_lp_finish(const uint32_t* bits, SegBuffers& b, uint32_t cap, const uint32_t* label,
                            DevCounters* ctr, hipStream_t s)
{
    k_lp_finish<<<grid_for(cap), kBlock, 0, s>>>(ctr, bits, b.wrank, label, b.parent, b.csize);
    return hipGetLastError();
}

}  // namespace vm

// vm_map.hip -- the sparse voxel map (Sec. III-B): insertion of a point frame
// (Eq. (1)), the occupancy index, and map export/import.
//
// Storage.  Occupied voxels live in an open-addressing hash keyed by the
// voxel's linear index; the payload per slot is a point count and three
// 64-bit sums of fixed-point in-voxel offsets (quantum s*2^-20).  Integer
// atomics make the accumulated mean exact and independent of the order in
// which points (and lanes, and XCDs) arrive.  Beside the hash, one bit per
// grid cell marks occupancy; its popcount prefix gives every occupied voxel a
// dense rank in ascending key order, which the clustering stages use as their
// index space (4 MB of bits for a 400x400x200 grid).
#include "vm_common.h"

namespace vm {
namespace {

__device__ __forceinline__ void wave_add_u64(unsigned long long* dst, uint32_t v)
{
    // one atomic per wave: sum over lanes via popcount-free shuffle tree
    unsigned long long s = v;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) s += __shfl_xor(s, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && s) atomicAdd(dst, s);
}

__global__ void __launch_bounds__(kBlock) k_insert(const float* __restrict__ xyz, int64_t n, Pose pose, Geom g,
                                                   Hash h, uint32_t* __restrict__ bits,
                                                   DevCounters* __restrict__ ctr)
{
    uint32_t n_in = 0, n_drop = 0, n_lost = 0, n_new = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const double lim0 = (double)g.dims[0] * 1048576.0;
    const double lim1 = (double)g.dims[1] * 1048576.0;
    const double lim2 = (double)g.dims[2] * 1048576.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double px = (double)xyz[3 * i + 0];
        const double py = (double)xyz[3 * i + 1];
        const double pz = (double)xyz[3 * i + 2];
        // map_from_sensor in fp64, one fused chain per output coordinate
        const double wx = fma(pose.R[2], pz, fma(pose.R[1], py, fma(pose.R[0], px, pose.t[0])));
        const double wy = fma(pose.R[5], pz, fma(pose.R[4], py, fma(pose.R[3], px, pose.t[1])));
        const double wz = fma(pose.R[8], pz, fma(pose.R[7], py, fma(pose.R[6], px, pose.t[2])));
        const double fx = floor((wx - g.origin[0]) * g.inv_q);
        const double fy = floor((wy - g.origin[1]) * g.inv_q);
        const double fz = floor((wz - g.origin[2]) * g.inv_q);
        // negated range tests also reject NaN
        if (!(fx >= 0.0 && fx < lim0 && fy >= 0.0 && fy < lim1 && fz >= 0.0 && fz < lim2)) {
            ++n_drop;
            continue;
        }
        const int64_t qx = (int64_t)fx, qy = (int64_t)fy, qz = (int64_t)fz;
        const uint32_t key = (uint32_t)((uint64_t)(qx >> 20) +
                                        (uint64_t)g.dims[0] * ((uint64_t)(qy >> 20) + (uint64_t)g.dims[1] * (uint64_t)(qz >> 20)));
        // find or claim the key's slot
        uint32_t s = hash_slot(key, h.log2cap);
        bool ok = false;
        for (uint32_t p = 0; p < kMaxProbe && p <= h.mask; ++p) {
            const uint32_t k = h.slot[s].key;
            if (k == key) { ok = true; break; }
            if (k == kEmpty) {
                const uint32_t old = atomicCAS(&h.slot[s].key, kEmpty, key);
                if (old == kEmpty) {
                    atomicOr(&bits[key >> 5], 1u << (key & 31));
                    ++n_new;
                    ok = true;
                    break;
                }
                if (old == key) { ok = true; break; }
            }
            s = (s + 1) & h.mask;
        }
        if (!ok) {
            ++n_lost;
            continue;
        }
        Slot* sl = &h.slot[s];
        atomicAdd(&sl->cnt, 1u);
        atomicAdd(&sl->sum[0], (unsigned long long)(qx & 0xFFFFF));
        atomicAdd(&sl->sum[1], (unsigned long long)(qy & 0xFFFFF));
        atomicAdd(&sl->sum[2], (unsigned long long)(qz & 0xFFFFF));
        ++n_in;
    }
    wave_add_u64(&ctr->points_in, n_in);
    wave_add_u64(&ctr->points_dropped, n_drop);
    wave_add_u64(&ctr->points_lost, n_lost);
    wave_add_u64(&ctr->occupied, n_new);
    if (__ballot(n_lost != 0) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&ctr->flags, (uint32_t)VM_FLAG_HASH_FULL);
}

__global__ void __launch_bounds__(kBlock) k_popc(const uint32_t* __restrict__ bits, uint32_t nwords,
                                                 uint32_t* __restrict__ out)
{
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += gridDim.x * blockDim.x)
        out[w] = __popc(bits[w]);
}

// Occupied keys in ascending order: word w's set bits go to ranks wrank[w]...
__global__ void __launch_bounds__(kBlock) k_compact(const uint32_t* __restrict__ bits, uint32_t nwords,
                                                    const uint32_t* __restrict__ wrank,
                                                    uint32_t* __restrict__ occ_key)
{
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += gridDim.x * blockDim.x) {
        uint32_t b = bits[w];
        uint32_t r = wrank[w];
        while (b) {
            const uint32_t j = __ffs(b) - 1;
            occ_key[r++] = (w << 5) | j;
            b &= b - 1;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_export(Geom g, Hash h, const uint32_t* __restrict__ occ_key,
                                                   const DevCounters* __restrict__ ctr, uint32_t* key_out,
                                                   uint32_t* cnt_out, unsigned long long* sum_out, float* mean_out,
                                                   uint64_t cap)
{
    const uint64_t n = ctr->n_occ < cap ? ctr->n_occ : cap;
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = occ_key[r];
        const uint32_t s = hash_find(h, k);
        uint32_t c = 0;
        unsigned long long sx = 0, sy = 0, sz = 0;
        if (s != kEmpty) {
            c = h.slot[s].cnt;
            sx = h.slot[s].sum[0];
            sy = h.slot[s].sum[1];
            sz = h.slot[s].sum[2];
        }
        if (key_out) key_out[r] = k;
        if (cnt_out) cnt_out[r] = c;
        if (sum_out) {
            sum_out[3 * r + 0] = sx;
            sum_out[3 * r + 1] = sy;
            sum_out[3 * r + 2] = sz;
        }
        if (mean_out && c) {
            const uint32_t ix = k % (uint32_t)g.dims[0];
            const uint32_t iy = (k / (uint32_t)g.dims[0]) % (uint32_t)g.dims[1];
            const uint32_t iz = k / ((uint32_t)g.dims[0] * (uint32_t)g.dims[1]);
            mean_out[3 * r + 0] = voxel_mean_axis(ix, sx, c, g.voxel_size, g.origin[0]);
            mean_out[3 * r + 1] = voxel_mean_axis(iy, sy, c, g.voxel_size, g.origin[1]);
            mean_out[3 * r + 2] = voxel_mean_axis(iz, sz, c, g.voxel_size, g.origin[2]);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_import(Geom g, Hash h, uint32_t* __restrict__ bits, DevCounters* ctr,
                                                   const uint32_t* __restrict__ key, const uint32_t* __restrict__ cnt,
                                                   const unsigned long long* __restrict__ sum, uint64_t n)
{
    uint32_t n_new = 0, n_lost = 0;
    const uint64_t ncell = (uint64_t)g.dims[0] * (uint64_t)g.dims[1] * (uint64_t)g.dims[2];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = key[i];
        if ((uint64_t)k >= ncell || cnt[i] == 0) { ++n_lost; continue; }   // not a voxel of this grid
        uint32_t s = hash_slot(k, h.log2cap);
        bool ok = false;
        for (uint32_t p = 0; p < kMaxProbe && p <= h.mask; ++p) {
            const uint32_t old = atomicCAS(&h.slot[s].key, kEmpty, k);
            if (old == kEmpty || old == k) { ok = true; break; }
            s = (s + 1) & h.mask;
        }
        if (!ok) { ++n_lost; continue; }
        h.slot[s].cnt = cnt[i];
        h.slot[s].sum[0] = sum[3 * i + 0];
        h.slot[s].sum[1] = sum[3 * i + 1];
        h.slot[s].sum[2] = sum[3 * i + 2];
        atomicOr(&bits[k >> 5], 1u << (k & 31));
        ++n_new;
    }
    wave_add_u64(&ctr->occupied, n_new);
    if (__ballot(n_lost != 0) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&ctr->flags, (uint32_t)VM_FLAG_HASH_FULL);
}

__global__ void __launch_bounds__(kBlock) k_clear_slots(Slot* __restrict__ slot, uint32_t cap)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += gridDim.x * blockDim.x) {
        Slot z;
        z.key = kEmpty;
        z.cnt = 0;
        z.sum[0] = z.sum[1] = z.sum[2] = 0;
        slot[i] = z;
    }
}

__global__ void k_stats(const DevCounters* __restrict__ c, uint32_t log2cap, vm_map_stats_t* out)
{
    if (threadIdx.x == 0) {
        out->occupied = c->occupied;
        out->points_in = c->points_in;
        out->points_dropped = c->points_dropped;
        out->points_lost = c->points_lost;
        out->status_flags = c->flags;
        out->hash_capacity_log2 = log2cap;
    }
}

}  // namespace

hipError_t launch_stats(const DevCounters* ctr, uint32_t log2cap, vm_map_stats_t* out, hipStream_t s)
{
    k_stats<<<1, 64, 0, s>>>(ctr, log2cap, out);
    return hipGetLastError();
}

hipError_t launch_insert(const float* xyz, int64_t n, const Pose& pose, const Geom& g, const Hash& h,
                         uint32_t* bits, DevCounters* ctr, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_insert<<<grid_for((uint64_t)n, kBlock, 16384), kBlock, 0, s>>>(xyz, n, pose, g, h, bits, ctr);
    return hipGetLastError();
}

hipError_t launch_rank(const Geom& g, const uint32_t* bits, SegBuffers& b, uint32_t /*cap*/, DevCounters* ctr,
                       hipStream_t s)
{
    k_popc<<<grid_for(g.nwords), kBlock, 0, s>>>(bits, g.nwords, b.wrank);
    hipError_t e = scan_exclusive_dev(b.wrank, b.wrank, nullptr, g.nwords, &ctr->n_occ, b.blk, s);
    if (e != hipSuccess) return e;
    k_compact<<<grid_for(g.nwords), kBlock, 0, s>>>(bits, g.nwords, b.wrank, b.occ_key);
    return hipGetLastError();
}

hipError_t launch_clear(const Geom& g, const Hash& h, uint32_t* bits, DevCounters* ctr, hipStream_t s)
{
    const uint32_t cap = h.mask + 1;
    hipError_t e;
    k_clear_slots<<<grid_for(cap, kBlock, 16384), kBlock, 0, s>>>(h.slot, cap);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemsetAsync(bits, 0, (size_t)g.nwords * sizeof(uint32_t), s)) != hipSuccess) return e;
    return hipMemsetAsync(ctr, 0, sizeof(DevCounters), s);
}

hipError_t launch_export(const Geom& g, const Hash& h, const SegBuffers& b, const DevCounters* ctr, uint32_t* key,
                         uint32_t* cnt, unsigned long long* sum, float* mean, uint64_t cap, hipStream_t s)
{
    k_export<<<grid_for(cap), kBlock, 0, s>>>(g, h, b.occ_key, ctr, key, cnt, sum, mean, cap);
    return hipGetLastError();
}

hipError_t launch_import(const Geom& g, const Hash& h, uint32_t* bits, DevCounters* ctr, const uint32_t* key,
                         const uint32_t* cnt, const unsigned long long* sum, uint64_t n, hipStream_t s)
{
    hipError_t e = launch_clear(g, h, bits, ctr, s);
    if (e != hipSuccess || n == 0) return e;
    k_import<<<grid_for(n), kBlock, 0, s>>>(g, h, bits, ctr, key, cnt, sum, n);
    return hipGetLastError();
}

}  // namespace vm

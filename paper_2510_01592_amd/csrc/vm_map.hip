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
#include "vm_tilescan.h"

namespace vm {
namespace {

// Counters are reduced per block before one atomic each (same-address device
// atomics from every wave would serialise).  Grids stay at most kMapGrid
// blocks; threads stride over the points.
constexpr int kMapGrid = 1024;

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
                if (old == kEmpty || old == key) { ok = true; break; }
            }
            s = (s + 1) & h.mask;
        }
        if (!ok) {
            ++n_lost;
            continue;
        }
        Slot* sl = &h.slot[s];
        // the point that takes a slot's count from 0 marks the voxel occupied:
        // a newly claimed slot, or one whose voxel was cleared (cleared voxels
        // keep their key, so probe chains stay intact)
        if (atomicAdd(&sl->cnt, 1u) == 0u) {
            atomicOr(&bits[key >> 5], 1u << (key & 31));
            ++n_new;
        }
        atomicAdd(&sl->sum[0], (unsigned long long)(qx & 0xFFFFF));
        atomicAdd(&sl->sum[1], (unsigned long long)(qy & 0xFFFFF));
        atomicAdd(&sl->sum[2], (unsigned long long)(qz & 0xFFFFF));
        ++n_in;
    }
    {
        unsigned long long* const dst[4] = {&ctr->points_in, &ctr->points_dropped, &ctr->points_lost, &ctr->occupied};
        const uint32_t v[4] = {n_in, n_drop, n_lost, n_new};
        block_add_counters<4>(dst, v);
    }
    if (n_lost) atomicOr(&ctr->flags, (uint32_t)VM_FLAG_HASH_FULL);
}

// ---- sorted insert path -------------------------------------------------------
// 1. voxelise every point: (key, point index) pairs plus its packed offsets;
//    points outside the grid get a key above every valid one.

// 3. after the sort by key: one lane per run of equal keys sums the run and
//    updates the voxel's slot once.  Every key occurs in one run only, so no
//    other lane touches that slot in this pass: the payload is a plain
//    read-modify-write; only claiming an empty slot needs a CAS.
// ---- grouped insert (large calls) ---------------------------------------------
// The points of a batch are voxelised, partitioned into hash buckets of about
// kBucketAvg points (a bucket is a range of home slots of the map's hash, so
// every point of a voxel lands in the same bucket), and each bucket is then
// aggregated by one workgroup in an LDS table: one slot update per distinct
// voxel, a plain read-modify-write since no other workgroup touches those
// voxels.
constexpr uint32_t kBucketTile = 4096;    // points per workgroup in the partition passes (at least)
constexpr int kPartBlock = 1024;          // partition workgroup: 16 waves, four points per thread per tile
constexpr uint32_t kBucketBlocks = 1024;  // partition workgroups per batch (at most)
constexpr uint32_t kBucketAvg = 512;      // target points per bucket
constexpr uint32_t kBucketMaxLog2 = 12;   // at most 4096 buckets (LDS counters)
constexpr uint32_t kBucketChunk = 1024;   // points aggregated per LDS table fill
constexpr uint32_t kBucketTableLog2 = 10;
constexpr uint32_t kBucketTable = 1u << kBucketTableLog2;   // LDS table slots: 20 KB, so eight workgroups
                                                             // fit on a CU; a bucket averages kBucketAvg
                                                             // points, so the table is about half full
static_assert(kBucketTile % kPartBlock == 0, "whole rows of points per partition workgroup");
static_assert(kBucketTable >= kBucketChunk, "a chunk's distinct keys always fit: every probe ends");
constexpr uint32_t kRecPerThread = kBucketChunk / kBlock;   // records per thread per fill
constexpr uint32_t kSlotPerThread = kBucketTable / kBlock;  // table entries per thread
static_assert(kRecPerThread * kBlock == kBucketChunk && kSlotPerThread * kBlock == kBucketTable, "whole rows per thread");

__device__ __forceinline__ uint32_t bucket_of(uint32_t key, uint32_t lb)
{
    // the top lb bits of the map's own slot hash
    return lb ? (key * 2654435769u) >> (32 - lb) : 0u;
}

__device__ __forceinline__ uint32_t table_slot(uint32_t key)
{
    // independent of the bucket bits: a different multiplier
    return (key * 0xCC9E2D51u) >> (32 - kBucketTableLog2);
}

__global__ void __launch_bounds__(kPartBlock) k_vox_bucket(const float* __restrict__ xyz, uint32_t n, Pose pose, Geom g,
                                                       uint32_t lb, uint32_t nblk, uint32_t tile, bool first_batch,
                                                       uint32_t* __restrict__ key_out,
                                                       unsigned long long* __restrict__ packed,
                                                       uint32_t* __restrict__ hist, DevCounters* __restrict__ ctr)
{
    __shared__ uint32_t cnt[1u << kBucketMaxLog2];
    const uint32_t B = 1u << lb;
    for (uint32_t b = threadIdx.x; b < B; b += kPartBlock) cnt[b] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && first_batch) ctr->touched = 0;
    __syncthreads();
    uint32_t n_in = 0, n_drop = 0;
    const double lim0 = (double)g.dims[0] * 1048576.0;
    const double lim1 = (double)g.dims[1] * 1048576.0;
    const double lim2 = (double)g.dims[2] * 1048576.0;
    const uint64_t base = (uint64_t)blockIdx.x * tile;
    for (uint32_t j = 0; j < tile / kPartBlock; ++j) {
        const uint64_t i = base + (uint64_t)j * kPartBlock + threadIdx.x;
        if (i >= n) break;
        const double px = (double)xyz[3 * (size_t)i + 0];
        const double py = (double)xyz[3 * (size_t)i + 1];
        const double pz = (double)xyz[3 * (size_t)i + 2];
        const double wx = fma(pose.R[2], pz, fma(pose.R[1], py, fma(pose.R[0], px, pose.t[0])));
        const double wy = fma(pose.R[5], pz, fma(pose.R[4], py, fma(pose.R[3], px, pose.t[1])));
        const double wz = fma(pose.R[8], pz, fma(pose.R[7], py, fma(pose.R[6], px, pose.t[2])));
        const double fx = floor((wx - g.origin[0]) * g.inv_q);
        const double fy = floor((wy - g.origin[1]) * g.inv_q);
        const double fz = floor((wz - g.origin[2]) * g.inv_q);
        uint32_t key = kEmpty;
        unsigned long long pk = 0;
        // negated range tests also reject NaN
        if (fx >= 0.0 && fx < lim0 && fy >= 0.0 && fy < lim1 && fz >= 0.0 && fz < lim2) {
            const int64_t qx = (int64_t)fx, qy = (int64_t)fy, qz = (int64_t)fz;
            key = (uint32_t)((uint64_t)(qx >> 20) +
                             (uint64_t)g.dims[0] * ((uint64_t)(qy >> 20) + (uint64_t)g.dims[1] * (uint64_t)(qz >> 20)));
            pk = (unsigned long long)(qx & 0xFFFFF) | ((unsigned long long)(qy & 0xFFFFF) << 20) |
                 ((unsigned long long)(qz & 0xFFFFF) << 40);
            atomicAdd(&cnt[bucket_of(key, lb)], 1u);
            ++n_in;
        } else {
            ++n_drop;
        }
        key_out[i] = key;
        packed[i] = pk;
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < B; b += kPartBlock) hist[(uint64_t)b * nblk + blockIdx.x] = cnt[b];
    unsigned long long* const dst[2] = {&ctr->points_in, &ctr->points_dropped};
    const uint32_t v[2] = {n_in, n_drop};
    block_add_counters<2, kPartBlock>(dst, v);
}

// Points to their buckets (hist holds the exclusive scan, bucket-major).
__global__ void __launch_bounds__(kPartBlock) k_bucket_scatter(const uint32_t* __restrict__ key_in,
                                                           const unsigned long long* __restrict__ packed, uint32_t n,
                                                           uint32_t lb, uint32_t nblk, uint32_t tile,
                                                           const uint32_t* __restrict__ hist,
                                                           uint4* __restrict__ rec_out)
{
    __shared__ uint32_t pos[1u << kBucketMaxLog2];
    const uint32_t B = 1u << lb;
    for (uint32_t b = threadIdx.x; b < B; b += kPartBlock) pos[b] = hist[(uint64_t)b * nblk + blockIdx.x];
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * tile;
    for (uint32_t j = 0; j < tile / kPartBlock; ++j) {
        const uint64_t i = base + (uint64_t)j * kPartBlock + threadIdx.x;
        if (i >= n) break;
        const uint32_t k = key_in[i];
        if (k == kEmpty) continue;
        const unsigned long long pk = packed[i];
        const uint32_t p = atomicAdd(&pos[bucket_of(k, lb)], 1u);
        rec_out[p] = make_uint4(k, (uint32_t)pk, (uint32_t)(pk >> 32), 0u);   // one 16-byte store
    }
}

// One workgroup per bucket: sum its points per voxel in LDS (at most
// kBucketChunk points per fill, so the 32-bit sums of 20-bit offsets cannot
// overflow), then update each voxel's slot once per fill.
__global__ void __launch_bounds__(kBlock) k_bucket_insert(const uint4* __restrict__ rec, uint32_t lb, uint32_t nblk,
                                                          const uint32_t* __restrict__ hist, Hash h,
                                                          uint32_t* __restrict__ bits, DevCounters* __restrict__ ctr)
{
    __shared__ uint32_t tkey[kBucketTable];
    __shared__ uint32_t tcnt[kBucketTable];
    __shared__ uint32_t tsum[3][kBucketTable];
    const uint32_t B = 1u << lb;
    const uint32_t total = ctr->sort_n;
    uint32_t n_lost = 0, n_new = 0, n_upd = 0;
    for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
        const uint32_t start = hist[(uint64_t)b * nblk];
        const uint32_t end = b + 1 < B ? hist[(uint64_t)(b + 1) * nblk] : total;
        for (uint32_t c0 = start; c0 < end; c0 += kBucketChunk) {
            const uint32_t c1 = min(end, c0 + kBucketChunk);
            for (uint32_t q = threadIdx.x; q < kBucketTable; q += kBlock) {
                tkey[q] = kEmpty;
                tcnt[q] = 0;
                tsum[0][q] = tsum[1][q] = tsum[2][q] = 0;
            }
            __syncthreads();
            // a chunk is kRecPerThread records per thread: all loaded before the
            // table inserts
            uint4 rr[kRecPerThread];
#pragma unroll
            for (uint32_t u = 0; u < kRecPerThread; ++u) {
                const uint32_t i = c0 + threadIdx.x + u * kBlock;
                if (i < c1) rr[u] = rec[i];
            }
#pragma unroll
            for (uint32_t u = 0; u < kRecPerThread; ++u) {
                if (c0 + threadIdx.x + u * kBlock >= c1) continue;
                const uint32_t k = rr[u].x;
                const unsigned long long pk = (unsigned long long)rr[u].y | ((unsigned long long)rr[u].z << 32);
                uint32_t q = table_slot(k);
                for (;;) {   // at most kBucketChunk keys in a table of kBucketTable slots: ends
                    const uint32_t old = atomicCAS(&tkey[q], kEmpty, k);
                    if (old == kEmpty || old == k) break;
                    q = (q + 1) & (kBucketTable - 1);
                }
                atomicAdd(&tcnt[q], 1u);
                atomicAdd(&tsum[0][q], (uint32_t)(pk & 0xFFFFF));
                atomicAdd(&tsum[1][q], (uint32_t)((pk >> 20) & 0xFFFFF));
                atomicAdd(&tsum[2][q], (uint32_t)((pk >> 40) & 0xFFFFF));
            }
            __syncthreads();
            // the thread's kSlotPerThread table entries: first probes (whole
            // 32-byte slots) issued together
            uint32_t tk[kSlotPerThread], sl[kSlotPerThread];
            uint4 sa[kSlotPerThread], sb[kSlotPerThread];
#pragma unroll
            for (uint32_t u = 0; u < kSlotPerThread; ++u) {
                tk[u] = tkey[threadIdx.x + u * kBlock];
                sl[u] = hash_slot(tk[u], h.log2cap);
                if (tk[u] != kEmpty) {
                    const uint4* sp = reinterpret_cast<const uint4*>(&h.slot[sl[u]]);
                    sa[u] = sp[0];
                    sb[u] = sp[1];
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < kSlotPerThread; ++u) {
                const uint32_t q = threadIdx.x + u * kBlock;
                const uint32_t k = tk[u];
                if (k == kEmpty) continue;
                ++n_upd;
                uint32_t s = sl[u];
                uint4 a = sa[u], b2 = sb[u];
                bool ok = a.x == k;
                if (!ok) {
                    for (uint32_t p = 0; p < kMaxProbe && p <= h.mask; ++p) {
                        if (p) a.x = h.slot[s].key;
                        if (a.x == k) { ok = true; break; }
                        if (a.x == kEmpty) {
                            const uint32_t old = atomicCAS(&h.slot[s].key, kEmpty, k);
                            if (old == kEmpty || old == k) { ok = true; break; }
                        }
                        s = (s + 1) & h.mask;
                    }
                    if (ok) {
                        // claimed or found past the first probe: the slot's
                        // counts as they stand now
                        const uint4* sp = reinterpret_cast<const uint4*>(&h.slot[s]);
                        a = sp[0];
                        b2 = sp[1];
                    }
                }
                if (!ok) {
                    n_lost += tcnt[q];
                    continue;
                }
                uint4* sp = reinterpret_cast<uint4*>(&h.slot[s]);
                const unsigned long long s0 = ((unsigned long long)a.w << 32 | a.z) + tsum[0][q];
                const unsigned long long s1 = ((unsigned long long)b2.y << 32 | b2.x) + tsum[1][q];
                const unsigned long long s2 = ((unsigned long long)b2.w << 32 | b2.z) + tsum[2][q];
                // the key is stored as claimed, not as loaded: a load served
                // from a line fetched before the claim would read it empty
                a.x = k;
                if (a.y == 0u) {   // new, or cleared since: occupied again
                    atomicOr(&bits[k >> 5], 1u << (k & 31));
                    ++n_new;
                }
                a.y += tcnt[q];
                a.z = (uint32_t)s0;
                a.w = (uint32_t)(s0 >> 32);
                b2 = make_uint4((uint32_t)s1, (uint32_t)(s1 >> 32), (uint32_t)s2, (uint32_t)(s2 >> 32));
                sp[0] = a;
                sp[1] = b2;
            }
            __syncthreads();
        }
    }
    {
        unsigned long long* const dst[3] = {&ctr->points_lost, &ctr->occupied, &ctr->touched};
        const uint32_t v[3] = {n_lost, n_new, n_upd};
        block_add_counters<3>(dst, v);
    }
    if (n_lost) {
        // points lost here were counted as inserted by the voxelise pass
        atomicAdd(&ctr->points_in, 0ull - (unsigned long long)n_lost);
        atomicOr(&ctr->flags, (uint32_t)VM_FLAG_HASH_FULL);
    }
}

// Occupied keys in rank order; the component-size counters of the ranks are
// cleared on the way (the labelling accumulates into them).  A workgroup
// takes kCompactWords consecutive grid words per pass: their keys (at most
// 32 per word) go to LDS at their ranks' offsets from the pass's first rank,
// then the workgroup stores them, and the cleared counters, as contiguous
// rows.
constexpr uint32_t kCompactWords = kBlock;

__global__ void __launch_bounds__(kBlock) k_compact(const uint32_t* __restrict__ bits, uint32_t nwords,
                                                    const uint32_t* __restrict__ wrank,
                                                    uint32_t* __restrict__ occ_key, uint32_t* __restrict__ csize)
{
    __shared__ uint32_t keys[kCompactWords * 32];
    __shared__ uint32_t s_base, s_end;
    for (uint32_t w0 = blockIdx.x * kCompactWords; w0 < nwords; w0 += gridDim.x * kCompactWords) {
        const uint32_t w = w0 + threadIdx.x;
        const uint32_t wl = (nwords - w0 < kCompactWords ? nwords : w0 + kCompactWords) - 1;   // last word
        uint32_t b = 0, r = 0;
        if (w < nwords) {
            b = bits[w];
            r = wrank[w];
        }
        if (w == w0) s_base = r;
        if (w == wl) s_end = r + (uint32_t)__popc(b);
        __syncthreads();
        const uint32_t base = s_base;
        for (uint32_t q = r - base; b; b &= b - 1, ++q) keys[q] = (w << 5) | (uint32_t)(__ffs(b) - 1);
        __syncthreads();
        const uint32_t n = s_end - base;   // at most 32 keys per word
        for (uint32_t i = threadIdx.x; i < n; i += kBlock) {
            occ_key[base + i] = keys[i];
            csize[base + i] = 0u;
        }
        __syncthreads();   // keys, s_base and s_end are reused by the next pass
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
    {
        unsigned long long* const dst[1] = {&ctr->occupied};
        const uint32_t v[1] = {n_new};
        block_add_counters<1>(dst, v);
    }
    if (n_lost) atomicOr(&ctr->flags, (uint32_t)VM_FLAG_HASH_FULL);
}

// ---- scrolling (the robot-centric map): a whole-voxel shift of the grid ------------
// 1. k_scroll_gather: every ranked voxel's slot content, with its key in the
//    shifted grid (kEmpty when it leaves), into staging arrays (32 bytes per
//    voxel: new key, count, the three sums as 32-bit halves);
// 2. the hash and the occupancy bits are emptied (fill kernels);
// 3. k_scroll_scatter: the staged voxels that stay are inserted under their
//    new keys.  Rebuilding the hash also drops the slots of cleared voxels.
struct ScrollStage {
    uint32_t* key;
    uint32_t* cnt;
    uint32_t* s[6];   // sum0 lo, hi, sum1 lo, hi, sum2 lo, hi
};

__global__ void __launch_bounds__(kBlock) k_scroll_gather(Geom g, Hash h, const DevCounters* __restrict__ ctr,
                                                          const uint32_t* __restrict__ occ_key, int32_t dx, int32_t dy,
                                                          int32_t dz, ScrollStage st)
{
    const uint32_t V = ctr->n_occ;
    const int64_t NX = g.dims[0], NY = g.dims[1], NZ = g.dims[2];
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t k = occ_key[r];
        const int64_t x = (int64_t)(k % (uint32_t)NX) - dx, y = (int64_t)((k / (uint32_t)NX) % (uint32_t)NY) - dy,
                      z = (int64_t)(k / ((uint32_t)NX * (uint32_t)NY)) - dz;
        const bool in = x >= 0 && y >= 0 && z >= 0 && x < NX && y < NY && z < NZ;
        const uint32_t s = hash_find(h, k);
        Slot sl{};
        if (s != kEmpty) sl = h.slot[s];
        st.key[r] = in && s != kEmpty ? (uint32_t)(x + NX * (y + NY * z)) : kEmpty;
        st.cnt[r] = sl.cnt;
        for (int a = 0; a < 3; ++a) {
            st.s[2 * a][r] = (uint32_t)sl.sum[a];
            st.s[2 * a + 1][r] = (uint32_t)(sl.sum[a] >> 32);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_fill_zero(uint32_t* __restrict__ p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// occupied restarts from zero (the scatter counts the voxels that stay); the
// voxels that leave are added to the scrolled-out counter
__global__ void k_scroll_counters(DevCounters* ctr)
{
    if (threadIdx.x == 0) ctr->occupied = 0ull;
}

__global__ void __launch_bounds__(kBlock) k_scroll_scatter(Hash h, uint32_t* __restrict__ bits, ScrollStage st,
                                                           DevCounters* ctr)
{
    uint32_t n_new = 0, n_out = 0, n_lost = 0;
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t k = st.key[r];
        if (k == kEmpty) {
            ++n_out;
            continue;
        }
        uint32_t s = hash_slot(k, h.log2cap);
        bool ok = false;
        for (uint32_t p = 0; p < kMaxProbe && p <= h.mask; ++p) {
            const uint32_t old = atomicCAS(&h.slot[s].key, kEmpty, k);
            if (old == kEmpty) { ok = true; break; }   // keys are distinct: never old == k
            s = (s + 1) & h.mask;
        }
        if (!ok) {
            ++n_lost;
            continue;
        }
        Slot* sl = &h.slot[s];
        sl->cnt = st.cnt[r];
        for (int a = 0; a < 3; ++a)
            sl->sum[a] = (unsigned long long)st.s[2 * a][r] | ((unsigned long long)st.s[2 * a + 1][r] << 32);
        atomicOr(&bits[k >> 5], 1u << (k & 31));
        ++n_new;
    }
    {
        unsigned long long* const dst[2] = {&ctr->occupied, &ctr->shifted_out};
        const uint32_t v[2] = {n_new, n_out};
        block_add_counters<2>(dst, v);
    }
    if (n_lost) atomicOr(&ctr->flags, (uint32_t)VM_FLAG_HASH_FULL);
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
        out->last_touched = c->touched;
        out->occupied = c->occupied;
        out->points_in = c->points_in;
        out->points_dropped = c->points_dropped;
        out->points_lost = c->points_lost;
        out->status_flags = c->flags;
        out->hash_capacity_log2 = log2cap;
        out->voxels_cleared = c->cleared;
        out->voxels_shifted_out = c->shifted_out;
    }
}

}  // namespace

hipError_t launch_stats(const DevCounters* ctr, uint32_t log2cap, vm_map_stats_t* out, hipStream_t s)
{
    k_stats<<<1, 64, 0, s>>>(ctr, log2cap, out);
    return hipGetLastError();
}

uint32_t bucket_log2(uint32_t m)
{
    uint32_t lb = 0;
    while (lb < kBucketMaxLog2 && ((uint64_t)kBucketAvg << lb) < m) ++lb;
    return lb;
}

// points per partition workgroup: kBucketTile, or more so that a batch takes
// at most kBucketBlocks workgroups (bounds the histogram)
static uint32_t bucket_tile(uint32_t m)
{
    uint32_t t = kBucketTile;
    while ((uint64_t)t * kBucketBlocks < m) t <<= 1;
    return t;
}

size_t bucket_hist_words(uint32_t batch)
{
    const uint32_t tile = bucket_tile(batch);
    const uint32_t nblk = (batch + tile - 1) / tile;
    return ((size_t)nblk << bucket_log2(batch)) + 64;
}

hipError_t launch_insert(const float* xyz, int64_t n, const Pose& pose, const Geom& g, const Hash& h,
                         uint32_t* bits, DevCounters* ctr, const InsertScratch& sc, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n < kSortedInsertMin || sc.cap == 0) {
        k_insert<<<grid_for((uint64_t)n, kBlock, kMapGrid), kBlock, 0, s>>>(xyz, n, pose, g, h, bits, ctr);
        return hipGetLastError();
    }
    for (int64_t done = 0; done < n; done += sc.cap) {
        const uint32_t m = (uint32_t)((n - done) < (int64_t)sc.cap ? (n - done) : (int64_t)sc.cap);
        // the batch size is known here, so grids and the bucket count follow it
        const uint32_t lb = bucket_log2(m);
        const uint32_t tile = bucket_tile(m);
        const uint32_t nblk = (m + tile - 1) / tile;
        k_vox_bucket<<<nblk, kPartBlock, 0, s>>>(xyz + 3 * done, m, pose, g, lb, nblk, tile, done == 0, sc.key,
                                            sc.packed, sc.hist, ctr);
        hipError_t e = scan_exclusive_dev(sc.hist, sc.hist, nullptr, (nblk << lb), &ctr->sort_n, sc.blk, s);
        if (e != hipSuccess) return e;
        k_bucket_scatter<<<nblk, kPartBlock, 0, s>>>(sc.key, sc.packed, m, lb, nblk, tile, sc.hist, sc.rec);
        k_bucket_insert<<<1u << lb, kBlock, 0, s>>>(sc.rec, lb, nblk, sc.hist, h, bits, ctr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

namespace {
// the occupancy index's scan: the popcount of each word is taken as the
// scan reads it, and the exclusive prefixes are the word ranks
struct RankF {
    const uint32_t* bits;
    __device__ Vec<1> operator()(uint32_t w) const
    {
        Vec<1> x;
        x.v[0] = (uint32_t)__popc(bits[w]);
        return x;
    }
};

struct RankG {
    uint32_t* wrank;
    DevCounters* ctr;
    __device__ void operator()(uint32_t w, const Vec<1>&, const Vec<1>& pre) const { wrank[w] = pre.v[0]; }
    __device__ void total(const Vec<1>& t) const { ctr->n_occ = t.v[0]; }
};
}   // namespace

hipError_t launch_rank(const Geom& g, const uint32_t* bits, SegBuffers& b, uint32_t /*cap*/, DevCounters* ctr,
                       hipStream_t s)
{
    tile_scan<1>(RankF{bits}, RankG{b.wrank, ctr}, nullptr, g.nwords, reinterpret_cast<Vec<1>*>(b.blk), s);
    k_compact<<<grid_for(g.nwords), kBlock, 0, s>>>(bits, g.nwords, b.wrank, b.occ_key, b.csize);
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

hipError_t launch_scroll(const Geom& g, const Hash& h, uint32_t* bits, SegBuffers& b, uint32_t cap, int32_t dx,
                         int32_t dy, int32_t dz, DevCounters* ctr, hipStream_t s)
{
    // staging in segmentation buffers that are free between frames
    ScrollStage st;
    st.key = b.parent;
    st.cnt = b.csize;
    st.s[0] = b.scan_a;
    st.s[1] = b.scan_b;
    st.s[2] = b.sort_k[0];
    st.s[3] = b.sort_k[1];
    st.s[4] = b.sort_v[0];
    st.s[5] = b.sort_v[1];
    k_scroll_gather<<<grid_for(cap), kBlock, 0, s>>>(g, h, ctr, b.occ_key, dx, dy, dz, st);
    const uint32_t hcap = h.mask + 1;
    k_clear_slots<<<grid_for(hcap, kBlock, 16384), kBlock, 0, s>>>(h.slot, hcap);
    k_fill_zero<<<grid_for(g.nwords), kBlock, 0, s>>>(bits, g.nwords);
    k_scroll_counters<<<1, kWave, 0, s>>>(ctr);
    k_scroll_scatter<<<grid_for(cap, kBlock, kMapGrid), kBlock, 0, s>>>(h, bits, st, ctr);
    return hipGetLastError();
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
    k_import<<<grid_for(n, kBlock, kMapGrid), kBlock, 0, s>>>(g, h, bits, ctr, key, cnt, sum, n);
    return hipGetLastError();
}

}  // namespace vm

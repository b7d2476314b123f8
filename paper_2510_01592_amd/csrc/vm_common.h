// vm_common.h -- internal declarations shared by the library's HIP translation
// units (gfx950 only).  Not part of the ABI; the ABI is include/vm.h.
#pragma once
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/vm.h"

namespace vm {

constexpr uint32_t kEmpty = 0xFFFFFFFFu;   // empty hash slot / "no key"
constexpr int kBlock = 256;                 // default workgroup: 4 wave64
constexpr int kWave = 64;
constexpr uint32_t kMaxProbe = 8192;        // linear-probe limit of the voxel hash

// Device-side counters of one map (one 128-byte line).
struct DevCounters {
    unsigned long long points_in;
    unsigned long long points_dropped;
    unsigned long long points_lost;
    unsigned long long occupied;      // voxels in the hash
    uint32_t flags;                   // VM_FLAG_*
    uint32_t n_occ;                   // occupied voxels ranked by the last rank pass
    uint32_t meta[2];                 // clusters view: [0] K, [1] total points
    uint32_t kmax;                    // largest cluster id (K - 1, or 0)
    uint32_t sort_n;                  // points in the current sorted insert batch
    uint32_t sort_max;                // largest sort key of that batch (2^bits - 1)
    unsigned long long touched;       // distinct voxels updated by the last insert call
    uint32_t sort_sel;                // buffer (0/1) holding the sorted insert batch
    uint32_t group_sel;               // buffer (0/1) holding the voxels sorted by cluster
    unsigned long long cleared;       // voxels cleared by ray casting since create/clear
    unsigned long long shifted_out;   // voxels dropped by grid shifts since create/clear
    uint32_t pad[5];
};

struct Geom {
    double origin[3];
    double voxel_size;
    double inv_q;          // 2^20 / voxel_size
    int32_t dims[3];
    uint32_t nwords;       // occupancy words (32 cells each)
};

struct Pose {
    double R[9];
    double t[3];
};

// One voxel of the hash: key, point count and the three fixed-point offset
// sums in one 32-byte slot, so a point's probe and its four atomics hit one
// memory sector.
struct __align__(32) Slot {
    uint32_t key;
    uint32_t cnt;
    unsigned long long sum[3];
};

// Open-addressing hash over voxel keys with linear probing.
struct Hash {
    Slot* slot;               // [cap]
    uint32_t log2cap;
    uint32_t mask;
};

__device__ __forceinline__ uint32_t hash_slot(uint32_t key, uint32_t log2cap)
{
    // Fibonacci hashing: spreads neighbouring voxel keys over the table.
    return (uint32_t)((key * 2654435769u) >> (32 - log2cap));
}

// Slot holding `key`, or kEmpty if absent.
__device__ __forceinline__ uint32_t hash_find(const Hash& h, uint32_t key)
{
    uint32_t s = hash_slot(key, h.log2cap);
    for (uint32_t p = 0; p < kMaxProbe && p <= h.mask; ++p) {
        const uint32_t k = h.slot[s].key;
        if (k == key) return s;
        if (k == kEmpty) return kEmpty;
        s = (s + 1) & h.mask;
    }
    return kEmpty;
}

// Eq. (1) closed form for one axis: the voxel's mean position from its
// integer offset sum (units of s*2^-20) and point count.
__device__ __forceinline__ float voxel_mean_axis(uint32_t idx, unsigned long long sum, uint32_t cnt, double s,
                                                 double o)
{
    const unsigned long long mq = sum / (unsigned long long)cnt;
    const double cell = (double)idx + (double)mq * 0x1p-20;
    return (float)fma(cell, s, o);
}

// Per-map workspace for the segmentation buffers (indexed by occupied rank
// or by cluster-CSR position; all sized by the hash capacity).
struct SegBuffers {
    uint32_t* occ_key;     // [cap] occupied keys, ascending
    uint32_t* parent;      // [cap] union-find parent (rank indices)
    uint32_t* csize;       // [cap] component size at its root
    uint32_t* scan_a;      // [cap] scan scratch
    uint32_t* scan_b;      // [cap]
    uint32_t* sort_k[2];   // [cap] radix keys (cluster id), ping-pong
    uint32_t* sort_v[2];   // [cap] radix values (voxel key), ping-pong
    uint32_t* cl_off;      // [cap+1]
    uint32_t* cl_tag;      // [cap]
    uint32_t* cl_key;      // [cap]
    float* cl_x;           // [cap]
    float* cl_y;
    float* cl_z;
    uint32_t* wrank;       // [nwords+1] exclusive popcount prefix of the occupancy words
    uint32_t* blk;         // block partials for scans (sized generously)
    uint32_t* hist;        // radix histograms
    uint64_t* pairs;       // [ccl_tiles * kCclTilePairs] cross-tile hook pairs, per tile
    uint32_t* npair;       // [ccl_tiles] pairs stored per tile
};

constexpr uint32_t kCclTilePairs = 256;   // cross-tile hook pairs buffered per labelling tile
uint64_t ccl_tiles(const Geom& g);        // labelling tiles covering the grid

// Number of clusters a pass may process: min(meta[0], k_cap) if the offsets
// are a valid CSR (off[0] = 0, non-decreasing, off[K] = meta[1] <= n_cap),
// else 0 with VM_FLAG_BAD_CLUSTERS raised.  Run by one workgroup.
__device__ __forceinline__ uint32_t validate_clusters(const uint32_t* meta, const uint32_t* off, uint32_t k_cap,
                                                      uint32_t n_cap, uint32_t* status, int* bad_lds)
{
    const uint32_t K = min(meta[0], k_cap);
    if (threadIdx.x == 0) *bad_lds = (off[0] != 0u) || (off[K] > n_cap) || (meta[0] <= k_cap && off[K] != meta[1]);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < K; k += blockDim.x)
        if (off[k] > off[k + 1]) *bad_lds = 1;
    __syncthreads();
    const bool bad = *bad_lds != 0;
    if (bad && threadIdx.x == 0) atomicOr(status, (uint32_t)VM_FLAG_BAD_CLUSTERS);
    return bad ? 0u : K;
}

// Add per-thread counts into global 64-bit counters with one atomic per block
// and counter (zero totals skipped).  Every thread of the block must call it.
template <int N, int T = kBlock>
__device__ __forceinline__ void block_add_counters(unsigned long long* const (&dst)[N], const uint32_t (&v)[N])
{
    __shared__ unsigned long long part[N][T / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        unsigned long long s = v[c];
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) s += __shfl_xor(s, d, kWave);
        if (lane == 0) part[c][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += part[threadIdx.x][w];
        if (t) atomicAdd(dst[threadIdx.x], t);
    }
}

// Exclusive scan over elements [0, n) of N counters each by one workgroup of
// T threads (every thread calls it): chunks of T*I elements, I consecutive
// ones per thread, with the running totals carried from chunk to chunk.
// get(i, v) fills element i's counters, put(i, excl) receives its exclusive
// prefix; the totals are returned in `total` (on every thread).  Used where
// the element count is a per-cluster count, so that the counts, the scan and
// what consumes the totals take one launch instead of three.
constexpr int kOneBlockThreads = 1024;
constexpr uint32_t kOneBlockMax = 65536;   // capacities up to this use the one-workgroup form

template <int T, int I, int N, class Get, class Put>
__device__ __forceinline__ void one_block_scan(uint32_t n, Get get, Put put, uint32_t (&total)[N])
{
    __shared__ uint32_t wsum[N][T / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t carry[N];
#pragma unroll
    for (int c = 0; c < N; ++c) carry[c] = 0;
    for (uint32_t c0 = 0; c0 < n; c0 += (uint32_t)(T * I)) {
        const uint32_t mine = c0 + threadIdx.x * I;
        uint32_t v[I][N], sum[N], inc[N];
#pragma unroll
        for (int c = 0; c < N; ++c) sum[c] = 0;
#pragma unroll
        for (int j = 0; j < I; ++j) {
            if (mine + j < n) {
                get(mine + j, v[j]);
            } else {
#pragma unroll
                for (int c = 0; c < N; ++c) v[j][c] = 0;
            }
#pragma unroll
            for (int c = 0; c < N; ++c) sum[c] += v[j][c];
        }
#pragma unroll
        for (int c = 0; c < N; ++c) {
            uint32_t x = sum[c];
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t o = __shfl_up(x, d, kWave);
                if (lane >= d) x += o;
            }
            inc[c] = x;
            if (lane == kWave - 1) wsum[c][wave] = x;
        }
        __syncthreads();
        uint32_t run[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
            uint32_t before = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < T / kWave; ++w) {
                const uint32_t t = wsum[c][w];
                before += (w < wave) ? t : 0u;
                tot += t;
            }
            run[c] = carry[c] + before + inc[c] - sum[c];
            carry[c] += tot;
        }
        __syncthreads();   // wsum is rewritten by the next chunk
#pragma unroll
        for (int j = 0; j < I; ++j) {
            if (mine + j < n) put(mine + j, run);
#pragma unroll
            for (int c = 0; c < N; ++c) run[c] += v[j][c];
        }
    }
#pragma unroll
    for (int c = 0; c < N; ++c) total[c] = carry[c];
}

// ---- host-side error plumbing ------------------------------------------
#define VM_HIP(call)                                                    \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return VM_E_DEVICE;                       \
    } while (0)

// ---- stage timing (vm_timing.cpp) --------------------------------------
struct StageScope {
    StageScope(int stage, hipStream_t s);
    ~StageScope();
    int stage_;
    hipStream_t s_;
    void* ev0_;
    void* ev1_;
};

// ---- launch helpers ----------------------------------------------------
inline int grid_for(uint64_t n, int block = kBlock, int max_grid = 8192)
{
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (uint64_t)max_grid) g = max_grid;
    return (int)g;
}

// ---- scans and sorts (vm_scan.hip) ----------------------------------------
// Exclusive prefix sum of n u32 values (n read from *d_n on the device, at
// most n_cap; or n = n_cap when d_n is null), in place allowed (in == out).  Writes the total to *d_total if
// non-null.  `blk` needs scan_blk_words(n_cap) words.
size_t scan_blk_words(uint64_t n_cap);
hipError_t scan_exclusive_dev(const uint32_t* in, uint32_t* out, const uint32_t* d_n, uint32_t n_cap,
                              uint32_t* d_total, uint32_t* blk, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low `bits` bits of key;
// n from *d_n (<= n_cap).  Every key is at most *d_max_key; a pass whose
// digit and all higher digits of that bound are zero does nothing (the
// passes that run are the first ones).  The result lands in keys[r]/vals[r] with r = *d_sel, written on
// the device.  `hist` needs radix_hist_words(n_cap) words, `blk` as for the
// scan.
size_t radix_hist_words(uint64_t n_cap);
hipError_t radix_sort_pairs_dev(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* d_n, uint32_t n_cap,
                                int bits, const uint32_t* d_max_key, uint32_t* hist, uint32_t* blk,
                                uint32_t* d_sel, hipStream_t s);

// Scratch of the grouped insert path (sized for `cap` points per batch).
struct InsertScratch {
    uint32_t* key;                // [cap] voxel key of each point (kEmpty if dropped)
    unsigned long long* packed;   // [cap] fixed-point offsets of each point, 20 bits per axis
    uint4* rec;                   // [cap] (key, offsets) records grouped by bucket
    uint32_t* hist;               // bucket histograms, bucket-major
    uint32_t* blk;
    uint32_t cap;
};

// ---- map stages (vm_map.hip) ------------------------------------------------
constexpr int64_t kSortedInsertMin = 1 << 17;   // smaller calls use per-point atomics
uint32_t bucket_log2(uint32_t batch_points);    // log2 of the bucket count of a grouped batch
size_t bucket_hist_words(uint32_t batch);       // histogram words of the largest batch
hipError_t launch_insert(const float* xyz, int64_t n, const Pose& pose, const Geom& g, const Hash& h,
                         uint32_t* bits, DevCounters* ctr, const InsertScratch& sc, hipStream_t s);
hipError_t launch_stats(const DevCounters* ctr, uint32_t log2cap, vm_map_stats_t* out, hipStream_t s);
hipError_t launch_rank(const Geom& g, const uint32_t* bits, SegBuffers& b, uint32_t cap,
                       DevCounters* ctr, hipStream_t s);
hipError_t launch_clear(const Geom& g, const Hash& h, uint32_t* bits, DevCounters* ctr, hipStream_t s);
// the map's content shifted by whole voxels (after launch_rank; uses the
// segmentation buffers as staging)
hipError_t launch_scroll(const Geom& g, const Hash& h, uint32_t* bits, SegBuffers& b, uint32_t cap, int32_t dx,
                         int32_t dy, int32_t dz, DevCounters* ctr, hipStream_t s);
hipError_t launch_export(const Geom& g, const Hash& h, const SegBuffers& b, const DevCounters* ctr,
                         uint32_t* key, uint32_t* cnt, unsigned long long* sum, float* mean, uint64_t cap,
                         hipStream_t s);
hipError_t launch_import(const Geom& g, const Hash& h, uint32_t* bits, DevCounters* ctr, const uint32_t* key,
                         const uint32_t* cnt, const unsigned long long* sum, uint64_t n, hipStream_t s);

// ---- CCL and grouping (vm_ccl.hip) --------------------------------------------
hipError_t launch_ccl(const Geom& g, const uint32_t* bits, SegBuffers& b, uint32_t cap, DevCounters* ctr,
                      hipStream_t s);
hipError_t launch_group(const Geom& g, const Hash& h, SegBuffers& b, uint32_t cap, uint32_t min_cluster,
                        uint32_t* d_labels, DevCounters* ctr, hipStream_t s);

// ---- steppable classification and gated clustering (vm_step.hip) -------------
struct StepBuffers {
    float4* mean;      // [cap] Eq. (1) mean of each occupied voxel, by rank
    float4* normal;    // [cap] Eq. (3) normal (xyz, pad)
    uint8_t* step;     // [cap] Eq. (4) steppability
};
// classification of every ranked voxel, then the gated union-find and the
// component sizes of steppable roots in b.parent / b.csize (ready for launch_group)
hipError_t launch_steppable(const Geom& g, const Hash& h, const uint32_t* bits, SegBuffers& b, uint32_t cap,
                            const StepBuffers& sb, uint32_t radius, uint32_t n_th, double cos_th, double d_th,
                            float* d_normal, uint8_t* d_steppable, DevCounters* ctr, hipStream_t s);
hipError_t launch_step_labels(const SegBuffers& b, const StepBuffers& sb, uint32_t cap, DevCounters* ctr,
                              uint32_t* d_labels, hipStream_t s);

// ---- label propagation (vm_propagate.hip) ------------------------------------
constexpr uint32_t kLpBatchMax = 32;   // sweeps enqueued between two host checks
hipError_t launch_lp_init(const SegBuffers& b, uint32_t cap, uint32_t* label, DevCounters* ctr, hipStream_t s);
// `sweeps` (<= kLpBatchMax) sweeps; sweep i ORs 1 into changed[i] when it lowered a label
hipError_t launch_lp_sweeps(const Geom& g, const uint32_t* bits, const SegBuffers& b, uint32_t cap, uint32_t* label,
                            uint32_t* changed, uint32_t sweeps, DevCounters* ctr, hipStream_t s);
hipError_t launch_lp_finish(const uint32_t* bits, SegBuffers& b, uint32_t cap, const uint32_t* label,
                            DevCounters* ctr, hipStream_t s);

// ---- ray casting and clearing (vm_clear.hip) ---------------------------------
// Eq. (2) for one frame: cast every point's ray from the sensor's voxel,
// then free the occupied cells on a ray that hold none of the frame's points.
// ray and keep are zero on entry (nwords words each) and zero again on exit.
hipError_t launch_clear_rays(const float* xyz, int64_t n, const Pose& pose, const Geom& g, const int32_t sensor[3],
                             const Hash& h, uint32_t* bits, uint32_t* ray, uint32_t* keep, DevCounters* ctr,
                             hipStream_t s);

// ---- RANSAC and hulls (vm_ransac.hip, vm_hull.hip) --------------------------
constexpr int kHullDirs = 8;   // support directions of the hull pre-filter

struct WorkLayout {
    uint32_t k_cap;         // clusters the layout was made for
    int32_t* counts;        // [k_cap * H]
    float4* hyp;            // [k_cap * H]
    uint32_t* tile_off;     // [k_cap + 1]
    uint32_t* tile_k;       // [n_cap / tile + k_cap + 1] cluster of each point tile
    uint32_t* tile_off_big;  // the same for the clusters beyond one wave's points
    uint32_t* tile_k_big;
    uint32_t* flags;        // [n_cap + 1] inliers per point tile, then their prefixes
    uint32_t* blk;          // scan partials
    uint32_t* hull_cnt;     // [k_cap + 2]
    uint32_t* hull_off;     // [k_cap + 2]
    uint32_t* hull_tmp;     // [n_cap + k_cap + 2]
    double* hull_u;         // [n_cap]
    double* hull_v;         // [n_cap]
    uint32_t* hull_i;       // [n_cap]
    uint32_t* hull_tile_off;  // [k_cap + 2]
    double* ext_v;          // [hull tiles * kHullDirs]
    uint32_t* ext_i;        // [hull tiles * kHullDirs]
    double* poly;           // [k_cap * (2 kHullDirs + 2)]
    uint32_t* surv_cnt;     // [k_cap]
    uint32_t* chain_list;   // [k_cap] clusters for the workgroup hull chain (count in small[7])
    uint32_t* small;        // [64] device scalars: K, tiles, inliers, large-cluster tiles, K (hull), vertices,
                            // hull tiles, chain-list length
    size_t bytes;
};
WorkLayout work_layout(void* base, uint32_t k_cap, uint32_t n_cap, uint32_t n_hyp);
uint64_t hull_tiles_bound(uint32_t k_cap, uint32_t n_cap);

// d_cframe: optional per-cluster RNG frame word (merged cluster sets); when
// null every cluster uses p.d_frame / p.frame
vm_status ransac_planes(const vm_clusters& cl, const vm_ransac_params& p, const vm_planes& out,
                        const WorkLayout& w, hipStream_t s, const uint32_t* d_cframe = nullptr);
// the process-wide counting decomposition (vm_count_config)
bool count_config_valid(const vm_count_config& c);
vm_count_config count_config_default();
vm_count_config count_config_get();
void count_config_set(const vm_count_config& c);
vm_status hulls(const vm_clusters& cl, const vm_planes& planes, const vm_hulls_out& out, const WorkLayout& w,
                hipStream_t s);
// the workgroup chain over listed clusters (count in small[7]) whose survivors
// sit at gu/gv/gi[in_off[k] + s]; vertices to hull_tmp[in_off[k] + k + q]
hipError_t launch_hull_chain_list(const uint32_t* small, const uint32_t* list, const uint32_t* in_off,
                                  const uint32_t* in_idx, const uint32_t* surv_cnt, double* gu, double* gv, uint32_t* gi,
                                  uint32_t* hull_cnt, uint32_t* hull_tmp, double* area_out, uint32_t grid, hipStream_t s);

// ---- RANSAC and polygons in one persistent launch (vm_fused.hip) ---------------
bool fused_config_valid(const vm_fused_config& c);
vm_fused_config fused_config_default();
vm_fused_config fused_config_get();
void fused_config_set(const vm_fused_config& c);
void fused_cache_put(uint32_t k_cap, uint32_t n_cap, uint32_t H, const vm_fused_config& c);
bool fused_cache_get(uint32_t k_cap, uint32_t n_cap, uint32_t H, vm_fused_config* c);
void fused_cache_clear();
size_t fused_workspace_bytes(uint32_t k_cap, uint32_t n_cap, uint32_t H);
// d_cframe: optional per-cluster frame numbers (else params' frame)
vm_status planes_and_hulls(const vm_clusters& cl, const vm_ransac_params& p, const uint32_t* d_cframe,
                           const vm_planes& planes, const vm_hulls_out& hulls, void* d_work, size_t work_bytes,
                           const vm_fused_config& cfg, hipStream_t s);
// ---- several cluster sets merged into one two-pass sequence (vm_multi.hip) -----
size_t multi_workspace_bytes(uint32_t k_cap, uint32_t n_cap, uint32_t H);
vm_status planes_hulls_multi(uint32_t n, const vm_clusters* sets, const uint32_t* frames, const vm_ransac_params& p,
                             const vm_planes* planes, const vm_hulls_out* hulls, uint32_t k_cap, uint32_t n_cap,
                             void* d_work, size_t work_bytes, hipStream_t s);

}  // namespace vm

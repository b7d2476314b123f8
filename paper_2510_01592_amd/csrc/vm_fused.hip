// vm_fused.hip -- RANSAC planes and boundary polygons of a whole cluster set
// in one persistent launch (Sec. III-C "Multi-plane estimation" (a)-(c) and
// "Boundary polygon generation", run cluster-parallel as in the paper's
// pipeline, with thousands of clusters of very uneven size).
//
// A one-workgroup preparation sorts the clusters by cost (point count,
// largest first) and lays out a device work queue of items:
//   * a cluster of at most small_max points is one item per chunk of its
//     hypotheses: the lanes take the planes and loop over the points (LDS);
//   * a larger cluster is one item per (4096-point tile, hypothesis chunk):
//     each lane keeps 16 points in registers, the chunk's planes come from LDS.
// Every hypothesis plane of the set is drawn and fitted by a grid-wide pass
// first (fp64 arithmetic and the Philox stream stay out of the persistent
// kernel's registers).  The persistent workgroups take items from the queue
// with one atomic each (no workgroup ever waits for another) and store each
// item's integer counts in its own slot, so the sums do not depend on the
// order.  Every item adds one to its cluster's completion counter; the
// workgroup that completes a cluster runs (c) for it -- the best
// hypothesis, its inlier list -- and the polygon: projection, the
// extreme-point filter, and the sort and monotone chain of up to 64
// survivors in one wave's registers; larger survivor sets are listed for one
// tail launch (the workgroup chain in LDS stays out of the persistent
// kernel, whose register and LDS budget sets how many of its workgroups
// share a compute unit).  A scan and a copy then pack
// the per-cluster lists into the caller's compact CSR outputs.  Results are
// bit-identical to vm_ransac_planes followed by vm_hulls.
#include "vm_common.h"
#include "vm_dev.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include <math.h>

namespace vm {
namespace {

using namespace dev;

constexpr int kFBlock = 256;                         // threads of every fused kernel
constexpr int kFRows = 16;                           // points per lane in a tile item
constexpr uint32_t kFTile = kFBlock * kFRows;        // 4096 points per tile item
constexpr uint32_t kFMaxChunk = 512;                 // hypotheses per item (LDS planes)
constexpr uint32_t kFSmallMax = 256;                 // clusters whose lanes take the planes
constexpr int kFWaves = kFBlock / kWave;
constexpr int kBuckets = 33;                         // cost classes: floor(log2(points)) + 1

struct FusedWork {
    int32_t* part;          // [tiles][H] per-tile partial counts
    float4* hyp;            // [k_cap][H] hypothesis planes
    uint32_t* order;        // [k_cap] clusters by cost, largest first
    uint32_t* item_off;     // [k_cap + 1] first queue item of order[i]
    uint32_t* tbase;        // [k_cap] first partial-count row of cluster k
    uint32_t* done;         // [k_cap] finished items of cluster k
    uint32_t* nin;          // [k_cap] inliers of cluster k
    uint32_t* hcnt;         // [k_cap] polygon vertices of cluster k
    uint32_t* surv;         // [k_cap] survivors of the filter (tail clusters)
    uint32_t* slot_in;      // [n_cap] cluster k's inliers at off[k] + j
    uint32_t* slot_hull;    // [n_cap + k_cap + 1] cluster k's vertices at off[k] + k + q
    double* su;             // [n_cap] survivors of cluster k at off[k] + s
    double* sv;
    uint32_t* si;
    uint32_t* tail;         // [k_cap] clusters for the tail chain (count in small[7])
    uint32_t* small;        // [64]: 0 K, 1 queue items, 2 queue head, 3 tile rows, 4 K, 5 vertices, 7 tail
    size_t bytes;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

FusedWork fused_layout(void* base, uint32_t k_cap, uint32_t n_cap, uint32_t H)
{
    FusedWork w{};
    char* p = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* r = p ? p + o : nullptr;
        o += align256(bytes);
        return r;
    };
    const size_t rows = (size_t)n_cap / kFTile + (size_t)k_cap + 1;
    w.part = (int32_t*)take(rows * H * sizeof(int32_t));
    w.hyp = (float4*)take((size_t)k_cap * H * sizeof(float4));
    w.order = (uint32_t*)take(((size_t)k_cap + 1) * 4);
    w.item_off = (uint32_t*)take(((size_t)k_cap + 1) * 4);
    w.tbase = (uint32_t*)take(((size_t)k_cap + 1) * 4);
    w.done = (uint32_t*)take(((size_t)k_cap + 1) * 4);
    w.nin = (uint32_t*)take(((size_t)k_cap + 1) * 4);
    w.hcnt = (uint32_t*)take(((size_t)k_cap + 1) * 4);
    w.surv = (uint32_t*)take(((size_t)k_cap + 1) * 4);
    w.slot_in = (uint32_t*)take(((size_t)n_cap + 1) * 4);
    w.slot_hull = (uint32_t*)take(((size_t)n_cap + k_cap + 2) * 4);
    w.su = (double*)take(((size_t)n_cap + 1) * 8);
    w.sv = (double*)take(((size_t)n_cap + 1) * 8);
    w.si = (uint32_t*)take(((size_t)n_cap + 1) * 4);
    w.tail = (uint32_t*)take(((size_t)k_cap + 1) * 4);
    w.small = (uint32_t*)take(64 * 4);
    w.bytes = o;
    return w;
}

// the work split of the fused pass (vm_fused_config)
struct Split {
    uint32_t H, chunk, nch, small_max;
};

__device__ __forceinline__ bool is_small(uint32_t n, const Split& s) { return n <= s.small_max; }

__device__ __forceinline__ uint32_t tiles_of(uint32_t n) { return n > kFTile ? (n + kFTile - 1) / kFTile : 1u; }

// queue items of a cluster of n points (at least one, so every cluster is finished)
__device__ __forceinline__ uint32_t items_of(uint32_t n, const Split& s)
{
    return is_small(n, s) ? s.nch : tiles_of(n) * s.nch;
}

// ---- preparation: validate, cost order, queue layout (one workgroup) ------------
__global__ void __launch_bounds__(kOneBlockThreads) k_fused_prepare(const uint32_t* __restrict__ meta, uint32_t k_cap,
                                                                    uint32_t out_k_cap, uint32_t n_cap,
                                                                    const uint32_t* __restrict__ off, Split sp,
                                                                    FusedWork w, uint32_t* __restrict__ status)
{
    __shared__ int bad;
    __shared__ uint32_t bucket[kBuckets + 1];
    const uint32_t K = validate_clusters(meta, off, k_cap, n_cap, status, &bad);
    for (int b = threadIdx.x; b <= kBuckets; b += blockDim.x) bucket[b] = 0;
    __syncthreads();
    // cost class of each cluster (largest first), counted per class
    auto cls = [&](uint32_t n) -> uint32_t { return n ? (uint32_t)(kBuckets - 1 - (31 - __clz(n))) : (uint32_t)kBuckets - 1; };
    for (uint32_t k = threadIdx.x; k < K; k += blockDim.x) atomicAdd(&bucket[cls(off[k + 1] - off[k]) + 1], 1u);
    __syncthreads();
    if (threadIdx.x == 0)
        for (int b = 1; b <= kBuckets; ++b) bucket[b] += bucket[b - 1];   // class starts
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < K; k += blockDim.x) w.order[atomicAdd(&bucket[cls(off[k + 1] - off[k])], 1u)] = k;
    // per-cluster state
    for (uint32_t k = threadIdx.x; k < K; k += blockDim.x) {
        w.done[k] = 0;
        w.nin[k] = 0;
        w.hcnt[k] = 0;
    }
    __syncthreads();
    // queue offsets in cost order, partial-count rows in cluster order
    uint32_t tot[1];
    one_block_scan<kOneBlockThreads, 4, 1>(
        K, [&](uint32_t i, uint32_t(&v)[1]) { v[0] = items_of(off[w.order[i] + 1] - off[w.order[i]], sp); },
        [&](uint32_t i, const uint32_t(&e)[1]) { w.item_off[i] = e[0]; }, tot);
    __syncthreads();
    uint32_t rows[1];
    one_block_scan<kOneBlockThreads, 4, 1>(
        K,
        [&](uint32_t k, uint32_t(&v)[1]) {
            const uint32_t n = off[k + 1] - off[k];
            v[0] = is_small(n, sp) ? 1u : tiles_of(n);
        },
        [&](uint32_t k, const uint32_t(&e)[1]) { w.tbase[k] = e[0]; }, rows);
    if (threadIdx.x == 0) {
        w.small[0] = K;
        w.small[1] = tot[0];
        w.small[2] = 0;
        w.small[3] = rows[0];
        w.small[4] = K;
        w.small[7] = 0;
        w.item_off[K] = tot[0];
        if (meta[0] > out_k_cap) atomicOr(status, (uint32_t)VM_FLAG_CLUSTERS_CAP);
    }
}

// ---- the persistent kernel --------------------------------------------------------
struct FusedArgs {
    const uint32_t* off;
    const float* X;
    const float* Y;
    const float* Z;
    const uint32_t* tag;
    const uint32_t* cframe;   // optional per-cluster frame number
    const uint32_t* d_frame;  // optional device frame number
    uint32_t frame;
    float eps;
    uint64_t seed;
    Split sp;
    FusedWork w;
    float4* plane_out;
    int32_t* best_out;
    int32_t* nin_out;
    int32_t* counts_out;      // optional [K][H]
    float4* hyp_out;          // optional [K][H]
    double* area_out;
};

struct TileLds {
    float4 pl[kFMaxChunk];
    uint32_t cnt[kFMaxChunk];
};
struct SmallLds {
    float x[kFSmallMax], y[kFSmallMax], z[kFSmallMax];
};
struct FinishLds {
    uint32_t mask[kFTile / 32];
    uint32_t wsum[kFWaves];
    int32_t bc[kFWaves];
    uint32_t bh[kFWaves];
    double rv[kFWaves][kDirs];
    uint32_t ri[kFWaves][kDirs];
    double P[kPolyWords];
    uint32_t count;
    double wu[kWave], wv[kWave];
    uint32_t wi[kWave];
    uint8_t wst[2 * kWave + 2];
};
union FusedLds {
    TileLds t;
    SmallLds s;
    FinishLds f;
};

// planes hb..he (at most 64) of the LDS chunk against the wave's rows of
// points; lane q of the result holds the count of plane hb + q.  The planes
// are read four at a time (their LDS loads are issued together) and counted
// without a branch: a degenerate plane is NaN and passes no test.
constexpr int kLdsBatch = 4;

template <int R>
__device__ __forceinline__ uint32_t plane_count(const float4 p, const float* px, const float* py, const float* pz,
                                                float eps)
{
    // stage by stage over the rows, so that their chains interleave
    float dd[R];
#pragma unroll
    for (int j = 0; j < R; ++j) dd[j] = fmaf(p.x, px[j], p.w);
#pragma unroll
    for (int j = 0; j < R; ++j) dd[j] = fmaf(p.y, py[j], dd[j]);
#pragma unroll
    for (int j = 0; j < R; ++j) dd[j] = fmaf(p.z, pz[j], dd[j]);
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) acc += (uint32_t)__popcll(__ballot(fabsf(dd[j]) < eps));
    return acc;
}

template <int R>
__device__ __forceinline__ uint32_t lds_batch(const float4* pl, uint32_t hb, uint32_t he, const float* px,
                                              const float* py, const float* pz, float eps, int lane)
{
    uint32_t cv = 0;
    uint32_t h = hb;
    for (; h + kLdsBatch <= he; h += kLdsBatch) {
        float4 p[kLdsBatch];
#pragma unroll
        for (int b = 0; b < kLdsBatch; ++b) p[b] = pl[h + b];
#pragma unroll
        for (int b = 0; b < kLdsBatch; ++b) {
            const uint32_t acc = plane_count<R>(p[b], px, py, pz, eps);
            cv = (lane == (int)(h + b - hb)) ? acc : cv;
        }
    }
    for (; h < he; ++h) {
        const uint32_t acc = plane_count<R>(pl[h], px, py, pz, eps);
        cv = (lane == (int)(h - hb)) ? acc : cv;
    }
    return cv;
}

template <int R>
__device__ __forceinline__ void lds_count(const float4* pl, uint32_t nc, const float* px, const float* py,
                                          const float* pz, float eps, uint32_t* cnt, int lane)
{
    for (uint32_t hb = 0; hb < nc; hb += kWave) {
        const uint32_t he = min(nc, hb + (uint32_t)kWave);
        const uint32_t cv = lds_batch<R>(pl, hb, he, px, py, pz, eps, lane);
        if ((uint32_t)lane < he - hb && cv) atomicAdd(&cnt[hb + (uint32_t)lane], cv);
    }
}

// (c) and the polygon of cluster k, by the workgroup that completed it
__device__ void finish_cluster(const FusedArgs& a, uint32_t k, uint32_t frame, FinishLds& L)
{
    const FusedWork& w = a.w;
    const uint32_t H = a.sp.H;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint32_t base = a.off[k], n = a.off[k + 1] - base;
    const uint32_t rows = is_small(n, a.sp) ? 1u : tiles_of(n);
    const int32_t* part = w.part + (size_t)w.tbase[k] * H;
    // best hypothesis: largest count, first index on ties; degenerate ones count -1
    int32_t bc = -1;
    uint32_t bh = 0xFFFFFFFFu;
    for (uint32_t h = threadIdx.x; h < H; h += kFBlock) {
        const float4 pl = w.hyp[(size_t)k * H + h];
        const bool degen = pl.x != pl.x;
        int32_t c = 0;
        for (uint32_t t = 0; t < rows; ++t) c += part[(size_t)t * H + h];
        if (degen) c = -1;
        if (c > bc) { bc = c; bh = h; }
        if (a.counts_out) a.counts_out[(size_t)k * H + h] = c;
        if (a.hyp_out) a.hyp_out[(size_t)k * H + h] = degen ? make_float4(0.f, 0.f, 0.f, 0.f) : pl;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const int32_t oc = __shfl_xor(bc, d, kWave);
        const uint32_t oh = __shfl_xor(bh, d, kWave);
        if (oc > bc || (oc == bc && oh < bh)) { bc = oc; bh = oh; }
    }
    if (lane == 0) {
        L.bc[wave] = bc;
        L.bh[wave] = bh;
    }
    __syncthreads();
    bc = L.bc[0];
    bh = L.bh[0];
    for (int v = 1; v < kFWaves; ++v)
        if (L.bc[v] > bc || (L.bc[v] == bc && L.bh[v] < bh)) { bc = L.bc[v]; bh = L.bh[v]; }
    const float4 pl = bc >= 0 ? w.hyp[(size_t)k * H + bh] : make_float4(0.f, 0.f, 0.f, 0.f);
    if (threadIdx.x == 0) {
        a.best_out[k] = bc >= 0 ? (int32_t)bh : -1;
        a.nin_out[k] = bc >= 0 ? bc : 0;
        a.plane_out[k] = pl;
        w.nin[k] = bc >= 0 ? (uint32_t)bc : 0u;
        w.hcnt[k] = 0;
        a.area_out[k] = 0.0;
    }
    if (bc <= 0) return;   // no plane or no inlier: no list, no polygon (workgroup-uniform)
    // the inlier list in point order: coalesced tests collected as bit masks
    // in LDS, then a thread per 32-point word places its inliers
    uint32_t run = 0;
    for (uint32_t r0 = 0; r0 < n; r0 += kFTile) {
        __syncthreads();   // mask and wsum of the previous round are consumed
#pragma unroll 4
        for (uint32_t j0 = 0; j0 < kFTile; j0 += kFBlock) {
            const uint32_t i = r0 + j0 + threadIdx.x;
            const bool in = i < n && inlier_test(pl, a.X[base + i], a.Y[base + i], a.Z[base + i], a.eps);
            const uint64_t b = __ballot(in);
            if (lane == 0) {
                const uint32_t wd = (j0 + (uint32_t)wave * kWave) / 32;
                L.mask[wd] = (uint32_t)b;
                L.mask[wd + 1] = (uint32_t)(b >> 32);
            }
        }
        __syncthreads();
        uint32_t m = threadIdx.x < kFTile / 32 ? L.mask[threadIdx.x] : 0u;
        const uint32_t c = (uint32_t)__popc(m);
        uint32_t inc = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d, kWave);
            if (lane >= d) inc += o;
        }
        if (lane == kWave - 1) L.wsum[wave] = inc;
        __syncthreads();
        uint32_t p = run + inc - c, tot = 0;
#pragma unroll
        for (int v = 0; v < kFWaves; ++v) {
            p += (v < wave) ? L.wsum[v] : 0u;
            tot += L.wsum[v];
        }
        const uint32_t q0 = r0 + threadIdx.x * 32;
        for (; m; m &= m - 1, ++p) w.slot_in[base + p] = q0 + (uint32_t)(__ffs(m) - 1);
        run += tot;
    }
    __syncthreads();
    // ---- the polygon of the inliers (the same steps as vm_hulls) ----
    const uint32_t mI = run;
    const uint32_t* inl = w.slot_in + base;
    ClusterFrame f;
    f.ib = 0;
    f.m = mI;
    f.pb = base;
    f.nk = n;
    f.B = plane_basis(pl);
    {
        const uint32_t i0 = base + inl[0];
        f.ox = a.X[i0];
        f.oy = a.Y[i0];
        f.oz = a.Z[i0];
    }
    auto proj = [&](uint32_t j, double* pu, double* pv) {
        const uint32_t i = base + inl[j];
        project(f, a.X[i], a.Y[i], a.Z[i], pu, pv);
    };
    uint32_t* vout = w.slot_hull + base + k;
    if (mI <= (uint32_t)kWave) {
        // all inliers on one wave, sorted and chained there
        if (wave == 0) {
            double u = INFINITY, v = INFINITY;
            uint32_t i = 0xFFFFFFFFu;
            if ((uint32_t)lane < mI) {
                proj((uint32_t)lane, &u, &v);
                i = (uint32_t)lane;
            }
            const WaveHull r = wave_hull(u, v, i, mI, lane, L.wu, L.wv, L.wi, L.wst);
            if (lane == 0) {
                a.area_out[k] = r.area;
                w.hcnt[k] = r.h;
            }
            if ((uint32_t)lane < r.h) vout[lane] = inl[L.wi[r.vi]];
        }
        return;
    }
    // extreme inliers in 8 directions (first position on ties)
    double bv[kDirs];
    uint32_t bi[kDirs];
#pragma unroll
    for (int d = 0; d < kDirs; ++d) { bv[d] = -INFINITY; bi[d] = 0xFFFFFFFFu; }
    for (uint32_t j = threadIdx.x; j < mI; j += kFBlock) {
        double pu, pv;
        proj(j, &pu, &pv);
#pragma unroll
        for (int d = 0; d < kDirs; ++d) {
            const double v = dir_val(d, pu, pv);
            if (v > bv[d]) { bv[d] = v; bi[d] = j; }
        }
    }
#pragma unroll
    for (int d = 0; d < kDirs; ++d) {
        for (int s = kWave / 2; s >= 1; s >>= 1) {
            const double ov = __shfl_xor(bv[d], s, kWave);
            const uint32_t oi = __shfl_xor(bi[d], s, kWave);
            if (ov > bv[d] || (ov == bv[d] && oi < bi[d])) { bv[d] = ov; bi[d] = oi; }
        }
        if (lane == 0) { L.rv[wave][d] = bv[d]; L.ri[wave][d] = bi[d]; }
    }
    if (threadIdx.x == 0) L.count = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t e[kDirs];
        for (int d = 0; d < kDirs; ++d) {
            double v = L.rv[0][d];
            uint32_t ix = L.ri[0][d];
            for (int q = 1; q < kFWaves; ++q)
                if (L.rv[q][d] > v || (L.rv[q][d] == v && L.ri[q][d] < ix)) { v = L.rv[q][d]; ix = L.ri[q][d]; }
            e[d] = ix;
        }
        extreme_polygon(e, mI, L.P, proj);
    }
    __syncthreads();
    // survivors: inliers not strictly inside the polygon, at off[k] + s
    {
        const int np = (int)L.P[kPolyWords - 1];
        const double mg = L.P[kPolyWords - 2];
        for (uint32_t j = threadIdx.x; j < mI; j += kFBlock) {
            double pu, pv;
            proj(j, &pu, &pv);
            bool inside = np >= 3;
            for (int q = 0; inside && q < np; ++q) {
                const int b = (q + 1 == np) ? 0 : q + 1;
                inside = cross3(L.P[q], L.P[kDirs + q], L.P[b], L.P[kDirs + b], pu, pv) > mg;
            }
            if (!inside) {
                const uint32_t s = atomicAdd(&L.count, 1u);
                w.su[base + s] = pu;
                w.sv[base + s] = pv;
                w.si[base + s] = j;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint32_t ns = L.count;
    if (ns <= (uint32_t)kWave) {
        if (wave == 0) {
            double u = INFINITY, v = INFINITY;
            uint32_t i = 0xFFFFFFFFu;
            if ((uint32_t)lane < ns) {
                u = w.su[base + lane];
                v = w.sv[base + lane];
                i = w.si[base + lane];
            }
            const WaveHull r = wave_hull(u, v, i, ns, lane, L.wu, L.wv, L.wi, L.wst);
            if (lane == 0) {
                a.area_out[k] = r.area;
                w.hcnt[k] = r.h;
            }
            if ((uint32_t)lane < r.h) vout[lane] = inl[L.wi[r.vi]];
        }
    } else if (threadIdx.x == 0) {
        // more survivors than one wave: the tail launch sorts and chains them
        w.surv[k] = ns;
        w.tail[atomicAdd(&w.small[7], 1u)] = k;
    }
}

__global__ void __launch_bounds__(kFBlock) k_fused(FusedArgs a)
{
    __shared__ FusedLds L;
    __shared__ uint32_t s_item, s_flag;
    const FusedWork& w = a.w;
    const Split& sp = a.sp;
    const uint32_t H = sp.H;
    const uint32_t frame_all = a.d_frame ? *a.d_frame : a.frame;
    const uint32_t K = w.small[0], total = w.small[1];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&w.small[2], 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= total) break;   // workgroup-uniform: every wave leaves
        // the queue position holding the item: largest i with item_off[i] <= item
        uint32_t lo = 0, hi = K;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (w.item_off[mid] <= item) lo = mid;
            else hi = mid;
        }
        const uint32_t k = w.order[lo], j = item - w.item_off[lo];
        const uint32_t base = a.off[k], n = a.off[k + 1] - base;
        const uint32_t frame = a.cframe ? a.cframe[k] : frame_all;
        const bool small = is_small(n, sp);
        const uint32_t c = small ? j : j % sp.nch, t = small ? 0u : j / sp.nch;
        const uint32_t h0 = c * sp.chunk, h1 = min(H, h0 + sp.chunk);
        int32_t* part = w.part + (size_t)(w.tbase[k] + t) * H;
        if (small) {
            // lanes over planes, all points of the cluster in LDS
            for (uint32_t i = threadIdx.x; i < n; i += kFBlock) {
                L.s.x[i] = a.X[base + i];
                L.s.y[i] = a.Y[base + i];
                L.s.z[i] = a.Z[base + i];
            }
            __syncthreads();
            for (uint32_t h = h0 + threadIdx.x; h < h1; h += kFBlock) {
                const float4 pl = w.hyp[(size_t)k * H + h];
                // points read eight at a time (broadcast LDS loads issued together)
                uint32_t cnt = 0, i = 0;
                for (; i + 8 <= n; i += 8) {
                    float qx[8], qy[8], qz[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        qx[u] = L.s.x[i + u];
                        qy[u] = L.s.y[i + u];
                        qz[u] = L.s.z[i + u];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float dd = fmaf(pl.z, qz[u], fmaf(pl.y, qy[u], fmaf(pl.x, qx[u], pl.w)));
                        cnt += fabsf(dd) < a.eps ? 1u : 0u;   // a degenerate (NaN) plane never passes
                    }
                }
                for (; i < n; ++i) {
                    const float dd = fmaf(pl.z, L.s.z[i], fmaf(pl.y, L.s.y[i], fmaf(pl.x, L.s.x[i], pl.w)));
                    cnt += fabsf(dd) < a.eps ? 1u : 0u;
                }
                part[h] = (int32_t)cnt;
            }
        } else {
            // the chunk's planes into LDS
            for (uint32_t h = h0 + threadIdx.x; h < h1; h += kFBlock) L.t.pl[h - h0] = w.hyp[(size_t)k * H + h];
            for (uint32_t h = threadIdx.x; h < h1 - h0; h += kFBlock) L.t.cnt[h] = 0;
            __syncthreads();
            // this wave's rows of the tile
            const uint32_t p0 = base + t * kFTile, pend = base + n;
            const uint32_t wb = p0 + (uint32_t)(wave * kWave * kFRows);
            const int rows = pend > wb ? (int)min((uint32_t)kFRows, (pend - wb + kWave - 1) / kWave) : 0;
            float px[kFRows], py[kFRows], pz[kFRows];
            const float qnan = __builtin_nanf("");
#pragma unroll
            for (int r = 0; r < kFRows; ++r) {
                const uint32_t i = wb + (uint32_t)(r * kWave + lane);
                const bool v = i < pend;
                px[r] = v ? a.X[i] : qnan;   // NaN never passes |d| < eps
                py[r] = v ? a.Y[i] : qnan;
                pz[r] = v ? a.Z[i] : qnan;
            }
            const uint32_t nc = h1 - h0;
            static_assert(kFRows == 16, "the row dispatch below assumes 16 rows per lane");
            if (rows > 8) lds_count<16>(L.t.pl, nc, px, py, pz, a.eps, L.t.cnt, lane);
            else if (rows > 4) lds_count<8>(L.t.pl, nc, px, py, pz, a.eps, L.t.cnt, lane);
            else if (rows > 2) lds_count<4>(L.t.pl, nc, px, py, pz, a.eps, L.t.cnt, lane);
            else if (rows > 1) lds_count<2>(L.t.pl, nc, px, py, pz, a.eps, L.t.cnt, lane);
            else if (rows == 1) lds_count<1>(L.t.pl, nc, px, py, pz, a.eps, L.t.cnt, lane);
            __syncthreads();
            for (uint32_t h = threadIdx.x; h < nc; h += kFBlock) part[h0 + h] = (int32_t)L.t.cnt[h];
        }
        // completion.  A cluster of one item is finished by the workgroup
        // that counted it (its counts are this workgroup's own stores, made
        // visible by the barrier).  Otherwise the item's stores become
        // visible device-wide before its count, and the workgroup that
        // completes the cluster acquires them: on this chip an agent-scope
        // release writes the XCD's L2 back and an acquire invalidates it,
        // so they are kept to the clusters that need them.
        const bool single = items_of(n, sp) == 1u;
        if (!single) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) s_flag = single || atomicAdd(&w.done[k], 1u) + 1u == items_of(n, sp);
        __syncthreads();
        if (s_flag) {
            if (!single) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            finish_cluster(a, k, frame, L.f);
        }
        __syncthreads();   // LDS and s_item are reused by the next item
    }
}

// (a) for the whole set: plane h of cluster k for every k < K, h < H
__global__ void __launch_bounds__(kFBlock) k_fused_hyp(FusedArgs a)
{
    const uint32_t H = a.sp.H, K = a.w.small[0];
    const uint32_t frame_all = a.d_frame ? *a.d_frame : a.frame;
    const uint64_t total = (uint64_t)K * H;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = (uint32_t)(i / H), h = (uint32_t)(i % H);
        const uint32_t base = a.off[k], n = a.off[k + 1] - base;
        const uint32_t frame = a.cframe ? a.cframe[k] : frame_all;
        a.w.hyp[i] = hyp_plane(a.X + base, a.Y + base, a.Z + base, n, h, a.tag[k], frame, a.seed);
    }
}

// ---- packing into the caller's compact CSR outputs ---------------------------------
// One workgroup: inlier and vertex offsets (a cluster whose inlier list does
// not fit in_cap gets no polygon, as in vm_hulls), totals, overflow flags.
__global__ void __launch_bounds__(kOneBlockThreads) k_fused_scan(FusedWork w, uint32_t in_cap, uint32_t* __restrict__ in_off,
                                                                  uint32_t* __restrict__ v_off, double* __restrict__ area,
                                                                  uint32_t* __restrict__ pstatus,
                                                                  uint32_t* __restrict__ hstatus)
{
    const uint32_t K = w.small[0];
    uint32_t tot[1];
    one_block_scan<kOneBlockThreads, 4, 1>(
        K, [&](uint32_t k, uint32_t(&v)[1]) { v[0] = w.nin[k]; },
        [&](uint32_t k, const uint32_t(&e)[1]) { in_off[k] = e[0]; }, tot);
    __syncthreads();   // in_off of the other threads
    uint32_t vt[1];
    one_block_scan<kOneBlockThreads, 4, 1>(
        K,
        [&](uint32_t k, uint32_t(&v)[1]) {
            const bool fits = in_off[k] + w.nin[k] <= in_cap;
            if (!fits && w.hcnt[k]) {
                w.hcnt[k] = 0;
                area[k] = 0.0;
            }
            v[0] = w.hcnt[k];
        },
        [&](uint32_t k, const uint32_t(&e)[1]) { v_off[k] = e[0]; }, vt);
    if (threadIdx.x == 0) {
        in_off[K] = tot[0];
        v_off[K] = vt[0];
        w.small[5] = vt[0];
        w.small[8] = tot[0];
        if (tot[0] > in_cap) atomicOr(pstatus, (uint32_t)VM_FLAG_INLIERS_CAP);
        if (tot[0] > in_cap) atomicOr(hstatus, (uint32_t)VM_FLAG_INLIERS_CAP);
    }
}

// The lists into the caller's compact outputs.  Inlier indices go by output
// position, a 4096-entry chunk per workgroup at a time (its first cluster
// found by a binary search over the offsets, later ones by stepping), so a
// 200k-inlier cluster is copied by many workgroups, not one; polygon
// vertices (a few dozen per cluster) go a workgroup per cluster, each
// projected onto its plane.
constexpr uint32_t kCopyChunk = 4096;

__global__ void __launch_bounds__(kFBlock) k_fused_copy(FusedWork w, const uint32_t* __restrict__ off,
                                                        const float* __restrict__ X, const float* __restrict__ Y,
                                                        const float* __restrict__ Z,
                                                        const float4* __restrict__ plane,
                                                        const uint32_t* __restrict__ in_off, uint32_t in_cap,
                                                        uint32_t* __restrict__ in_idx,
                                                        const uint32_t* __restrict__ v_off, uint32_t v_cap,
                                                        uint32_t* __restrict__ v_idx, float* __restrict__ v_xyz,
                                                        uint32_t* __restrict__ hstatus)
{
    __shared__ uint32_t s_k;
    const uint32_t K = w.small[0];
    const uint32_t total = min(w.small[8], in_cap);   // inlier entries that fit the output
    for (uint32_t c0 = blockIdx.x * kCopyChunk; c0 < total; c0 += gridDim.x * kCopyChunk) {
        if (threadIdx.x == 0) {
            // the last cluster whose list starts at or before c0
            uint32_t lo = 0, hi = K;
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (in_off[mid] <= c0) lo = mid;
                else hi = mid;
            }
            s_k = lo;
        }
        __syncthreads();
        uint32_t k = s_k;
        const uint32_t c1 = min(c0 + kCopyChunk, total);
        for (uint32_t p = c0 + threadIdx.x; p < c1; p += kFBlock) {
            while (in_off[k + 1] <= p) ++k;   // p < total <= in_off[K]: ends
            in_idx[p] = w.slot_in[off[k] + (p - in_off[k])];
        }
        __syncthreads();   // s_k is rewritten for the next chunk
    }
    bool over = false;
    for (uint32_t k = blockIdx.x; k < K; k += gridDim.x) {
        const uint32_t h = w.hcnt[k];
        if (h == 0) continue;
        const uint32_t base = off[k];
        const uint32_t vb = v_off[k];
        const float4 pl = plane[k];
        const double nx = pl.x, ny = pl.y, nz = pl.z, d = pl.w;
        for (uint32_t q = threadIdx.x; q < h; q += kFBlock) {
            const uint32_t pos = vb + q;
            if (pos >= v_cap) {
                over = true;
                continue;
            }
            const uint32_t jj = w.slot_hull[base + k + q];
            const double px = X[base + jj], py = Y[base + jj], pz = Z[base + jj];
            const double dist = nx * px + ny * py + nz * pz + d;
            v_idx[pos] = jj;
            v_xyz[3 * (size_t)pos + 0] = (float)(px - dist * nx);
            v_xyz[3 * (size_t)pos + 1] = (float)(py - dist * ny);
            v_xyz[3 * (size_t)pos + 2] = (float)(pz - dist * nz);
        }
    }
    if (over) atomicOr(hstatus, (uint32_t)VM_FLAG_HULL_CAP);
}

// ---- the work split: process-wide setting and per-shape autotuned choices ------
std::mutex g_fused_mu;
vm_fused_config g_fused_cfg = {512, 0, 5, 0};   // fused_config_default()
std::map<std::tuple<uint32_t, uint32_t, uint32_t>, vm_fused_config> g_fused_cache;

std::tuple<uint32_t, uint32_t, uint32_t> shape_bucket(uint32_t k_cap, uint32_t n_cap, uint32_t H)
{
    auto lg = [](uint32_t x) { uint32_t r = 0; while (x > 1) { x >>= 1; ++r; } return r; };
    return {lg(k_cap), lg(n_cap), lg(H)};
}

}  // namespace

bool fused_config_valid(const vm_fused_config& c)
{
    return c.hyp_chunk >= 64 && c.hyp_chunk <= kFMaxChunk && c.hyp_chunk % 64 == 0 && c.small_max <= kFSmallMax &&
           c.groups_per_cu >= 1 && c.groups_per_cu <= 8 && c.reserved == 0;
}

vm_fused_config fused_config_default() { return vm_fused_config{512, 0, 5, 0}; }

vm_fused_config fused_config_get()
{
    std::lock_guard<std::mutex> g(g_fused_mu);
    return g_fused_cfg;
}

void fused_config_set(const vm_fused_config& c)
{
    std::lock_guard<std::mutex> g(g_fused_mu);
    g_fused_cfg = c;
}

void fused_cache_put(uint32_t k_cap, uint32_t n_cap, uint32_t H, const vm_fused_config& c)
{
    std::lock_guard<std::mutex> g(g_fused_mu);
    g_fused_cache[shape_bucket(k_cap, n_cap, H)] = c;
}

bool fused_cache_get(uint32_t k_cap, uint32_t n_cap, uint32_t H, vm_fused_config* c)
{
    std::lock_guard<std::mutex> g(g_fused_mu);
    auto it = g_fused_cache.find(shape_bucket(k_cap, n_cap, H));
    if (it == g_fused_cache.end()) return false;
    *c = it->second;
    return true;
}

void fused_cache_clear()
{
    std::lock_guard<std::mutex> g(g_fused_mu);
    g_fused_cache.clear();
}

size_t fused_workspace_bytes(uint32_t k_cap, uint32_t n_cap, uint32_t H)
{
    return fused_layout(nullptr, k_cap, n_cap, H).bytes;
}

namespace {

Split make_split(uint32_t H, const vm_fused_config& cfg)
{
    Split sp;
    sp.H = H;
    sp.chunk = std::min<uint32_t>(cfg.hyp_chunk, ((H + kWave - 1) / kWave) * kWave);
    sp.nch = (H + sp.chunk - 1) / sp.chunk;
    sp.small_max = cfg.small_max;
    return sp;
}

int device_cus()
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
    }
    return cus;
}

// preparation, the persistent kernel and the tail chain: per-cluster
// results (best, plane, inlier count, area, optional counts/planes of every
// hypothesis) in the outputs, lists in the workspace slots
vm_status fused_core(const vm_clusters& cl, const vm_ransac_params& p, const uint32_t* d_cframe, uint32_t kc,
                     uint32_t out_k_cap, const FusedWork& w, const Split& sp, float4* plane_out, int32_t* best_out,
                     int32_t* nin_out, int32_t* counts_out, float4* hyp_out, double* area_out, uint32_t* status,
                     uint32_t groups_per_cu, hipStream_t s)
{
    {
        StageScope t(VM_STAGE_HYPOTHESES, s);
        k_fused_prepare<<<1, kOneBlockThreads, 0, s>>>(cl.d_meta, kc, out_k_cap, cl.n_cap, cl.d_off, sp, w, status);
        VM_HIP(hipGetLastError());
    }
    FusedArgs a;
    {
        a.off = cl.d_off;
        a.X = cl.d_x;
        a.Y = cl.d_y;
        a.Z = cl.d_z;
        a.tag = cl.d_tag;
        a.cframe = d_cframe;
        a.d_frame = p.d_frame;
        a.frame = p.frame;
        a.eps = p.eps;
        a.seed = p.seed;
        a.sp = sp;
        a.w = w;
        a.plane_out = plane_out;
        a.best_out = best_out;
        a.nin_out = nin_out;
        a.counts_out = counts_out;
        a.hyp_out = hyp_out;
        a.area_out = area_out;
    }
    {
        StageScope t(VM_STAGE_HYPOTHESES, s);
        k_fused_hyp<<<grid_for((uint64_t)kc * sp.H, kFBlock, 4096), kFBlock, 0, s>>>(a);
        VM_HIP(hipGetLastError());
    }
    {
        StageScope t(VM_STAGE_COUNT, s);
        k_fused<<<device_cus() * (int)groups_per_cu, kFBlock, 0, s>>>(a);
        VM_HIP(hipGetLastError());
    }
    StageScope t(VM_STAGE_HULL, s);
    VM_HIP(launch_hull_chain_list(w.small, w.tail, cl.d_off, w.slot_in, w.surv, w.su, w.sv, w.si, w.hcnt, w.slot_hull,
                                  area_out, std::min<uint32_t>(kc ? kc : 1, 512), s));
    return VM_OK;
}

}  // namespace

vm_status planes_and_hulls(const vm_clusters& cl, const vm_ransac_params& p, const uint32_t* d_cframe,
                           const vm_planes& planes, const vm_hulls_out& hulls, void* d_work, size_t work_bytes,
                           const vm_fused_config& cfg, hipStream_t s)
{
    uint32_t kc = std::min(cl.k_cap, std::min(planes.k_cap, hulls.k_cap));
    if (kc > kOneBlockMax) return VM_E_CAPACITY;
    const uint32_t H = p.n_hyp;
    const FusedWork w = fused_layout(d_work, kc, cl.n_cap, H);
    if (w.bytes > work_bytes) return VM_E_CAPACITY;
    const Split sp = make_split(H, cfg);
    vm_status st = fused_core(cl, p, d_cframe, kc, std::min(planes.k_cap, hulls.k_cap), w, sp,
                              (float4*)planes.d_plane, planes.d_best_h, planes.d_n_inliers, planes.d_counts,
                              (float4*)planes.d_hyp, hulls.d_area, planes.d_status, cfg.groups_per_cu, s);
    if (st != VM_OK) return st;
    StageScope t(VM_STAGE_HULL, s);
    k_fused_scan<<<1, kOneBlockThreads, 0, s>>>(w, planes.in_cap, planes.d_in_off, hulls.d_v_off, hulls.d_area,
                                                planes.d_status, hulls.d_status);
    k_fused_copy<<<2048, kFBlock, 0, s>>>(w, cl.d_off, cl.d_x, cl.d_y, cl.d_z, (const float4*)planes.d_plane,
                                           planes.d_in_off, planes.in_cap, planes.d_in_idx, hulls.d_v_off,
                                           hulls.v_cap, hulls.d_v_idx, hulls.d_v_xyz, hulls.d_status);
    VM_HIP(hipGetLastError());
    return VM_OK;
}

}  // namespace vm

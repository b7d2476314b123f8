// vm_hull.hip -- boundary polygons (Sec. III-C, "Boundary polygon
// generation"): the convex hull of each plane's inliers, in the plane.
//
// The paper filters most points on the GPU and finishes each hull on the CPU
// from the few candidates left.  Here the whole hull stays on the device and
// every pass over the inliers is tile-parallel, so one huge cluster (a floor)
// spreads over the whole chip instead of one workgroup:
//   B. per tile of inliers: project onto the in-plane basis (fp64) and find
//      the extreme inlier in each of 8 directions (every 45 degrees);
//   C. per cluster: combine the tiles' extremes; the convex polygon through
//      them lies inside the hull, so a point strictly inside it (by a margin
//      far above the fp64 rounding of the test) cannot be a hull vertex;
//   D. per tile: keep only the points not strictly inside that polygon
//      (block-aggregated compaction into the cluster's own region);
//   E. per cluster: sort the survivors by (u, v, inlier index) -- in a
//      wave's registers for at most 64, bitonic in LDS, or in global memory
//      for very large survivor sets -- and run Andrew's monotone chain,
//      popping on every non-left turn (strictly convex, counter-clockwise
//      from the smallest point).  Up to LDS size the lower and the upper
//      chain run at once; joined at their shared end points they give
//      exactly the single-stack chain's output;
//   F. scan the vertex counts and pack the polygons, each vertex projected
//      onto the plane.
#include "vm_common.h"
#include "vm_dev.h"

#include <math.h>

namespace vm {
namespace {

using namespace dev;

constexpr int kTileThreads = 256;
constexpr int kTileItems = 4;
constexpr int kHullTile = kTileThreads * kTileItems;   // inliers per tile
constexpr int kSmallGrid = 2048;   // workgroups of the wave-per-cluster kernels (8192 waves)
constexpr int kLdsCap = 2048;                           // survivors sorted in LDS

// Whether cluster k gets a polygon: it has a plane, its inlier list fits the
// output and indexes its own points.
__device__ __forceinline__ bool cluster_ok(uint32_t k, const uint32_t* off, const int32_t* best,
                                           const uint32_t* in_off, const uint32_t* in_idx, uint32_t in_cap)
{
    const uint32_t ib = in_off[k], ie = in_off[k + 1];
    if (best[k] < 0 || ie <= ib || ie > in_cap) return false;
    return in_idx[ib] < off[k + 1] - off[k];
}

__device__ __forceinline__ ClusterFrame cluster_frame(uint32_t k, const uint32_t* off, const float* X, const float* Y,
                                                      const float* Z, const float4* plane, const uint32_t* in_off,
                                                      const uint32_t* in_idx)
{
    ClusterFrame f;
    f.ib = in_off[k];
    f.m = in_off[k + 1] - f.ib;
    f.pb = off[k];
    f.nk = off[k + 1] - f.pb;
    f.B = plane_basis(plane[k]);
    const uint32_t i0 = f.pb + in_idx[f.ib];
    f.ox = X[i0];
    f.oy = Y[i0];
    f.oz = Z[i0];
    return f;
}


// largest k with tile_off[k] <= t (tile_off is an exclusive scan of K entries)
__device__ __forceinline__ uint32_t cluster_of_tile(const uint32_t* __restrict__ tile_off, uint32_t K, uint32_t t)
{
    uint32_t lo = 0, hi = K;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tile_off[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// tiles of cluster k: [tile_off[k], end)
__device__ __forceinline__ uint32_t tiles_end(const uint32_t* tile_off, uint32_t k, uint32_t K, uint32_t total)
{
    return k + 1 < K ? tile_off[k + 1] : total;
}

// ---- A: validate, tiles per cluster ------------------------------------------
__global__ void __launch_bounds__(kBlock) k_hull_validate(const uint32_t* __restrict__ meta, uint32_t kc,
                                                          uint32_t n_cap, const uint32_t* __restrict__ off,
                                                          uint32_t* small, uint32_t* status)
{
    __shared__ int bad;
    const uint32_t K = validate_clusters(meta, off, kc, n_cap, status, &bad);
    if (threadIdx.x == 0) {
        small[4] = K;
        small[7] = 0;   // chain list
        small[9] = 0;   // mid list
    }
}

__global__ void __launch_bounds__(kBlock) k_hull_tiles(const uint32_t* __restrict__ small,
                                                       const uint32_t* __restrict__ off,
                                                       const int32_t* __restrict__ best,
                                                       const uint32_t* __restrict__ in_off,
                                                       const uint32_t* __restrict__ in_idx, uint32_t in_cap,
                                                       uint32_t* __restrict__ ntiles, uint32_t* __restrict__ status)
{
    const uint32_t K = small[4];
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        const bool ok = cluster_ok(k, off, best, in_off, in_idx, in_cap);
        const uint32_t m = ok ? in_off[k + 1] - in_off[k] : 0u;
        // clusters with at most one wave of inliers skip the tiled filter
        ntiles[k] = m > (uint32_t)kWave ? (m + kHullTile - 1) / kHullTile : 0u;
        if (best[k] >= 0 && in_off[k + 1] > in_cap) atomicOr(status, (uint32_t)VM_FLAG_INLIERS_CAP);
    }
}

// validate, tiles per cluster and their offsets in one workgroup (the
// capacity is at most kOneBlockMax clusters)
__global__ void __launch_bounds__(kOneBlockThreads) k_hull_prepare(
    const uint32_t* __restrict__ meta, uint32_t kc, uint32_t n_cap, const uint32_t* __restrict__ off,
    const int32_t* __restrict__ best, const uint32_t* __restrict__ in_off, const uint32_t* __restrict__ in_idx,
    uint32_t in_cap, uint32_t* __restrict__ small, uint32_t* __restrict__ tile_off, uint32_t* __restrict__ status)
{
    __shared__ int bad;
    const uint32_t K = validate_clusters(meta, off, kc, n_cap, status, &bad);
    uint32_t total[1];
    one_block_scan<kOneBlockThreads, 4, 1>(
        K,
        [&](uint32_t k, uint32_t(&v)[1]) {
            const bool ok = cluster_ok(k, off, best, in_off, in_idx, in_cap);
            const uint32_t m = ok ? in_off[k + 1] - in_off[k] : 0u;
            v[0] = m > (uint32_t)kWave ? (m + kHullTile - 1) / kHullTile : 0u;
            if (best[k] >= 0 && in_off[k + 1] > in_cap) atomicOr(status, (uint32_t)VM_FLAG_INLIERS_CAP);
        },
        [&](uint32_t k, const uint32_t(&e)[1]) { tile_off[k] = e[0]; }, total);
    if (threadIdx.x == 0) {
        small[4] = K;
        small[6] = total[0];
        small[7] = 0;   // chain list
        small[9] = 0;   // mid list
    }
}

// ---- B: projection + directional extremes per tile --------------------------------
__global__ void __launch_bounds__(kTileThreads) k_hull_extremes(
    const uint32_t* __restrict__ small, const uint32_t* __restrict__ tile_off, const uint32_t* __restrict__ off,
    const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
    const float4* __restrict__ plane, const uint32_t* __restrict__ in_off, const uint32_t* __restrict__ in_idx,
    double* __restrict__ ext_v, uint32_t* __restrict__ ext_i)
{
    __shared__ double rv[kTileThreads / kWave][kDirs];
    __shared__ uint32_t ri[kTileThreads / kWave][kDirs];
    const uint32_t K = small[4];
    const uint32_t T = small[6];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (uint32_t t = blockIdx.x; t < T; t += gridDim.x) {
        const uint32_t k = cluster_of_tile(tile_off, K, t);
        const ClusterFrame f = cluster_frame(k, off, X, Y, Z, plane, in_off, in_idx);
        const uint32_t j0 = (t - tile_off[k]) * kHullTile, j1 = min(j0 + kHullTile, f.m);
        double bv[kDirs];
        uint32_t bi[kDirs];
#pragma unroll
        for (int d = 0; d < kDirs; ++d) { bv[d] = -INFINITY; bi[d] = 0xFFFFFFFFu; }
        for (uint32_t j = j0 + threadIdx.x; j < j1; j += kTileThreads) {
            const uint32_t li = in_idx[f.ib + j];
            if (li >= f.nk) continue;
            const uint32_t i = f.pb + li;
            double pu, pv;
            project(f, X[i], Y[i], Z[i], &pu, &pv);
#pragma unroll
            for (int d = 0; d < kDirs; ++d) {
                const double v = dir_val(d, pu, pv);
                if (v > bv[d]) { bv[d] = v; bi[d] = j; }   // j ascends per thread: first maximum kept
            }
        }
#pragma unroll
        for (int d = 0; d < kDirs; ++d) {
            for (int s = kWave / 2; s >= 1; s >>= 1) {
                const double ov = __shfl_xor(bv[d], s, kWave);
                const uint32_t oi = __shfl_xor(bi[d], s, kWave);
                if (ov > bv[d] || (ov == bv[d] && oi < bi[d])) { bv[d] = ov; bi[d] = oi; }
            }
            if (lane == 0) { rv[wave][d] = bv[d]; ri[wave][d] = bi[d]; }
        }
        __syncthreads();
        if (threadIdx.x < kDirs) {
            const int d = threadIdx.x;
            double v = rv[0][d];
            uint32_t ix = ri[0][d];
            for (int w = 1; w < kTileThreads / kWave; ++w)
                if (rv[w][d] > v || (rv[w][d] == v && ri[w][d] < ix)) { v = rv[w][d]; ix = ri[w][d]; }
            ext_v[kDirs * (size_t)t + d] = v;
            ext_i[kDirs * (size_t)t + d] = ix;
        }
        __syncthreads();
    }
}

// ---- C: per-cluster extreme polygon -----------------------------------------------
// poly layout per cluster (kPolyWords doubles): u[kDirs], v[kDirs], margin,
// vertex count (-1: no polygon for the cluster, 0: no filtering)
__global__ void __launch_bounds__(kBlock) k_hull_poly(const uint32_t* __restrict__ small,
                                                     const uint32_t* __restrict__ tile_off,
                                                     const uint32_t* __restrict__ off, const float* __restrict__ X,
                                                     const float* __restrict__ Y, const float* __restrict__ Z,
                                                     const float4* __restrict__ plane,
                                                     const uint32_t* __restrict__ in_off,
                                                     const uint32_t* __restrict__ in_idx,
                                                     const double* __restrict__ ext_v,
                                                     const uint32_t* __restrict__ ext_i, double* __restrict__ poly,
                                                     uint32_t* __restrict__ surv_cnt)
{
    const uint32_t K = small[4];
    const uint32_t T = small[6];
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (kBlock / kWave);
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave);
    for (uint32_t k = w0; k < K; k += waves) {   // a wave per cluster (wave-uniform index: scalar loads)
        const uint32_t t0 = tile_off[k], t1 = tiles_end(tile_off, k, K, T);
        if (lane == 0) surv_cnt[k] = 0;
        double* P = poly + kPolyWords * (size_t)k;
        if (t0 == t1) {
            if (lane == 0) P[kPolyWords - 1] = -1.0;
            continue;
        }
        // the wave strides over the cluster's tiles, then reduces each direction
        double bv[kDirs];
        uint32_t bi[kDirs];
#pragma unroll
        for (int d = 0; d < kDirs; ++d) { bv[d] = -INFINITY; bi[d] = 0xFFFFFFFFu; }
        for (uint32_t t = t0 + lane; t < t1; t += kWave) {
#pragma unroll
            for (int d = 0; d < kDirs; ++d) {
                const double tv = ext_v[kDirs * (size_t)t + d];
                const uint32_t ti = ext_i[kDirs * (size_t)t + d];
                if (tv > bv[d] || (tv == bv[d] && ti < bi[d])) { bv[d] = tv; bi[d] = ti; }
            }
        }
        uint32_t e[kDirs];
#pragma unroll
        for (int d = 0; d < kDirs; ++d) {
            for (int sft = kWave / 2; sft >= 1; sft >>= 1) {
                const double ov = __shfl_xor(bv[d], sft, kWave);
                const uint32_t oi = __shfl_xor(bi[d], sft, kWave);
                if (ov > bv[d] || (ov == bv[d] && oi < bi[d])) { bv[d] = ov; bi[d] = oi; }
            }
            e[d] = bi[d];
        }
        if (lane == 0) {
            const ClusterFrame f = cluster_frame(k, off, X, Y, Z, plane, in_off, in_idx);
            extreme_polygon(e, f.m, P, [&](uint32_t j, double* pu, double* pv) {
                const uint32_t i = f.pb + in_idx[f.ib + j];
                project(f, X[i], Y[i], Z[i], pu, pv);
            });
        }
    }
}

// ---- D: survivors of the polygon test, compacted per cluster ---------------------
__global__ void __launch_bounds__(kTileThreads) k_hull_filter(
    const uint32_t* __restrict__ small, const uint32_t* __restrict__ tile_off, const uint32_t* __restrict__ off,
    const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
    const float4* __restrict__ plane, const uint32_t* __restrict__ in_off, const uint32_t* __restrict__ in_idx,
    const double* __restrict__ poly, uint32_t* __restrict__ surv_cnt, double* __restrict__ gu,
    double* __restrict__ gv, uint32_t* __restrict__ gi)
{
    __shared__ double P[kPolyWords];
    __shared__ uint32_t lcount, lbase;
    const uint32_t K = small[4];
    const uint32_t T = small[6];
    for (uint32_t t = blockIdx.x; t < T; t += gridDim.x) {
        const uint32_t k = cluster_of_tile(tile_off, K, t);
        if (threadIdx.x < kPolyWords) P[threadIdx.x] = poly[kPolyWords * (size_t)k + threadIdx.x];
        if (threadIdx.x == 0) lcount = 0;
        __syncthreads();
        const ClusterFrame f = cluster_frame(k, off, X, Y, Z, plane, in_off, in_idx);
        const uint32_t j0 = (t - tile_off[k]) * kHullTile;
        const int np = (int)P[kPolyWords - 1];
        const double mg = P[kPolyWords - 2];
        double su[kTileItems], sv[kTileItems];
        uint32_t sj[kTileItems], slot[kTileItems];
        int ns = 0;
#pragma unroll
        for (int it = 0; it < kTileItems; ++it) {
            const uint32_t j = j0 + it * kTileThreads + threadIdx.x;
            if (j >= f.m) continue;
            const uint32_t li = in_idx[f.ib + j];
            if (li >= f.nk) continue;
            const uint32_t i = f.pb + li;
            double pu, pv;
            project(f, X[i], Y[i], Z[i], &pu, &pv);
            bool inside = np >= 3;
            for (int a = 0; inside && a < np; ++a) {
                const int b = (a + 1 == np) ? 0 : a + 1;
                inside = cross3(P[a], P[kDirs + a], P[b], P[kDirs + b], pu, pv) > mg;
            }
            if (!inside) {
                su[ns] = pu;
                sv[ns] = pv;
                sj[ns] = j;
                slot[ns] = atomicAdd(&lcount, 1u);
                ++ns;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) lbase = lcount ? atomicAdd(&surv_cnt[k], lcount) : 0u;
        __syncthreads();
        for (int a = 0; a < ns; ++a) {
            const uint32_t dst = f.ib + lbase + slot[a];
            gu[dst] = su[a];
            gv[dst] = sv[a];
            gi[dst] = sj[a];
        }
        __syncthreads();
    }
}

// Filtered clusters whose survivors need a workgroup: up to kMidMax of them
// go to the mid list (stored from the end of the list buffer, count in
// small[9]) for k_hull_small, more to the chain list (count in small[7]) for
// k_hull_chain.  The two never meet: together they hold at most K <= cap
// entries.
constexpr uint32_t kMidMax = kChainBlock;
static_assert(kBlock == kChainBlock, "k_hull_small runs the workgroup chain with its own workgroup");

__global__ void __launch_bounds__(kBlock) k_hull_list(uint32_t* __restrict__ small,
                                                      const uint32_t* __restrict__ tile_off,
                                                      const uint32_t* __restrict__ surv_cnt,
                                                      uint32_t* __restrict__ list, uint32_t cap)
{
    const uint32_t K = small[4];
    const uint32_t T = small[6];
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        if (tile_off[k] == tiles_end(tile_off, k, K, T)) continue;   // not filtered: the wave path
        const uint32_t ns = surv_cnt[k];
        if (ns <= (uint32_t)kWave) continue;
        if (ns <= kMidMax) list[cap - 1u - atomicAdd(&small[9], 1u)] = k;
        else list[atomicAdd(&small[7], 1u)] = k;
    }
}

// Clusters with at most 64 points to chain -- survivors of the filter, or
// (clusters the filter skips) all inliers, projected here exactly as the
// filter projects them -- one wave each, four per workgroup.  The points are
// sorted across the wave's lanes (bitonic network on shuffles, same order:
// u, then v, then inlier position), then one lane runs the lower and the
// upper chain; the result is the same as the workgroup path's.  Up to half
// of the workgroups first take the mid list's clusters (65..kMidMax
// survivors) with the workgroup chain, so that those serial chains run while
// the other workgroups go through the small clusters instead of in a launch
// of their own afterwards; the rest split the small clusters among their
// waves.
__global__ void __launch_bounds__(kBlock) k_hull_small(
    uint32_t* __restrict__ small, const uint32_t* __restrict__ list, uint32_t cap, const uint32_t* __restrict__ tile_off,
    const uint32_t* __restrict__ off,
    const float* __restrict__ X, const float* __restrict__ Y, const float* __restrict__ Z,
    const float4* __restrict__ plane, const int32_t* __restrict__ best, uint32_t in_cap,
    const uint32_t* __restrict__ in_off, const uint32_t* __restrict__ in_idx, const uint32_t* __restrict__ surv_cnt,
    const double* __restrict__ gu, const double* __restrict__ gv, const uint32_t* __restrict__ gi,
    uint32_t* __restrict__ hull_cnt, uint32_t* __restrict__ hull_tmp, double* __restrict__ area_out)
{
    __shared__ double su[kBlock / kWave][kWave];
    __shared__ double sv[kBlock / kWave][kWave];
    __shared__ uint32_t si[kBlock / kWave][kWave];
    __shared__ uint8_t st[kBlock / kWave][2 * kWave + 2];
    __shared__ ChainLds<kMidMax> L;
    const uint32_t K = small[4];
    const uint32_t T = small[6];
    const uint32_t nmid = small[9];
    const uint32_t gmid = nmid < gridDim.x / 2 ? nmid : gridDim.x / 2;   // uniform over the grid
    if (blockIdx.x < gmid) {
        for (uint32_t c = blockIdx.x; c < nmid; c += gmid) {
            const uint32_t k = list[cap - 1u - c];
            const uint32_t ib = in_off[k];
            const uint32_t ns = surv_cnt[k];   // 65..kMidMax
            double area = 0.0;
            const uint32_t hh = block_chain(L, ns,
                                            [&](uint32_t t, double* u, double* v, uint32_t* id) {
                                                *u = gu[ib + t];
                                                *v = gv[ib + t];
                                                *id = gi[ib + t];
                                            },
                                            [&](uint32_t q, uint32_t p) { hull_tmp[ib + k + q] = in_idx[ib + L.si[p]]; },
                                            &area);
            if (threadIdx.x == 0) {
                area_out[k] = area;
                hull_cnt[k] = hh;
            }
            __syncthreads();   // L is reused by the next cluster
        }
        return;
    }
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint32_t waves = (gridDim.x - gmid) * (kBlock / kWave);
    // wave-uniform cluster index: the cluster's own loads become scalar
    const uint32_t w0 = __builtin_amdgcn_readfirstlane((blockIdx.x - gmid) * (kBlock / kWave) + wv);
    for (uint32_t k = w0; k < K; k += waves) {
        const bool tiled = tile_off[k] != tiles_end(tile_off, k, K, T);
        uint32_t ns;
        double u = INFINITY, v = INFINITY;
        uint32_t i = 0xFFFFFFFFu;
        const uint32_t ib = in_off[k];
        if (tiled) {
            ns = surv_cnt[k];
            if (ns > (uint32_t)kWave) continue;   // listed for a workgroup chain
            if ((uint32_t)lane < ns) {
                u = gu[ib + lane];
                v = gv[ib + lane];
                i = gi[ib + lane];
            }
        } else {
            if (!cluster_ok(k, off, best, in_off, in_idx, in_cap)) {   // no polygon
                if (lane == 0) {
                    hull_cnt[k] = 0;
                    area_out[k] = 0.0;
                }
                continue;
            }
            ns = in_off[k + 1] - ib;
            const ClusterFrame f = cluster_frame(k, off, X, Y, Z, plane, in_off, in_idx);
            if ((uint32_t)lane < ns) {
                const uint32_t p = f.pb + in_idx[ib + lane];
                project(f, X[p], Y[p], Z[p], &u, &v);
                i = (uint32_t)lane;
            }
        }
        const WaveHull r = wave_hull(u, v, i, ns, lane, su[wv], sv[wv], si[wv], st[wv]);
        if (lane == 0) {
            area_out[k] = r.area;
            hull_cnt[k] = r.h;
        }
        if ((uint32_t)lane < r.h) hull_tmp[ib + k + lane] = in_idx[ib + si[wv][r.vi]];
        __builtin_amdgcn_wave_barrier();
    }
}

// Survivor sets of more than kRefineMin points are thinned once more before sorting:
// the extremes of the survivors in kRefineDirs directions (every 360/64
// degrees, counter-clockwise) bound a convex polygon inside the hull, and the
// survivors strictly inside it (by the same margin as the octagon's) are
// dropped.  The hull of what is left is the same polygon, since every vertex
// survives; a disc keeps about 0.2 % of its points outside a 64-gon.
constexpr int kRefineDirs = 64;
constexpr uint32_t kRefineMin = 512;   // survivor sets above this are refined (a few passes beat a long sort)
constexpr int kRefineBatch = 8;   // directions reduced per pass over the survivors

struct RefineLds {
    double rv[kChainBlock / kWave][kRefineBatch];
    uint32_t ri[kChainBlock / kWave][kRefineBatch];
    uint32_t ext[kRefineDirs];
    double pu[kRefineDirs], pv[kRefineDirs];
    double margin;
    int np;
    uint32_t wcnt[kChainBlock / kWave];
};

// compacts U/V/I[0, ns) in place to the points not strictly inside the
// refinement polygon; returns their number (every thread of the block calls it)
__device__ uint32_t refine_survivors(RefineLds& R, double* U, double* V, uint32_t* I, uint32_t ns)
{
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (int d0 = 0; d0 < kRefineDirs; d0 += kRefineBatch) {
        double cs[kRefineBatch], sn[kRefineBatch], bv[kRefineBatch];
        uint32_t bi[kRefineBatch];
#pragma unroll
        for (int j = 0; j < kRefineBatch; ++j) {
            sincospi((double)(d0 + j) / (kRefineDirs / 2), &sn[j], &cs[j]);
            bv[j] = -INFINITY;
            bi[j] = 0xFFFFFFFFu;
        }
        for (uint32_t t = threadIdx.x; t < ns; t += kChainBlock) {
            const double u = U[t], v = V[t];
#pragma unroll
            for (int j = 0; j < kRefineBatch; ++j) {
                const double val = u * cs[j] + v * sn[j];
                if (val > bv[j]) {   // t ascends per thread: the first maximum is kept
                    bv[j] = val;
                    bi[j] = t;
                }
            }
        }
        // the largest value, lowest position on ties
#pragma unroll
        for (int j = 0; j < kRefineBatch; ++j) {
            for (int o = kWave / 2; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv[j], o, kWave);
                const uint32_t oi = __shfl_xor(bi[j], o, kWave);
                if (ov > bv[j] || (ov == bv[j] && oi < bi[j])) {
                    bv[j] = ov;
                    bi[j] = oi;
                }
            }
            if (lane == 0) {
                R.rv[wv][j] = bv[j];
                R.ri[wv][j] = bi[j];
            }
        }
        __syncthreads();
        if (threadIdx.x < kRefineBatch) {
            const int j = threadIdx.x;
            double b = R.rv[0][j];
            uint32_t i = R.ri[0][j];
            for (int w = 1; w < kChainBlock / kWave; ++w)
                if (R.rv[w][j] > b || (R.rv[w][j] == b && R.ri[w][j] < i)) {
                    b = R.rv[w][j];
                    i = R.ri[w][j];
                }
            R.ext[d0 + j] = i;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // the extremes in direction order, repeats merged, then pruned to
        // strictly convex corners (as the octagon is)
        int np = 0;
        for (int d = 0; d < kRefineDirs; ++d)   // in place: np <= d
            if (R.ext[d] < ns && (np == 0 || R.ext[np - 1] != R.ext[d])) R.ext[np++] = R.ext[d];
        while (np > 1 && R.ext[np - 1] == R.ext[0]) --np;
        double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
        for (int a = 0; a < np; ++a) {
            R.pu[a] = U[R.ext[a]];
            R.pv[a] = V[R.ext[a]];
            umin = fmin(umin, R.pu[a]);
            umax = fmax(umax, R.pu[a]);
            vmin = fmin(vmin, R.pv[a]);
            vmax = fmax(vmax, R.pv[a]);
        }
        const double span = np > 0 ? fmax(umax - umin, vmax - vmin) : 0.0;
        const double margin = 1e-9 * span * span + 1e-300;
        for (bool changed = np >= 3; changed && np >= 3;) {
            changed = false;
            for (int a = 0; a < np && np >= 3; ++a) {
                const int b = (a + 1) % np, c = (a + 2) % np;
                if (cross3(R.pu[a], R.pv[a], R.pu[b], R.pv[b], R.pu[c], R.pv[c]) <= margin) {
                    for (int r = b; r + 1 < np; ++r) {
                        R.pu[r] = R.pu[r + 1];
                        R.pv[r] = R.pv[r + 1];
                    }
                    --np;
                    changed = true;
                }
            }
        }
        R.margin = margin;
        R.np = np;
    }
    __syncthreads();
    const int np = R.np;
    if (np < 3) return ns;
    const double mg = R.margin;
    // in-place compaction, a block-wide chunk at a time: every thread of a
    // chunk has read its point before any is written, and writes land at or
    // below the chunk's positions
    uint32_t nout = 0;
    for (uint32_t base = 0; base < ns; base += kChainBlock) {
        const uint32_t t = base + threadIdx.x;
        double u = 0.0, v = 0.0;
        uint32_t id = 0;
        bool keep = false;
        if (t < ns) {
            u = U[t];
            v = V[t];
            id = I[t];
            bool inside = true;
            for (int a = 0; inside && a < np; ++a) {
                const int b = a + 1 == np ? 0 : a + 1;
                inside = cross3(R.pu[a], R.pv[a], R.pu[b], R.pv[b], u, v) > mg;
            }
            keep = !inside;
        }
        const uint64_t bal = __ballot(keep);
        const uint32_t below = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) R.wcnt[wv] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t pre = 0, tot = 0;
        for (int w = 0; w < kChainBlock / kWave; ++w) {
            if (w < wv) pre += R.wcnt[w];
            tot += R.wcnt[w];
        }
        if (keep) {
            const uint32_t o = nout + pre + below;
            U[o] = u;
            V[o] = v;
            I[o] = id;
        }
        nout += tot;
        __syncthreads();
    }
    return nout;
}

__global__ void __launch_bounds__(kChainBlock) k_hull_chain(
    const uint32_t* __restrict__ small, const uint32_t* __restrict__ chain_list, const uint32_t* __restrict__ in_off,
    const uint32_t* __restrict__ in_idx, const uint32_t* __restrict__ surv_cnt, double* __restrict__ gu,
    double* __restrict__ gv, uint32_t* __restrict__ gi, uint32_t* __restrict__ hull_cnt,
    uint32_t* __restrict__ hull_tmp, double* __restrict__ area_out)
{
    __shared__ ChainLds<kLdsCap> L;
    __shared__ RefineLds R;
    // the listed clusters: more than kMidMax survivors (k_hull_list), or the
    // persistent pass's clusters with more than one wave of survivors
    const uint32_t nc = small[7];
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const uint32_t k = chain_list[c];
        const uint32_t ib = in_off[k];
        uint32_t ns = surv_cnt[k];
        if (ns > kRefineMin) ns = refine_survivors(R, gu + ib, gv + ib, gi + ib, ns);
        if (ns <= (uint32_t)kLdsCap) {
            double area = 0.0;
            const uint32_t hh = block_chain(L, ns,
                                            [&](uint32_t t, double* u, double* v, uint32_t* id) {
                                                *u = gu[ib + t];
                                                *v = gv[ib + t];
                                                *id = gi[ib + t];
                                            },
                                            [&](uint32_t q, uint32_t p) { hull_tmp[ib + k + q] = in_idx[ib + L.si[p]]; },
                                            &area);
            if (threadIdx.x == 0) {
                area_out[k] = area;
                hull_cnt[k] = hh;
            }
        } else {
            // bitonic network in global memory; partners beyond ns are +infinity
            uint32_t N = 1;
            while (N < ns) N <<= 1;
            double* U = gu + ib;
            double* Vv = gv + ib;
            uint32_t* I = gi + ib;
            for (uint32_t size = 2; size <= N; size <<= 1) {
                for (uint32_t t = threadIdx.x; t < N / 2; t += kChainBlock) {
                    const uint32_t blk = t / (size >> 1), r = t % (size >> 1);
                    const uint32_t a = blk * size + r, b = blk * size + size - 1 - r;
                    if (b < ns && p2_less(U[b], Vv[b], I[b], U[a], Vv[a], I[a])) swap3(U, Vv, I, a, b);
                }
                __syncthreads();
                for (uint32_t stride = size >> 2; stride > 0; stride >>= 1) {
                    for (uint32_t t = threadIdx.x; t < N / 2; t += kChainBlock) {
                        const uint32_t a = 2 * t - (t & (stride - 1)), b = a + stride;
                        if (b < ns && p2_less(U[b], Vv[b], I[b], U[a], Vv[a], I[a])) swap3(U, Vv, I, a, b);
                    }
                    __syncthreads();
                }
            }
            if (threadIdx.x == 0) {
                // single-stack chain; cluster k's stack is hull_tmp[ib + k, ib + k + m + 1)
                // and never holds more than ns + 1 <= m + 1 entries
                uint32_t* st = hull_tmp + ib + k;
                uint32_t h = 0;
                for (uint32_t i = 0; i < ns; ++i) {
                    while (h >= 2) {
                        const uint32_t a = st[h - 2], b = st[h - 1];
                        if (cross3(U[a], Vv[a], U[b], Vv[b], U[i], Vv[i]) <= 0.0) --h;
                        else break;
                    }
                    st[h++] = i;
                }
                const uint32_t lower = h + 1;
                for (int32_t i = (int32_t)ns - 2; i >= 0; --i) {
                    while (h >= lower) {
                        const uint32_t a = st[h - 2], b = st[h - 1];
                        if (cross3(U[a], Vv[a], U[b], Vv[b], U[i], Vv[i]) <= 0.0) --h;
                        else break;
                    }
                    st[h++] = (uint32_t)i;
                }
                --h;   // the last point repeats the first
                double s = 0.0;
                if (h >= 3) {
                    for (uint32_t q = 0; q < h; ++q) {
                        const uint32_t p0 = st[q], p1 = st[q + 1 == h ? 0 : q + 1];
                        s = s + (U[p0] * Vv[p1] - U[p1] * Vv[p0]);
                    }
                }
                area_out[k] = h >= 3 ? 0.5 * s : 0.0;
                // entry q of the stack is read before slot q is overwritten
                for (uint32_t q = 0; q < h; ++q) hull_tmp[ib + k + q] = in_idx[ib + I[st[q]]];
                hull_cnt[k] = h;
            }
        }
        __syncthreads();
    }
}

// ---- F: pack --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_hull_pack(const uint32_t* __restrict__ small,
                                                      const uint32_t* __restrict__ off, const float* __restrict__ X,
                                                      const float* __restrict__ Y, const float* __restrict__ Z,
                                                      const float4* __restrict__ plane,
                                                      const uint32_t* __restrict__ in_off,
                                                      const uint32_t* __restrict__ hull_cnt,
                                                      const uint32_t* __restrict__ hull_tmp,
                                                      const uint32_t* __restrict__ v_scan, uint32_t v_cap,
                                                      uint32_t* __restrict__ v_off, uint32_t* __restrict__ v_idx,
                                                      float* __restrict__ v_xyz, uint32_t* __restrict__ status)
{
    const uint32_t K = small[4];
    bool over = false;
    for (uint32_t k = blockIdx.x; k < K; k += gridDim.x) {
        const uint32_t h = hull_cnt[k];
        const uint32_t base = v_scan[k];
        if (threadIdx.x == 0) v_off[k] = base;
        if (h == 0) continue;
        const float4 pl = plane[k];
        const double nx = pl.x, ny = pl.y, nz = pl.z, d = pl.w;
        const uint32_t ib = in_off[k], pb = off[k];
        for (uint32_t q = threadIdx.x; q < h; q += blockDim.x) {
            const uint32_t pos = base + q;
            if (pos >= v_cap) {
                over = true;
                continue;
            }
            const uint32_t j = hull_tmp[ib + k + q];
            const double px = X[pb + j], py = Y[pb + j], pz = Z[pb + j];
            const double dist = nx * px + ny * py + nz * pz + d;
            v_idx[pos] = j;
            v_xyz[3 * (size_t)pos + 0] = (float)(px - dist * nx);
            v_xyz[3 * (size_t)pos + 1] = (float)(py - dist * ny);
            v_xyz[3 * (size_t)pos + 2] = (float)(pz - dist * nz);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) v_off[K] = small[5];
    if (over) atomicOr(status, (uint32_t)VM_FLAG_HULL_CAP);
}

}  // namespace

hipError_t launch_hull_chain_list(const uint32_t* small, const uint32_t* list, const uint32_t* in_off,
                                  const uint32_t* in_idx, const uint32_t* surv_cnt, double* gu, double* gv, uint32_t* gi,
                                  uint32_t* hull_cnt, uint32_t* hull_tmp, double* area_out, uint32_t grid, hipStream_t s)
{
    k_hull_chain<<<grid ? grid : 1, kChainBlock, 0, s>>>(small, list, in_off, in_idx, surv_cnt, gu, gv, gi, hull_cnt,
                                                         hull_tmp, area_out);
    return hipGetLastError();
}

uint64_t hull_tiles_bound(uint32_t k_cap, uint32_t n_cap)
{
    return (uint64_t)n_cap / kHullTile + (uint64_t)k_cap + 2;
}

vm_status hulls(const vm_clusters& cl, const vm_planes& planes, const vm_hulls_out& out, const WorkLayout& w,
                hipStream_t s)
{
    uint32_t kc = cl.k_cap;
    if (planes.k_cap < kc) kc = planes.k_cap;
    if (out.k_cap < kc) kc = out.k_cap;
    if (kc > w.k_cap) return VM_E_STATE;
    StageScope t(VM_STAGE_HULL, s);
    const float4* pl = (const float4*)planes.d_plane;
    if (kc <= kOneBlockMax) {
        k_hull_prepare<<<1, kOneBlockThreads, 0, s>>>(cl.d_meta, kc, cl.n_cap, cl.d_off, planes.d_best_h,
                                                      planes.d_in_off, planes.d_in_idx, planes.in_cap, w.small,
                                                      w.hull_tile_off, out.d_status);
    } else {
        k_hull_validate<<<1, kBlock, 0, s>>>(cl.d_meta, kc, cl.n_cap, cl.d_off, w.small, out.d_status);
        k_hull_tiles<<<grid_for(kc), kBlock, 0, s>>>(w.small, cl.d_off, planes.d_best_h, planes.d_in_off,
                                                     planes.d_in_idx, planes.in_cap, w.hull_tile_off, out.d_status);
        VM_HIP(scan_exclusive_dev(w.hull_tile_off, w.hull_tile_off, w.small + 4, kc, w.small + 6, w.blk, s));
    }
    // grids sized for a few workgroups per CU; the kernels stride over the
    // device-side counts, so empty workgroups are not launched by the thousand
    const int tgrid = grid_for(hull_tiles_bound(kc, cl.n_cap), 1, 2048);
    k_hull_extremes<<<tgrid, kTileThreads, 0, s>>>(w.small, w.hull_tile_off, cl.d_off, cl.d_x, cl.d_y, cl.d_z, pl,
                                                   planes.d_in_off, planes.d_in_idx, w.ext_v, w.ext_i);
    const int kgrid = kc < 1024 ? (int)(kc ? kc : 1) : 1024;
    const int cgrid = kc < 512 ? (int)(kc ? kc : 1) : 512;   // the chain kernel holds ~70 KB of LDS
    k_hull_poly<<<kSmallGrid, kBlock, 0, s>>>(w.small, w.hull_tile_off, cl.d_off, cl.d_x, cl.d_y, cl.d_z, pl,
                                        planes.d_in_off, planes.d_in_idx, w.ext_v, w.ext_i, w.poly, w.surv_cnt);
    k_hull_filter<<<tgrid, kTileThreads, 0, s>>>(w.small, w.hull_tile_off, cl.d_off, cl.d_x, cl.d_y, cl.d_z, pl,
                                                 planes.d_in_off, planes.d_in_idx, w.poly, w.surv_cnt, w.hull_u,
                                                 w.hull_v, w.hull_i);
    k_hull_list<<<grid_for(kc), kBlock, 0, s>>>(w.small, w.hull_tile_off, w.surv_cnt, w.chain_list, kc);
    k_hull_small<<<kSmallGrid, kBlock, 0, s>>>(w.small, w.chain_list, kc, w.hull_tile_off, cl.d_off, cl.d_x, cl.d_y,
                                              cl.d_z, pl,
                                              planes.d_best_h, planes.in_cap, planes.d_in_off, planes.d_in_idx,
                                              w.surv_cnt, w.hull_u, w.hull_v, w.hull_i, w.hull_cnt, w.hull_tmp,
                                              out.d_area);
    k_hull_chain<<<cgrid, kChainBlock, 0, s>>>(w.small, w.chain_list, planes.d_in_off, planes.d_in_idx, w.surv_cnt,
                                               w.hull_u, w.hull_v, w.hull_i, w.hull_cnt, w.hull_tmp, out.d_area);
    VM_HIP(hipGetLastError());
    VM_HIP(scan_exclusive_dev(w.hull_cnt, w.hull_off, w.small + 4, kc, w.small + 5, w.blk, s));
    k_hull_pack<<<kgrid, kBlock, 0, s>>>(w.small, cl.d_off, cl.d_x, cl.d_y, cl.d_z, pl, planes.d_in_off, w.hull_cnt,
                                         w.hull_tmp, w.hull_off, out.v_cap, out.d_v_off, out.d_v_idx, out.d_v_xyz,
                                         out.d_status);
    VM_HIP(hipGetLastError());
    return VM_OK;
}

}  // namespace vm

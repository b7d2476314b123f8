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

#include <math.h>

namespace vm {
namespace {

constexpr int kTileThreads = 256;
constexpr int kTileItems = 4;
constexpr int kHullTile = kTileThreads * kTileItems;   // inliers per tile
constexpr int kChainBlock = 256;
constexpr int kSmallGrid = 2048;   // workgroups of the wave-per-cluster kernels (8192 waves)
constexpr int kLdsCap = 2048;                           // survivors sorted in LDS

__device__ __forceinline__ bool p2_less(double au, double av, uint32_t ai, double bu, double bv, uint32_t bi)
{
    if (au != bu) return au < bu;
    if (av != bv) return av < bv;
    return ai < bi;
}

__device__ __forceinline__ double cross3(double ou, double ov, double au, double av, double bu, double bv)
{
    return (au - ou) * (bv - ov) - (av - ov) * (bu - ou);
}

struct Basis {
    double u[3], v[3];
};

__device__ __forceinline__ Basis plane_basis(float4 pl)
{
    Basis b;
    const double n0 = pl.x, n1 = pl.y, n2 = pl.z;
    double a[3] = {0.0, 0.0, 0.0};
    if (fabs(n0) < 0.9) a[0] = 1.0;
    else a[1] = 1.0;
    const double c0 = a[1] * n2 - a[2] * n1;
    const double c1 = a[2] * n0 - a[0] * n2;
    const double c2 = a[0] * n1 - a[1] * n0;
    const double inv = 1.0 / sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    b.u[0] = c0 * inv;
    b.u[1] = c1 * inv;
    b.u[2] = c2 * inv;
    b.v[0] = n1 * b.u[2] - n2 * b.u[1];
    b.v[1] = n2 * b.u[0] - n0 * b.u[2];
    b.v[2] = n0 * b.u[1] - n1 * b.u[0];
    return b;
}

// directional functional of direction d (0..7, every 45 degrees, CCW from +u)
// Support directions of the extreme-point polygon, in counter-clockwise
// order (every 45 degrees).  A point strictly inside the polygon of the
// extremes is no hull vertex; a disc keeps about 10 % of its points outside
// this octagon.  (Sixteen directions keep 3 %, but the extra tests cost more
// than the shorter sorts save.)
constexpr int kDirs = kHullDirs;
constexpr int kPolyWords = 2 * kDirs + 2;   // u[kDirs], v[kDirs], margin, vertex count
static_assert(kDirs == 8, "dir_val lists 8 directions");

__device__ __forceinline__ double dir_val(int d, double u, double v)
{
    switch (d) {
        case 0: return u;
        case 1: return u + v;
        case 2: return v;
        case 3: return v - u;
        case 4: return -u;
        case 5: return -u - v;
        case 6: return -v;
        default: return u - v;
    }
}

// per-cluster constants of the passes over inliers
struct ClusterFrame {
    uint32_t ib, m, pb, nk;   // inlier offset/count, point offset/count
    Basis B;
    double ox, oy, oz;        // origin = first inlier
};

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

__device__ __forceinline__ void project(const ClusterFrame& f, float x, float y, float z, double* pu, double* pv)
{
    const double dx = (double)x - f.ox, dy = (double)y - f.oy, dz = (double)z - f.oz;
    *pu = f.B.u[0] * dx + f.B.u[1] * dy + f.B.u[2] * dz;
    *pv = f.B.v[0] * dx + f.B.v[1] * dy + f.B.v[2] * dz;
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
            int np = 0;
            uint32_t q[kDirs];
            bool found = true;
            for (int d = 0; d < kDirs; ++d) found = found && e[d] < f.m;
            for (int d = 0; found && d < kDirs; ++d)
                if (np == 0 || q[np - 1] != e[d]) q[np++] = e[d];
            while (np > 1 && q[np - 1] == q[0]) --np;
            double pu[kDirs], pv[kDirs];
            double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
            for (int a = 0; a < np; ++a) {
                const uint32_t i = f.pb + in_idx[f.ib + q[a]];
                project(f, X[i], Y[i], Z[i], &pu[a], &pv[a]);
                umin = fmin(umin, pu[a]);
                umax = fmax(umax, pu[a]);
                vmin = fmin(vmin, pv[a]);
                vmax = fmax(vmax, pv[a]);
            }
            const double span = np > 0 ? fmax(umax - umin, vmax - vmin) : 0.0;
            // far above the fp64 rounding of a cross product at this scale
            const double margin = 1e-9 * span * span + 1e-300;
            // vertices that do not turn left by more than the margin (on an
            // edge of the others, or repeated) are dropped until every corner
            // is strictly convex; the rest bound a convex polygon inside the
            // hull (fewer than 3: no filtering)
            for (bool changed = np >= 3; changed && np >= 3;) {
                changed = false;
                for (int a = 0; a < np && np >= 3; ++a) {
                    const int b = (a + 1) % np, c = (a + 2) % np;
                    if (cross3(pu[a], pv[a], pu[b], pv[b], pu[c], pv[c]) <= margin) {
                        for (int r = b; r + 1 < np; ++r) {
                            pu[r] = pu[r + 1];
                            pv[r] = pv[r + 1];
                        }
                        --np;
                        changed = true;
                    }
                }
            }
            for (int a = 0; a < kDirs; ++a) {
                P[a] = a < np ? pu[a] : 0.0;
                P[kDirs + a] = a < np ? pv[a] : 0.0;
            }
            P[2 * kDirs] = margin;
            P[2 * kDirs + 1] = np >= 3 ? (double)np : 0.0;
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

// ---- E: sort + monotone chain per cluster ------------------------------------------
__device__ __forceinline__ void swap3(double* U, double* V, uint32_t* I, uint32_t a, uint32_t b)
{
    const double tu = U[a], tv = V[a];
    const uint32_t ti = I[a];
    U[a] = U[b];
    V[a] = V[b];
    I[a] = I[b];
    U[b] = tu;
    V[b] = tv;
    I[b] = ti;
}

// One monotone chain over n sorted points (forward: lower chain, backward:
// upper chain), computed by one wave in three levels.  The first two levels
// drop only points that lie strictly on the inner side of a segment between
// two other points (such a point is no vertex of the hull of any set holding
// those three; collinear and coincident points are kept, so the choice among
// them is left to the full rule):
//   level 1: lane l chains its contiguous chunk of the n points into tmp,
//            and the chunk results are concatenated into seq;
//   level 2: lane w < 8 chains the concatenated results of chunks 8w..8w+7
//            in place;
//   level 3: one thread runs the full chain (dropping collinear and
//            coincident points as well) over the level-2 results in order,
//            which gives the output of the plain chain over all n points.
constexpr int kChainL2 = 8;   // level-2 windows (of kWave / kChainL2 chunks each)

template <typename S>
__device__ __forceinline__ void chain_level1(const double* U, const double* V, uint32_t n, bool forward, S* tmp,
                                             S* seq, uint32_t* offs)
{
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t c = (n + kWave - 1) / kWave;
    const uint32_t s0 = lane * c < n ? lane * c : n;
    const uint32_t s1 = s0 + c < n ? s0 + c : n;
    uint32_t h = 0;
    for (uint32_t s = s0; s < s1; ++s) {
        const uint32_t i = forward ? s : n - 1 - s;
        while (h >= 2) {
            const uint32_t a = tmp[s0 + h - 2], b = tmp[s0 + h - 1];
            if (cross3(U[a], V[a], U[b], V[b], U[i], V[i]) < 0.0) --h;
            else break;
        }
        tmp[s0 + h++] = (S)i;
    }
    // concatenate the chunk results into seq (wave prefix sum of the lengths)
    uint32_t inc = h;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, kWave);
        if ((int)lane >= d) inc += t;
    }
    const uint32_t off = inc - h;
    for (uint32_t q = 0; q < h; ++q) seq[off + q] = tmp[s0 + q];
    offs[lane] = off;
    if (lane == kWave - 1) offs[kWave] = inc;
}

// One thread's chain over the points idx[0..m) (indices into U, V) in that
// order: a point pops the stack top while it turns right of the top two
// (strict: only strictly right; otherwise also collinear and repeated
// points); the kept indices go to out[0..h) and h is returned.  out may be
// idx itself (a store lands at or below the read position).  The two top
// entries' coordinates stay in registers, the next point's coordinates and
// the index after it are loaded a step ahead, so a step waits for one LDS
// load at most when it does not pop.
template <bool kStrict, typename S>
__device__ __forceinline__ uint32_t chain_run(const double* U, const double* V, const S* idx, uint32_t m, S* out)
{
    uint32_t h = 0;
    double au = 0.0, av = 0.0, bu = 0.0, bv = 0.0;   // out[h - 2], out[h - 1]
    uint32_t i1 = m > 0 ? (uint32_t)idx[0] : 0u;
    double u1 = m > 0 ? U[i1] : 0.0, v1 = m > 0 ? V[i1] : 0.0;
    uint32_t i2 = m > 1 ? (uint32_t)idx[1] : 0u;
    for (uint32_t j = 0; j < m; ++j) {
        const uint32_t i = i1;
        const double iu = u1, iv = v1;
        if (j + 1 < m) {
            i1 = i2;
            u1 = U[i1];
            v1 = V[i1];
        }
        if (j + 2 < m) i2 = idx[j + 2];
        while (h >= 2) {
            const double c = cross3(au, av, bu, bv, iu, iv);
            if (!(kStrict ? c < 0.0 : c <= 0.0)) break;
            --h;
            bu = au;
            bv = av;
            if (h >= 2) {
                const uint32_t a = out[h - 2];
                au = U[a];
                av = V[a];
            }
        }
        out[h] = (S)i;
        if (h >= 1) {
            au = bu;
            av = bv;
        }
        bu = iu;
        bv = iv;
        ++h;
    }
    return h;
}

// level 2 for window w (called by one lane per window), in place; returns
// its length
template <typename S>
__device__ __forceinline__ uint32_t chain_level2(const double* U, const double* V, S* seq, const uint32_t* offs,
                                                 uint32_t w)
{
    const uint32_t a0 = offs[w * (kWave / kChainL2)], a1 = offs[(w + 1) * (kWave / kChainL2)];
    return chain_run<true>(U, V, seq + a0, a1 - a0, seq + a0);
}

// the level-2 results of all windows, in order, copied to dst by the
// threads of the workgroup; returns their total
template <typename S>
__device__ __forceinline__ uint32_t chain_gather2(const S* seq, const uint32_t* offs, const uint32_t* len2, S* dst)
{
    uint32_t pre = 0;
    for (uint32_t w = 0; w < (uint32_t)kChainL2; ++w) {
        const uint32_t a0 = offs[w * (kWave / kChainL2)], m = len2[w];
        for (uint32_t q = threadIdx.x; q < m; q += blockDim.x) dst[pre + q] = seq[a0 + q];
        pre += m;
    }
    return pre;
}

// Clusters with at most 64 points to chain -- survivors of the filter, or
// (clusters the filter skips) all inliers, projected here exactly as the
// filter projects them -- one wave each, four per workgroup.  The points are
// sorted across the wave's lanes (bitonic network on shuffles, same order:
// u, then v, then inlier position), then one lane runs the lower and the
// upper chain; the result is the same as the workgroup path's.
__global__ void __launch_bounds__(kBlock) k_hull_small(
    uint32_t* __restrict__ small, uint32_t* __restrict__ chain_list, const uint32_t* __restrict__ tile_off,
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
    const uint32_t K = small[4];
    const uint32_t T = small[6];
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint32_t waves = gridDim.x * (kBlock / kWave);
    // wave-uniform cluster index: the cluster's own loads become scalar
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / kWave) + wv);
    for (uint32_t k = w0; k < K; k += waves) {
        const bool tiled = tile_off[k] != tiles_end(tile_off, k, K, T);
        uint32_t ns;
        double u = INFINITY, v = INFINITY;
        uint32_t i = 0xFFFFFFFFu;
        const uint32_t ib = in_off[k];
        if (tiled) {
            ns = surv_cnt[k];
            if (ns > (uint32_t)kWave) {   // the workgroup path takes it from the list
                if (lane == 0) chain_list[atomicAdd(&small[7], 1u)] = k;
                continue;
            }
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
        for (int kk = 2; kk <= kWave; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                const double ou = __shfl_xor(u, j, kWave), ov = __shfl_xor(v, j, kWave);
                const uint32_t oi = __shfl_xor(i, j, kWave);
                const bool up = (lane & kk) == 0, low = (lane & j) == 0;
                const bool mine_less = p2_less(u, v, i, ou, ov, oi);
                if ((low == up) != mine_less) {
                    u = ou;
                    v = ov;
                    i = oi;
                }
            }
        }
        su[wv][lane] = u;
        sv[wv][lane] = v;
        si[wv][lane] = i;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // lane 0 builds the lower chain (points in sorted order), lane 1 at
        // the same time the upper one (reverse order), each with the two top
        // points of its stack held in registers
        uint32_t h = 0;
        if (lane < 2) {
            const double* U = su[wv];
            const double* V = sv[wv];
            uint8_t* S = st[wv] + (lane ? kWave + 1 : 0);
            double ua = 0.0, va = 0.0, ub = 0.0, vb = 0.0;   // S[h - 2], S[h - 1]
            for (uint32_t n = 0; n < ns; ++n) {
                const uint32_t q = lane ? ns - 1 - n : n;
                const double uq = U[q], vq = V[q];
                while (h >= 2 && cross3(ua, va, ub, vb, uq, vq) <= 0.0) {
                    --h;
                    ub = ua;
                    vb = va;
                    if (h >= 2) {
                        const uint32_t s2 = S[h - 2];
                        ua = U[s2];
                        va = V[s2];
                    }
                }
                S[h++] = (uint8_t)q;
                ua = ub;
                va = vb;
                ub = uq;
                vb = vq;
            }
        }
        const uint32_t hl = __shfl(h, 0, kWave), hu = __shfl(h, 1, kWave);
        // the polygon: the lower chain, then the upper one without its end
        // points (the lower chain's last and first points)
        h = hl + (hu >= 2 ? hu - 2 : 0u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        auto vertex = [&](uint32_t p) -> uint32_t {
            return p < hl ? st[wv][p] : st[wv][kWave + 1 + (p - hl + 1)];
        };
        double term = 0.0;
        uint32_t vi = 0;
        if ((uint32_t)lane < h) {
            vi = vertex((uint32_t)lane);
            const uint32_t v1 = vertex((uint32_t)lane + 1 == h ? 0u : (uint32_t)lane + 1);
            term = su[wv][vi] * sv[wv][v1] - su[wv][v1] * sv[wv][vi];
        }
        // shoelace sum over the vertices (a wave reduction)
#pragma unroll
        for (int dd = kWave / 2; dd >= 1; dd >>= 1) term += __shfl_xor(term, dd, kWave);
        if (lane == 0) {
            area_out[k] = h >= 3 ? 0.5 * term : 0.0;
            hull_cnt[k] = h;
        }
        if ((uint32_t)lane < h) hull_tmp[ib + k + lane] = in_idx[ib + si[wv][vi]];
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void __launch_bounds__(kChainBlock) k_hull_chain(
    const uint32_t* __restrict__ small, const uint32_t* __restrict__ chain_list, const uint32_t* __restrict__ in_off,
    const uint32_t* __restrict__ in_idx, const uint32_t* __restrict__ surv_cnt, double* __restrict__ gu,
    double* __restrict__ gv, uint32_t* __restrict__ gi, uint32_t* __restrict__ hull_cnt,
    uint32_t* __restrict__ hull_tmp, double* __restrict__ area_out)
{
    __shared__ double su[kLdsCap];
    __shared__ double sv[kLdsCap];
    __shared__ uint32_t si[kLdsCap];
    __shared__ uint16_t st_lo[2 * kLdsCap];
    __shared__ uint16_t st_up[kLdsCap + 1];
    __shared__ uint16_t tmp_lo[kLdsCap];
    __shared__ uint16_t tmp_up[kLdsCap];
    __shared__ uint16_t seq_lo[kLdsCap];
    __shared__ uint16_t seq_up[kLdsCap];
    __shared__ uint32_t offs_lo[kWave + 1], offs_up[kWave + 1];
    __shared__ uint32_t len2_lo[kChainL2], len2_up[kChainL2];
    __shared__ uint32_t hlo, hup;
    __shared__ double red[kChainBlock / kWave];
    // the clusters with more than one wave of survivors, listed by k_hull_small
    const uint32_t nc = small[7];
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const uint32_t k = chain_list[c];
        const uint32_t ib = in_off[k];
        const uint32_t ns = surv_cnt[k];
        if (ns <= (uint32_t)kLdsCap) {
            uint32_t N = 1;
            while (N < ns) N <<= 1;
            if (N <= (uint32_t)kChainBlock) {
                // one point per thread: bitonic stages over distances below 64
                // are shuffles inside a wave, the others go through LDS
                const uint32_t t = threadIdx.x;
                double u = t < ns ? gu[ib + t] : INFINITY, v = t < ns ? gv[ib + t] : INFINITY;
                uint32_t id = t < ns ? gi[ib + t] : 0xFFFFFFFFu;
                for (uint32_t size = 2; size <= N; size <<= 1) {
                    for (uint32_t j = size >> 1; j > 0; j >>= 1) {
                        double ou, ov;
                        uint32_t oi;
                        if (j >= (uint32_t)kWave) {
                            su[t] = u;
                            sv[t] = v;
                            si[t] = id;
                            __syncthreads();
                            ou = su[t ^ j];
                            ov = sv[t ^ j];
                            oi = si[t ^ j];
                            __syncthreads();
                        } else {
                            ou = __shfl_xor(u, (int)j, kWave);
                            ov = __shfl_xor(v, (int)j, kWave);
                            oi = __shfl_xor(id, (int)j, kWave);
                        }
                        const bool up = (t & size) == 0, low = (t & j) == 0;
                        if ((low == up) != p2_less(u, v, id, ou, ov, oi)) {
                            u = ou;
                            v = ov;
                            id = oi;
                        }
                    }
                }
                su[t] = u;
                sv[t] = v;
                si[t] = id;
                __syncthreads();
            } else {
                for (uint32_t t = threadIdx.x; t < N; t += kChainBlock) {
                    if (t < ns) {
                        su[t] = gu[ib + t];
                        sv[t] = gv[ib + t];
                        si[t] = gi[ib + t];
                    } else {
                        su[t] = INFINITY;
                        sv[t] = INFINITY;
                        si[t] = 0xFFFFFFFFu;
                    }
                }
                __syncthreads();
                for (uint32_t size = 2; size <= N; size <<= 1) {
                    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                        for (uint32_t t = threadIdx.x; t < N / 2; t += kChainBlock) {
                            const uint32_t a = 2 * t - (t & (stride - 1)), b = a + stride;
                            const bool upw = (a & size) == 0;
                            if (p2_less(su[b], sv[b], si[b], su[a], sv[a], si[a]) == upw) swap3(su, sv, si, a, b);
                        }
                        __syncthreads();
                    }
                }
            }
            // lower chain on wave 0, upper chain on wave 1
            if (threadIdx.x < kWave) chain_level1(su, sv, ns, true, tmp_lo, seq_lo, offs_lo);
            else if (threadIdx.x < 2 * kWave) chain_level1(su, sv, ns, false, tmp_up, seq_up, offs_up);
            __syncthreads();
            if (threadIdx.x < kChainL2) len2_lo[threadIdx.x] = chain_level2(su, sv, seq_lo, offs_lo, threadIdx.x);
            else if (threadIdx.x >= kWave && threadIdx.x < kWave + kChainL2)
                len2_up[threadIdx.x - kWave] = chain_level2(su, sv, seq_up, offs_up, threadIdx.x - kWave);
            __syncthreads();
            // level 3: the plain chain over the level-2 results, made contiguous
            // (the level-1 scratch is free again)
            const uint32_t l2lo = chain_gather2(seq_lo, offs_lo, len2_lo, tmp_lo);
            const uint32_t l2up = chain_gather2(seq_up, offs_up, len2_up, tmp_up);
            __syncthreads();
            if (threadIdx.x == 0) hlo = chain_run<false>(su, sv, tmp_lo, l2lo, st_lo);
            if (threadIdx.x == kWave) hup = chain_run<false>(su, sv, tmp_up, l2up, st_up);
            __syncthreads();
            // hull = lower chain, then the upper chain without its end points
            // (they are the lower chain's last and first points); the
            // vertices and the shoelace terms are taken in parallel
            {
                const uint32_t hl = hlo, hu = hup;
                const uint32_t h = hl + (hu >= 2 ? hu - 2 : 0u);
                auto vertex = [&](uint32_t q) -> uint32_t { return q < hl ? st_lo[q] : st_up[q - hl + 1]; };
                double term = 0.0;
                for (uint32_t q = threadIdx.x; q < h; q += kChainBlock) {
                    const uint32_t p0 = vertex(q), p1 = vertex(q + 1 == h ? 0u : q + 1);
                    term += su[p0] * sv[p1] - su[p1] * sv[p0];
                    hull_tmp[ib + k + q] = in_idx[ib + si[p0]];   // vertex indices
                }
#pragma unroll
                for (int dd = kWave / 2; dd >= 1; dd >>= 1) term += __shfl_xor(term, dd, kWave);
                if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = term;
                __syncthreads();
                if (threadIdx.x == 0) {
                    double tot = 0.0;
                    for (int w2 = 0; w2 < kChainBlock / kWave; ++w2) tot += red[w2];
                    area_out[k] = h >= 3 ? 0.5 * tot : 0.0;
                    hull_cnt[k] = h;
                }
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
    k_hull_small<<<kSmallGrid, kBlock, 0, s>>>(w.small, w.chain_list, w.hull_tile_off, cl.d_off, cl.d_x, cl.d_y,
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

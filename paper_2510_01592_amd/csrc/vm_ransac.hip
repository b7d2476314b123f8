// vm_ransac.hip -- cluster-parallel RANSAC (Sec. III-C, "Multi-plane
// estimation"): (a) hypotheses from three sampled points, (b) inlier
// counting, (c) selection of the best hypothesis and extraction of its inliers.
//
// All clusters are processed together.  Work is cut into tiles of a fixed
// number of points inside one cluster (the tile list is built on the device
// from the cluster offsets), so thousands of clusters of very different sizes
// load-balance across the 256 CUs without the host knowing any size.
//
// Inlier counting is the arithmetic hot spot (sum over clusters of n_k x H
// point-plane tests).  Each lane keeps P points of its tile in registers; the
// plane of the current hypothesis is wave-uniform (scalar loads), so one test
// is three v_fma_f32 and one v_cmp with the |.| modifier, and the count of a
// whole wave is a ballot and one scalar popcount.  Counts are integers added
// with atomics, hence independent of the order of tiles.
#include "vm_common.h"
#include "vm_dev.h"

#include <mutex>

#include <math.h>

namespace vm {
namespace {

using namespace dev;

constexpr int kCountBlock = 256;
constexpr int kPtsPerLane = 16;
constexpr int kTile = kCountBlock * kPtsPerLane;   // points per tile (4096)
constexpr int kMaxHypChunk = 4096;                 // hypotheses per work item (LDS counters)
constexpr int kHypBatch = 4;                       // planes loaded together
constexpr uint32_t kXcds = 8;                      // accelerator complex dies (separate L2s)

// (a) hypothesis (k, h): three distinct points -> unit normal (+z first) and
// offset in fp64, rounded to float32.  Degenerate triples get a NaN plane.
__global__ void __launch_bounds__(kBlock) k_hypotheses(const uint32_t* __restrict__ small,
                                                       const uint32_t* __restrict__ off,
                                                       const uint32_t* __restrict__ tag, const float* __restrict__ X,
                                                       const float* __restrict__ Y, const float* __restrict__ Z,
                                                       uint32_t H, uint64_t seed, uint32_t frame_arg,
                                                       const uint32_t* __restrict__ d_frame,
                                                       const uint32_t* __restrict__ cframe,
                                                       const uint32_t* __restrict__ tile_off,
                                                       uint32_t* __restrict__ tile_k,
                                                       const uint32_t* __restrict__ tile_off_big,
                                                       uint32_t* __restrict__ tile_k_big, uint32_t wave_max,
                                                       int32_t* __restrict__ counts, float4* __restrict__ hyp)
{
    const uint32_t frame_all = d_frame ? *d_frame : frame_arg;
    const uint32_t K = small[0];
    const uint64_t total = (uint64_t)K * H;
    for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (uint64_t)gridDim.x * blockDim.x) {
        // (32-bit division where the index fits: the 64-bit one is a long
        // instruction sequence per hypothesis)
        uint32_t k, h;
        if (total <= 0xFFFFFFFFull) {
            k = (uint32_t)idx / H;
            h = (uint32_t)idx - k * H;
        } else {
            k = (uint32_t)(idx / H);
            h = (uint32_t)(idx % H);
        }
        const uint32_t base = off[k];
        const uint64_t n = (uint64_t)(off[k + 1] - base);
        // the cluster of each of its point tiles, for the inlier kernels and
        // (clusters beyond one wave's points) for the tiled counting kernel
        const uint32_t nt = (uint32_t)((n + kTile - 1) / kTile);
        for (uint32_t q = h; q < nt; q += H) tile_k[tile_off[k] + q] = k;
        if (n > wave_max)
            for (uint32_t q = h; q < nt; q += H) tile_k_big[tile_off_big[k] + q] = k;
        const uint32_t frame = cframe ? cframe[k] : frame_all;   // a merged set's clusters carry their own
        const float4 pl = hyp_plane(X + base, Y + base, Z + base, n, h, tag[k], frame, seed);
        // the tiled kernel adds into the counts; the wave kernel stores every
        // count of its clusters, and clusters of fewer than 3 points have no
        // valid hypothesis (their counts are never read)
        if (n > wave_max) counts[idx] = 0;
        hyp[idx] = pl;
    }
}

// the clusters this pass processes (small[0] = K, 0 if the CSR is invalid)
__global__ void __launch_bounds__(kBlock) k_validate(const uint32_t* __restrict__ meta, uint32_t k_cap,
                                                     uint32_t out_k_cap, uint32_t n_cap,
                                                     const uint32_t* __restrict__ off, uint32_t* __restrict__ small,
                                                     uint32_t* __restrict__ status)
{
    __shared__ int bad;
    const uint32_t K = validate_clusters(meta, off, k_cap, n_cap, status, &bad);
    if (threadIdx.x == 0) {
        small[0] = K;
        if (meta[0] > out_k_cap) atomicOr(status, (uint32_t)VM_FLAG_CLUSTERS_CAP);
    }
}

// validate, tiles per cluster and both tile-offset scans in one workgroup
// (the capacity is at most kOneBlockMax clusters)
__global__ void __launch_bounds__(kOneBlockThreads) k_prepare(const uint32_t* __restrict__ meta, uint32_t k_cap,
                                                              uint32_t out_k_cap, uint32_t n_cap,
                                                              const uint32_t* __restrict__ off,
                                                              uint32_t* __restrict__ small,
                                                              uint32_t* __restrict__ tile_off,
                                                              uint32_t* __restrict__ tile_off_big, uint32_t wave_max,
                                                              uint32_t* __restrict__ status)
{
    __shared__ int bad;
    const uint32_t K = validate_clusters(meta, off, k_cap, n_cap, status, &bad);
    uint32_t total[2];
    one_block_scan<kOneBlockThreads, 4, 2>(
        K,
        [&](uint32_t k, uint32_t(&v)[2]) {
            const uint32_t n = off[k + 1] - off[k];
            v[0] = (n + kTile - 1) / kTile;
            v[1] = n > wave_max ? v[0] : 0u;   // counted by the tiled kernel
        },
        [&](uint32_t k, const uint32_t(&e)[2]) {
            tile_off[k] = e[0];
            tile_off_big[k] = e[1];
        },
        total);
    if (threadIdx.x == 0) {
        small[0] = K;
        small[1] = total[0];
        small[3] = total[1];
        if (meta[0] > out_k_cap) atomicOr(status, (uint32_t)VM_FLAG_CLUSTERS_CAP);
    }
}

// tiles per cluster (for the device-built tile list)
__global__ void __launch_bounds__(kBlock) k_tiles(const uint32_t* __restrict__ small,
                                                  const uint32_t* __restrict__ off, uint32_t* __restrict__ ntiles,
                                                  uint32_t* __restrict__ ntiles_big, uint32_t wave_max)
{
    const uint32_t K = small[0];
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        const uint32_t n = off[k + 1] - off[k];
        ntiles[k] = (n + kTile - 1) / kTile;
        ntiles_big[k] = n > wave_max ? (n + kTile - 1) / kTile : 0u;   // counted by the tiled kernel
    }
}

// (b) inlier counting over (tile, hypothesis-chunk) items.  The number of
// hypothesis chunks is chosen on the device from the tile count so that small
// frames still cover every CU; each item keeps its points in registers and
// sweeps its chunk of planes, kHypBatch planes per scalar-load batch.  A wave
// evaluates only the rows of 64 points that hold points of the tile's
// cluster: the last tile of a cluster is usually short, and most clusters
// are smaller than one tile.
template <int R>
__device__ __forceinline__ uint32_t count_rows(const float4 pl, const float* px, const float* py, const float* pz,
                                               float eps)
{
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const float dd = fmaf(pl.z, pz[j], fmaf(pl.y, py[j], fmaf(pl.x, px[j], pl.w)));
        acc += (uint32_t)__popcll(__ballot(fabsf(dd) < eps));
    }
    return acc;
}

// Planes hb..he (at most 64) against the wave's points.  A wave's count for
// a plane is uniform; the counts are gathered in one register, lane q
// keeping plane hb + q.
template <int R>
__device__ __forceinline__ int count_batch(const float4* __restrict__ hk, uint32_t hb, uint32_t he, const float* px,
                                           const float* py, const float* pz, float eps, int lane)
{
    int cv = 0;
    uint32_t h = hb;
    for (; h + kHypBatch <= he; h += kHypBatch) {
        float4 pl[kHypBatch];
#pragma unroll
        for (int b = 0; b < kHypBatch; ++b) pl[b] = hk[h + b];
#pragma unroll
        for (int b = 0; b < kHypBatch; ++b) {
            if (pl[b].x != pl[b].x) continue;   // degenerate hypothesis
            const uint32_t acc = count_rows<R>(pl[b], px, py, pz, eps);
            cv = (lane == (int)(h + b - hb)) ? (int)acc : cv;
        }
    }
    for (; h < he; ++h) {
        const float4 pl = hk[h];
        if (pl.x != pl.x) continue;
        const uint32_t acc = count_rows<R>(pl, px, py, pz, eps);
        cv = (lane == (int)(h - hb)) ? (int)acc : cv;
    }
    return cv;
}

// Planes h0..h1 of a tile: one vector LDS add per 64 planes into the block's
// counters.
template <int R>
__device__ __forceinline__ void count_planes(const float4* __restrict__ hk, uint32_t h0, uint32_t h1,
                                             const float* px, const float* py, const float* pz, float eps,
                                             uint32_t* lcnt, int lane)
{
    for (uint32_t hb = h0; hb < h1; hb += kWave) {
        const uint32_t he = min(h1, hb + (uint32_t)kWave);
        const int cv = count_batch<R>(hk, hb, he, px, py, pz, eps, lane);
        if ((uint32_t)lane < he - hb && cv) atomicAdd(&lcnt[hb - h0 + (uint32_t)lane], (uint32_t)cv);
    }
}

// All planes of a cluster that one wave holds: the counts are final, stored.
// With few points per lane the work per plane is short, so the planes of a
// 64-plane batch are fetched with one vector load (lane q loads plane
// hb + q) and broadcast lane by lane, instead of one scalar load per few
// planes whose latency the short work cannot hide.
template <int R>
__device__ __forceinline__ void count_all(const float4* __restrict__ hk, uint32_t h0, uint32_t h1, const float* px,
                                          const float* py, const float* pz, float eps, int32_t* __restrict__ ck,
                                          int lane)
{
    for (uint32_t hb = h0; hb < h1; hb += kWave) {
        const uint32_t nb = min(h1 - hb, (uint32_t)kWave);
        const float4 mine = (uint32_t)lane < nb ? hk[hb + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
        int cv = 0;
        for (uint32_t b = 0; b < nb; ++b) {
            float4 pl;
            pl.x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.x), (int)b));
            pl.y = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.y), (int)b));
            pl.z = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.z), (int)b));
            pl.w = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mine.w), (int)b));
            if (pl.x != pl.x) continue;   // degenerate hypothesis
            const uint32_t acc = count_rows<R>(pl, px, py, pz, eps);
            cv = (lane == (int)b) ? (int)acc : cv;
        }
        if ((uint32_t)lane < nb) ck[hb + (uint32_t)lane] = cv;
    }
}

// Clusters of at most a few rows of points: the lanes take the planes
// instead (lane q counts plane hb + q) and loop over the points, whose
// coordinates are wave-uniform loads (scalar loads, 16 points per step),
// so no lane idles and no per-plane reduction is needed.  The count is the
// same sum of the same tests.
__device__ __forceinline__ void count_by_planes(const float4* __restrict__ hk, uint32_t h0, uint32_t h1, uint32_t n,
                                                const float* __restrict__ X, const float* __restrict__ Y,
                                                const float* __restrict__ Z, float eps, int32_t* __restrict__ ck,
                                                int lane)
{
    // four 64-plane batches at a time: their plane loads are issued
    // together and each point is loaded once for all four
    constexpr int kB = 4;
    for (uint32_t hb = h0; hb < h1; hb += kB * kWave) {
        float4 pl[kB];
        bool has[kB];
        uint32_t c[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            const uint32_t h = hb + (uint32_t)(b * kWave + lane);
            has[b] = h < h1;
            pl[b] = has[b] ? hk[h] : make_float4(0.f, 0.f, 0.f, 0.f);
            c[b] = 0;
        }
        uint32_t j = 0;
        for (; j + 16 <= n; j += 16) {
            float x[16], y[16], z[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                x[q] = X[j + q];
                y[q] = Y[j + q];
                z[q] = Z[j + q];
            }
#pragma unroll
            for (int b = 0; b < kB; ++b) {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const float dd = fmaf(pl[b].z, z[q], fmaf(pl[b].y, y[q], fmaf(pl[b].x, x[q], pl[b].w)));
                    c[b] += fabsf(dd) < eps ? 1u : 0u;   // a degenerate (NaN) plane never passes
                }
            }
        }
        for (; j < n; ++j) {
            const float x = X[j], y = Y[j], z = Z[j];
#pragma unroll
            for (int b = 0; b < kB; ++b) {
                const float dd = fmaf(pl[b].z, z, fmaf(pl[b].y, y, fmaf(pl[b].x, x, pl[b].w)));
                c[b] += fabsf(dd) < eps ? 1u : 0u;
            }
        }
#pragma unroll
        for (int b = 0; b < kB; ++b)
            if (has[b]) ck[hb + (uint32_t)(b * kWave + lane)] = (int32_t)c[b];
    }
}

// Clusters of at most wave_max points (at most 1024: one wave's registers)
// are counted by waves without LDS or workgroup barriers, a wave per
// (cluster, chunk of hypotheses) item: the counts of a chunk are final.  The
// hypotheses are split into chunks (multiples of 64) only as far as needed
// for about chunk_mult items per wave, so few clusters still fill the chip.
// Larger clusters go through the tiled kernel below.  Clusters of at most
// plane_max points (at most 256) put the lanes over planes.
constexpr uint32_t kWaveMaxPts = kWave * kPtsPerLane;   // 1024
constexpr uint32_t kPlaneMaxPts = 4 * kWave;            // 256

__global__ void __launch_bounds__(kCountBlock) k_count_small(const uint32_t* __restrict__ small,
                                                             const uint32_t* __restrict__ off,
                                                             const float* __restrict__ X, const float* __restrict__ Y,
                                                             const float* __restrict__ Z, uint32_t H, float eps,
                                                             const float4* __restrict__ hyp,
                                                             int32_t* __restrict__ counts, uint32_t wave_max,
                                                             uint32_t plane_max, uint32_t chunk_mult)
{
    const uint32_t K = small[0];
    if (K == 0) return;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (kCountBlock / kWave);
    const float qnan = __builtin_nanf("");
    // chunks of cb 64-plane batches, HC chunks per cluster
    const uint32_t nb64 = (H + kWave - 1) / kWave;
    uint32_t HC = (uint32_t)min((uint64_t)nb64, ((uint64_t)chunk_mult * waves + K - 1) / K);
    if (HC < 1) HC = 1;
    const uint32_t cb = (nb64 + HC - 1) / HC;
    HC = (nb64 + cb - 1) / cb;
    const uint64_t items = (uint64_t)K * HC;
    // the wave's item index, made explicitly wave-uniform so that its loads
    // (offsets, points, planes' addresses) are scalar
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (kCountBlock / kWave) + threadIdx.x / kWave);
    for (uint64_t item = w0; item < items; item += waves) {
        const uint32_t k = (uint32_t)(item / HC), hc = (uint32_t)(item % HC);
        const uint32_t h0 = hc * cb * kWave, h1 = min(H, h0 + cb * kWave);
        const uint32_t base = off[k], n = off[k + 1] - base;
        if (n < 3 || n > wave_max) continue;   // fewer than 3: no planes; more: the tiled kernel
        const int rows = (int)((n + kWave - 1) / kWave);
        float px[kPtsPerLane], py[kPtsPerLane], pz[kPtsPerLane];
#pragma unroll
        for (int j = 0; j < kPtsPerLane; ++j) {
            const uint32_t i = (uint32_t)(j * kWave + lane);
            const bool v = i < n;
            px[j] = v ? X[base + i] : qnan;   // NaN never passes |d| < eps
            py[j] = v ? Y[base + i] : qnan;
            pz[j] = v ? Z[base + i] : qnan;
        }
        const float4* hk = hyp + (size_t)k * H;
        int32_t* ck = counts + (size_t)k * H;
        if (n <= plane_max) count_by_planes(hk, h0, h1, n, X + base, Y + base, Z + base, eps, ck, lane);
        else if (rows > 8) count_all<16>(hk, h0, h1, px, py, pz, eps, ck, lane);
        else if (rows > 4) count_all<8>(hk, h0, h1, px, py, pz, eps, ck, lane);
        else if (rows > 2) count_all<4>(hk, h0, h1, px, py, pz, eps, ck, lane);
        else if (rows > 1) count_all<2>(hk, h0, h1, px, py, pz, eps, ck, lane);
        else count_all<1>(hk, h0, h1, px, py, pz, eps, ck, lane);
    }
}

__global__ void __launch_bounds__(kCountBlock) k_count(const uint32_t* __restrict__ small,
                                                       const uint32_t* __restrict__ tile_off, const uint32_t* __restrict__ tile_k,
                                                       const uint32_t* __restrict__ off, const float* __restrict__ X,
                                                       const float* __restrict__ Y, const float* __restrict__ Z,
                                                       uint32_t H, float eps, const float4* __restrict__ hyp,
                                                       int32_t* __restrict__ counts, uint32_t chunk_mult)
{
    __shared__ uint32_t lcnt[kMaxHypChunk];
    const uint32_t T = small[3];   // tiles of the clusters beyond one wave
    if (T == 0) return;
    // chunks per tile: enough items for two per block of the grid, chunks of
    // at least 32 hypotheses, at most kMaxHypChunk
    uint32_t HC = (chunk_mult * gridDim.x + T - 1) / T;
    const uint32_t hc_max = (H + 31) / 32;
    if (HC > hc_max) HC = hc_max;
    if (HC < (H + kMaxHypChunk - 1) / kMaxHypChunk) HC = (H + kMaxHypChunk - 1) / kMaxHypChunk;
    if (HC < 1) HC = 1;
    const uint32_t chunk = (H + HC - 1) / HC;
    // Workgroups are dispatched round-robin over the XCDs, each with its own
    // L2: tile t is handled on XCD t mod kXcds only, so the hypothesis chunks
    // of a tile (run at about the same time) fetch its points from memory once.
    const uint32_t xcd = blockIdx.x % kXcds, sub = blockIdx.x / kXcds, nsub = gridDim.x / kXcds;
    const uint32_t tiles_x = T > xcd ? (T - xcd + kXcds - 1) / kXcds : 0u;
    const uint64_t items = (uint64_t)tiles_x * HC;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (uint64_t item = sub; item < items; item += nsub) {
        const uint32_t t = (uint32_t)(item / HC) * kXcds + xcd, hc = (uint32_t)(item % HC);
        const uint32_t k = tile_k[t];
        const uint32_t p0 = off[k] + (t - tile_off[k]) * kTile;
        const uint32_t pend = off[k + 1];
        const uint32_t h0 = hc * chunk, h1 = min(H, h0 + chunk);
        const uint32_t wbase = p0 + (uint32_t)(wave * kWave * kPtsPerLane);
        const int rows = pend > wbase ? (int)min((uint32_t)kPtsPerLane, (pend - wbase + kWave - 1) / kWave) : 0;
        float px[kPtsPerLane], py[kPtsPerLane], pz[kPtsPerLane];
        const float qnan = __builtin_nanf("");
#pragma unroll
        for (int j = 0; j < kPtsPerLane; ++j) {
            const uint32_t i = wbase + (uint32_t)(j * kWave + lane);
            const bool v = i < pend;
            px[j] = v ? X[i] : qnan;   // NaN never passes |d| < eps
            py[j] = v ? Y[i] : qnan;
            pz[j] = v ? Z[i] : qnan;
        }
        for (uint32_t h = h0 + threadIdx.x; h < h1; h += kCountBlock) lcnt[h - h0] = 0;
        __syncthreads();
        const float4* hk = hyp + (size_t)k * H;
        // rows is wave-uniform; rows past the cluster's end hold NaN points
        static_assert(kPtsPerLane == 16, "the row dispatch below assumes 16 rows per lane");
        if (rows > 8) count_planes<16>(hk, h0, h1, px, py, pz, eps, lcnt, lane);
        else if (rows > 4) count_planes<8>(hk, h0, h1, px, py, pz, eps, lcnt, lane);
        else if (rows > 2) count_planes<4>(hk, h0, h1, px, py, pz, eps, lcnt, lane);
        else if (rows > 1) count_planes<2>(hk, h0, h1, px, py, pz, eps, lcnt, lane);
        else if (rows == 1) count_planes<1>(hk, h0, h1, px, py, pz, eps, lcnt, lane);
        __syncthreads();
        int32_t* ck = counts + (size_t)k * H;
        for (uint32_t hh = h0 + threadIdx.x; hh < h1; hh += kCountBlock) {
            const uint32_t c = lcnt[hh - h0];
            if (c) atomicAdd(&ck[hh], (int32_t)c);
        }
        __syncthreads();
    }
}

// (c) best hypothesis per cluster: largest count, first index on ties
__global__ void __launch_bounds__(kBlock) k_select(const uint32_t* __restrict__ small, uint32_t H,
                                                   const int32_t* __restrict__ counts, const float4* __restrict__ hyp,
                                                   float4* __restrict__ plane_out, int32_t* __restrict__ best_out,
                                                   int32_t* __restrict__ nin_out, int32_t* __restrict__ counts_out,
                                                   float4* __restrict__ hyp_out)
{
    const uint32_t K = small[0];
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (blockDim.x / kWave);
    for (uint32_t k = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; k < K; k += waves) {
        int32_t bc = -1;
        uint32_t bh = 0xFFFFFFFFu;
        for (uint32_t h = lane; h < H; h += kWave) {
            const float4 pl = hyp[(size_t)k * H + h];
            const bool degen = pl.x != pl.x;
            const int32_t c = degen ? -1 : counts[(size_t)k * H + h];
            if (c > bc) { bc = c; bh = h; }
            if (counts_out) counts_out[(size_t)k * H + h] = c;
            if (hyp_out) hyp_out[(size_t)k * H + h] = degen ? make_float4(0.f, 0.f, 0.f, 0.f) : pl;
        }
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) {
            const int32_t oc = __shfl_xor(bc, d, kWave);
            const uint32_t oh = __shfl_xor(bh, d, kWave);
            if (oc > bc || (oc == bc && oh < bh)) { bc = oc; bh = oh; }
        }
        if (lane == 0) {
            if (bc < 0) {
                best_out[k] = -1;
                nin_out[k] = 0;
                plane_out[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            } else {
                best_out[k] = (int32_t)bh;
                nin_out[k] = bc;
                plane_out[k] = hyp[(size_t)k * H + bh];
            }
        }
    }
}

// (c) the inlier lists of the winning planes, over the same point tiles, in
// three launches: inliers per tile; one workgroup's scan of the tile counts
// (which also gives each cluster's list offset); the lists, each workgroup
// placing its tile's inliers in point order with a block scan.
__global__ void __launch_bounds__(kCountBlock) k_inlier_count(const uint32_t* __restrict__ small,
                                                              const uint32_t* __restrict__ tile_off,
                                                              const uint32_t* __restrict__ tile_k,
                                                              const uint32_t* __restrict__ off,
                                                              const float* __restrict__ X, const float* __restrict__ Y,
                                                              const float* __restrict__ Z, float eps,
                                                              const int32_t* __restrict__ best,
                                                              const float4* __restrict__ plane,
                                                              uint32_t* __restrict__ tile_cnt)
{
    __shared__ uint32_t wsum[kCountBlock / kWave];
    const uint32_t T = small[1];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (uint32_t t = blockIdx.x; t < T; t += gridDim.x) {
        const uint32_t k = tile_k[t];
        const uint32_t p0 = off[k] + (t - tile_off[k]) * kTile;
        const uint32_t pend = min(p0 + kTile, off[k + 1]);
        uint32_t c = 0;
        if (best[k] >= 0) {
            const float4 pl = plane[k];
            for (uint32_t i = p0 + threadIdx.x; i < pend; i += kCountBlock) c += inlier_test(pl, X[i], Y[i], Z[i], eps);
        }
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) c += __shfl_xor(c, d, kWave);
        if (lane == 0) wsum[wave] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < kCountBlock / kWave; ++w) tot += wsum[w];
            tile_cnt[t] = tot;
        }
        __syncthreads();   // wsum is reused by the next tile
    }
}

__global__ void __launch_bounds__(kOneBlockThreads) k_inlier_scan(uint32_t* __restrict__ small,
                                                                  const uint32_t* __restrict__ tile_off,
                                                                  uint32_t* __restrict__ tile_cnt,
                                                                  uint32_t* __restrict__ in_off)
{
    const uint32_t K = small[0], T = small[1];
    uint32_t total[1];
    one_block_scan<kOneBlockThreads, 4, 1>(
        T, [&](uint32_t t, uint32_t(&v)[1]) { v[0] = tile_cnt[t]; },
        [&](uint32_t t, const uint32_t(&e)[1]) { tile_cnt[t] = e[0]; }, total);
    __syncthreads();   // the prefixes other threads wrote
    // a cluster's list starts at the prefix of its first tile (a cluster
    // without points has no tile: the next cluster's start, or the total)
    for (uint32_t k = threadIdx.x; k <= K; k += blockDim.x)
        in_off[k] = (k < K && tile_off[k] < T) ? tile_cnt[tile_off[k]] : total[0];
    if (threadIdx.x == 0) small[2] = total[0];
}

__global__ void __launch_bounds__(kCountBlock) k_inlier_write(const uint32_t* __restrict__ small,
                                                              const uint32_t* __restrict__ tile_off,
                                                              const uint32_t* __restrict__ tile_k,
                                                              const uint32_t* __restrict__ off,
                                                              const float* __restrict__ X, const float* __restrict__ Y,
                                                              const float* __restrict__ Z, float eps,
                                                              const int32_t* __restrict__ best,
                                                              const float4* __restrict__ plane,
                                                              const uint32_t* __restrict__ tile_pre, uint32_t in_cap,
                                                              uint32_t* __restrict__ in_idx, uint32_t* __restrict__ status)
{
    // The tile's tests are made with coalesced loads (consecutive lanes,
    // consecutive points) and collected as a bit mask in LDS, 64 bits per
    // wave step by a ballot; then thread w takes mask word w (32 points), a
    // block scan of the words' counts places their inliers in point order.
    constexpr uint32_t kWords = kTile / 32;   // 128
    static_assert(kWords <= kCountBlock, "a thread per mask word");
    __shared__ uint32_t mask[kWords];
    __shared__ uint32_t wsum[kCountBlock / kWave];
    const uint32_t T = small[1];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    bool over = false;
    for (uint32_t t = blockIdx.x; t < T; t += gridDim.x) {
        const uint32_t k = tile_k[t];
        if (best[k] < 0) continue;   // workgroup-uniform
        const uint32_t base = off[k];
        const uint32_t p0 = base + (t - tile_off[k]) * kTile;
        const uint32_t pend = min(p0 + kTile, off[k + 1]);
        const float4 pl = plane[k];
#pragma unroll 4
        for (uint32_t j0 = 0; j0 < kTile; j0 += kCountBlock) {
            const uint32_t i = p0 + j0 + threadIdx.x;
            const bool in = i < pend && inlier_test(pl, X[i], Y[i], Z[i], eps);
            const uint64_t b = __ballot(in);
            if (lane == 0) {
                const uint32_t w = (j0 + (uint32_t)wave * kWave) / 32;
                mask[w] = (uint32_t)b;
                mask[w + 1] = (uint32_t)(b >> 32);
            }
        }
        __syncthreads();
        uint32_t m = threadIdx.x < kWords ? mask[threadIdx.x] : 0u;
        const uint32_t c = (uint32_t)__popc(m);
        uint32_t inc = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d, kWave);
            if (lane >= d) inc += o;
        }
        if (lane == kWave - 1) wsum[wave] = inc;
        __syncthreads();
        uint32_t p = tile_pre[t] + inc - c;
#pragma unroll
        for (int w = 0; w < kCountBlock / kWave; ++w) p += (w < wave) ? wsum[w] : 0u;
        const uint32_t q0 = p0 + threadIdx.x * 32 - base;   // cluster-local index of the word's first point
        for (; m; m &= m - 1, ++p) {
            if (p < in_cap) in_idx[p] = q0 + (uint32_t)(__ffs(m) - 1);
            else over = true;
        }
        __syncthreads();   // mask and wsum are reused by the next tile
    }
    if (over) atomicOr(status, (uint32_t)VM_FLAG_INLIERS_CAP);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

WorkLayout work_layout(void* base, uint32_t k_cap, uint32_t n_cap, uint32_t n_hyp)
{
    WorkLayout w{};
    w.k_cap = k_cap;
    char* p = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* r = p ? p + o : nullptr;
        o += align256(bytes);
        return r;
    };
    const size_t kh = (size_t)k_cap * (size_t)n_hyp;
    w.counts = (int32_t*)take(kh * sizeof(int32_t));
    w.hyp = (float4*)take(kh * sizeof(float4));
    w.tile_off = (uint32_t*)take(((size_t)k_cap + 2) * sizeof(uint32_t));
    w.tile_k = (uint32_t*)take(((size_t)n_cap / kTile + k_cap + 2) * sizeof(uint32_t));
    w.tile_off_big = (uint32_t*)take(((size_t)k_cap + 2) * sizeof(uint32_t));
    w.tile_k_big = (uint32_t*)take(((size_t)n_cap / kTile + k_cap + 2) * sizeof(uint32_t));
    w.flags = (uint32_t*)take(((size_t)n_cap + 1) * sizeof(uint32_t));
    const size_t blk_words = scan_blk_words((uint64_t)n_cap + k_cap + 2) + 64;
    w.blk = (uint32_t*)take(blk_words * sizeof(uint32_t));
    w.hull_cnt = (uint32_t*)take(((size_t)k_cap + 2) * sizeof(uint32_t));
    w.hull_off = (uint32_t*)take(((size_t)k_cap + 2) * sizeof(uint32_t));
    w.hull_tmp = (uint32_t*)take(((size_t)n_cap + k_cap + 2) * sizeof(uint32_t));
    w.hull_u = (double*)take(((size_t)n_cap + 1) * sizeof(double));
    w.hull_v = (double*)take(((size_t)n_cap + 1) * sizeof(double));
    w.hull_i = (uint32_t*)take(((size_t)n_cap + 1) * sizeof(uint32_t));
    w.hull_tile_off = (uint32_t*)take(((size_t)k_cap + 2) * sizeof(uint32_t));
    const size_t ht = hull_tiles_bound(k_cap, n_cap);
    w.ext_v = (double*)take(ht * kHullDirs * sizeof(double));
    w.ext_i = (uint32_t*)take(ht * kHullDirs * sizeof(uint32_t));
    w.poly = (double*)take((size_t)k_cap * (2 * kHullDirs + 2) * sizeof(double) + 8);
    w.surv_cnt = (uint32_t*)take(((size_t)k_cap + 1) * sizeof(uint32_t));
    w.chain_list = (uint32_t*)take(((size_t)k_cap + 1) * sizeof(uint32_t));
    w.small = (uint32_t*)take(64 * sizeof(uint32_t));
    w.bytes = o;
    return w;
}

namespace {
std::mutex g_count_mu;
vm_count_config g_count_cfg = count_config_default();
}   // namespace

vm_count_config count_config_default()
{
    vm_count_config c;
    c.count_grid = 16384;
    c.chunk_mult = 2;
    c.wave_max_points = kPlaneMaxPts;   // larger clusters: the tiled kernel splits their hypotheses
    c.plane_max_points = kPlaneMaxPts;
    return c;
}

bool count_config_valid(const vm_count_config& c)
{
    if (c.count_grid < kXcds || c.count_grid > 65536 || c.count_grid % kXcds != 0) return false;
    if (c.chunk_mult < 1 || c.chunk_mult > 16) return false;
    if (c.wave_max_points > kWaveMaxPts) return false;
    return c.plane_max_points <= kPlaneMaxPts && c.plane_max_points <= c.wave_max_points;
}

vm_count_config count_config_get()
{
    std::lock_guard<std::mutex> g(g_count_mu);
    return g_count_cfg;
}

void count_config_set(const vm_count_config& c)
{
    std::lock_guard<std::mutex> g(g_count_mu);
    g_count_cfg = c;
}

vm_status ransac_planes(const vm_clusters& cl, const vm_ransac_params& p, const vm_planes& out,
                        const WorkLayout& w, hipStream_t s, const uint32_t* d_cframe)
{
    // the workspace is laid out for kc = min(cl.k_cap, out.k_cap) clusters
    const uint32_t kc = cl.k_cap < out.k_cap ? cl.k_cap : out.k_cap;
    if (kc > w.k_cap) return VM_E_STATE;
    const uint32_t H = p.n_hyp;
    const vm_count_config cc = count_config_get();
    // small[0] = K (clamped), small[1] = tiles, small[2] = inliers, small[3] = tiles of clusters beyond one wave
    {
        StageScope t(VM_STAGE_HYPOTHESES, s);
        if (kc <= kOneBlockMax) {
            k_prepare<<<1, kOneBlockThreads, 0, s>>>(cl.d_meta, kc, out.k_cap, cl.n_cap, cl.d_off, w.small, w.tile_off,
                                                     w.tile_off_big, cc.wave_max_points, out.d_status);
        } else {
            k_validate<<<1, kBlock, 0, s>>>(cl.d_meta, kc, out.k_cap, cl.n_cap, cl.d_off, w.small, out.d_status);
            k_tiles<<<grid_for(kc), kBlock, 0, s>>>(w.small, cl.d_off, w.tile_off, w.tile_off_big,
                                                    cc.wave_max_points);
            VM_HIP(scan_exclusive_dev(w.tile_off, w.tile_off, w.small, kc, w.small + 1, w.blk, s));
            VM_HIP(scan_exclusive_dev(w.tile_off_big, w.tile_off_big, w.small, kc, w.small + 3, w.blk, s));
        }
        const uint64_t kh = (uint64_t)kc * H;
        k_hypotheses<<<grid_for(kh, kBlock, 16384), kBlock, 0, s>>>(w.small, cl.d_off, cl.d_tag, cl.d_x, cl.d_y,
                                                                    cl.d_z, H, p.seed, p.frame, p.d_frame, d_cframe,
                                                                    w.tile_off, w.tile_k, w.tile_off_big, w.tile_k_big,
                                                                    cc.wave_max_points, w.counts, w.hyp);
        VM_HIP(hipGetLastError());
    }
    {
        StageScope t(VM_STAGE_COUNT, s);
        if (cc.wave_max_points >= 3)
            k_count_small<<<grid_for((uint64_t)kc * ((H + kWave - 1) / kWave) * kWave, kCountBlock, 1024), kCountBlock,
                            0, s>>>(
                w.small, cl.d_off, cl.d_x, cl.d_y, cl.d_z, H, p.eps, w.hyp, w.counts, cc.wave_max_points,
                cc.plane_max_points, cc.chunk_mult);
        k_count<<<cc.count_grid, kCountBlock, 0, s>>>(w.small, w.tile_off_big, w.tile_k_big, cl.d_off, cl.d_x, cl.d_y,
                                                      cl.d_z, H, p.eps, w.hyp, w.counts, cc.chunk_mult);
        VM_HIP(hipGetLastError());
    }
    {
        StageScope t(VM_STAGE_SELECT, s);
        k_select<<<grid_for((uint64_t)kc * kWave), kBlock, 0, s>>>(w.small, H, w.counts, w.hyp, (float4*)out.d_plane,
                                                                   out.d_best_h, out.d_n_inliers, out.d_counts,
                                                                   (float4*)out.d_hyp);
        const int tgrid = grid_for((uint64_t)cl.n_cap / kTile + kc + 1, 1, 8192);   // most tiles are small: many workgroups
        // w.flags holds the per-tile counts, then their prefixes (tiles <= points)
        k_inlier_count<<<tgrid, kCountBlock, 0, s>>>(w.small, w.tile_off, w.tile_k, cl.d_off, cl.d_x, cl.d_y, cl.d_z,
                                                     p.eps, out.d_best_h, (const float4*)out.d_plane, w.flags);
        k_inlier_scan<<<1, kOneBlockThreads, 0, s>>>(w.small, w.tile_off, w.flags, out.d_in_off);
        k_inlier_write<<<tgrid, kCountBlock, 0, s>>>(w.small, w.tile_off, w.tile_k, cl.d_off, cl.d_x, cl.d_y, cl.d_z, p.eps,
                                                     out.d_best_h, (const float4*)out.d_plane, w.flags, out.in_cap,
                                                     out.d_in_idx, out.d_status);
        VM_HIP(hipGetLastError());
    }
    return VM_OK;
}

}  // namespace vm

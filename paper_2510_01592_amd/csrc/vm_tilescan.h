// vm_tilescan.h -- two-kernel exclusive scans whose values are computed on the
// fly and whose results are consumed in place, so that a
// "flag -> scan -> use" sequence takes two launches and no flag arrays.
//
//   k_tile_reduce:  tile t sums f(i) over its kTsTile items into blk[t];
//   k_tile_down:    tile t adds up blk[0, t) (a block-wide sum over a few
//                   thousand words from L2), scans its own items (wave by
//                   wave, consecutive lanes on consecutive items) and calls
//                   g(i, f(i), exclusive prefix) for every item; the tile
//                   holding the last item (or tile 0 when there are no items)
//                   calls g.total(sum of all).
// Items are i < n with n = min(*d_n, n_fixed) (or n_fixed when d_n is null).
// Launch through tile_scan(); blk needs N * ts_tiles(n_fixed) words.  f and
// g are small structs of device pointers, passed by value.
#pragma once
#include "vm_common.h"

namespace vm {

template <int N>
struct Vec {
    uint32_t v[N];
};

template <int N>
__device__ __forceinline__ Vec<N> vzero()
{
    Vec<N> r;
#pragma unroll
    for (int q = 0; q < N; ++q) r.v[q] = 0u;
    return r;
}

template <int N>
__device__ __forceinline__ Vec<N> vadd(const Vec<N>& a, const Vec<N>& b)
{
    Vec<N> r;
#pragma unroll
    for (int q = 0; q < N; ++q) r.v[q] = a.v[q] + b.v[q];
    return r;
}

constexpr int kTsItems = 4;                      // items per thread (small tiles: many workgroups)
constexpr uint32_t kTsTile = kBlock * kTsItems;  // items per tile (1024)
// Up to this many tiles, a tile sums the tile totals before it itself;
// beyond, one workgroup scans the totals in between.
constexpr uint32_t kTsDirectTiles = 16384;

inline uint32_t ts_tiles(uint64_t n_fixed)
{
    const uint64_t t = (n_fixed + kTsTile - 1) / kTsTile;
    return (uint32_t)(t ? t : 1);
}

// exclusive prefix of x over the block (thread order); *total = block sum.
// lds needs kBlock / kWave entries.
template <int N>
__device__ __forceinline__ Vec<N> ts_block_excl(Vec<N> x, Vec<N>* lds, Vec<N>* total)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    Vec<N> inc = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const uint32_t o = __shfl_up(inc.v[q], d, kWave);
            if (lane >= d) inc.v[q] += o;
        }
    }
    if (lane == kWave - 1) lds[wave] = inc;
    __syncthreads();
    Vec<N> off = vzero<N>(), tot = vzero<N>();
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        const Vec<N> t = lds[w];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            off.v[q] += (w < wave) ? t.v[q] : 0u;
            tot.v[q] += t.v[q];
        }
    }
    __syncthreads();
    *total = tot;
    Vec<N> r;
#pragma unroll
    for (int q = 0; q < N; ++q) r.v[q] = off.v[q] + inc.v[q] - x.v[q];
    return r;
}

template <int N, class F>
__global__ void __launch_bounds__(kBlock) k_tile_reduce(F f, const uint32_t* d_n, uint32_t n_fixed,
                                                        Vec<N>* __restrict__ blk)
{
    __shared__ Vec<N> lds[kBlock / kWave];
    const uint32_t n = d_n ? min(*d_n, n_fixed) : n_fixed;
    const uint64_t base = (uint64_t)blockIdx.x * kTsTile;
    if (base >= n) {
        if (threadIdx.x == 0) blk[blockIdx.x] = vzero<N>();
        return;
    }
    Vec<N> s = vzero<N>();
#pragma unroll 4
    for (int j = 0; j < kTsItems; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        if (i < n) s = vadd(s, f((uint32_t)i));
    }
    Vec<N> tot;
    ts_block_excl(s, lds, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

template <int N>
__device__ __forceinline__ Vec<N> ts_wave_incl(Vec<N> x, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const uint32_t o = __shfl_up(x.v[q], d, kWave);
            if (lane >= d) x.v[q] += o;
        }
    }
    return x;
}

template <int N>
__device__ __forceinline__ Vec<N> ts_shfl(const Vec<N>& x, int src)
{
    Vec<N> r;
#pragma unroll
    for (int q = 0; q < N; ++q) r.v[q] = __shfl(x.v[q], src, kWave);
    return r;
}

// Wave w of the tile handles items base + w * kTsWaveSpan + j * 64 + lane
// (j < kTsItems), so consecutive lanes handle consecutive items in every
// step and the consumer's reads and writes coalesce.
constexpr uint32_t kTsWaveSpan = kWave * kTsItems;

template <int N, class F, class G>
__global__ void __launch_bounds__(kBlock) k_tile_down(F f, G g, const uint32_t* d_n, uint32_t n_fixed,
                                                      const Vec<N>* __restrict__ blk, bool scanned)
{
    __shared__ Vec<N> lds[kBlock / kWave];
    __shared__ Vec<N> wsum[kBlock / kWave];
    const uint32_t n = d_n ? min(*d_n, n_fixed) : n_fixed;
    const uint64_t base = (uint64_t)blockIdx.x * kTsTile;
    if (base >= n) {
        if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) g.total(vzero<N>());
        return;
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    // prefix of this tile: the sum of the tiles before it (or the scanned totals)
    Vec<N> tile_pre;
    if (scanned) {
        tile_pre = blk[blockIdx.x];
    } else {
        Vec<N> pre = vzero<N>();
        for (uint32_t t = threadIdx.x; t < blockIdx.x; t += kBlock) pre = vadd(pre, blk[t]);
        ts_block_excl(pre, lds, &tile_pre);
    }
    const uint64_t wbase = base + (uint64_t)wave * kTsWaveSpan;
    Vec<N> xs[kTsItems];
    Vec<N> s = vzero<N>();
#pragma unroll
    for (int j = 0; j < kTsItems; ++j) {
        const uint64_t i = wbase + (uint64_t)j * kWave + lane;
        xs[j] = i < n ? f((uint32_t)i) : vzero<N>();
        s = vadd(s, xs[j]);
    }
    // wave totals, then each wave's starting prefix
    const Vec<N> wtot = ts_shfl(ts_wave_incl(s, lane), kWave - 1);
    if (lane == 0) wsum[wave] = wtot;
    __syncthreads();
    Vec<N> run = tile_pre, all = tile_pre;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (w < wave) run = vadd(run, wsum[w]);
        all = vadd(all, wsum[w]);
    }
#pragma unroll
    for (int j = 0; j < kTsItems; ++j) {
        const uint64_t i = wbase + (uint64_t)j * kWave + lane;
        const Vec<N> inc = ts_wave_incl(xs[j], lane);
        Vec<N> ex;
#pragma unroll
        for (int q = 0; q < N; ++q) ex.v[q] = run.v[q] + inc.v[q] - xs[j].v[q];
        if (i < n) g((uint32_t)i, xs[j], ex);
        run = vadd(run, ts_shfl(inc, kWave - 1));
    }
    if (threadIdx.x == 0 && base + kTsTile >= n) g.total(all);
}

// exclusive scan of the tile totals in place (one workgroup), for grids of
// more than kTsDirectTiles tiles
template <int N>
__global__ void __launch_bounds__(kBlock) k_tile_totals(Vec<N>* blk, uint32_t ntiles)
{
    __shared__ Vec<N> lds[kBlock / kWave];
    Vec<N> carry = vzero<N>();
    for (uint32_t b0 = 0; b0 < ntiles; b0 += kBlock) {
        const uint32_t t = b0 + threadIdx.x;
        const Vec<N> x = t < ntiles ? blk[t] : vzero<N>();
        Vec<N> tot;
        const Vec<N> ex = ts_block_excl(x, lds, &tot);
        if (t < ntiles) blk[t] = vadd(carry, ex);
        carry = vadd(carry, tot);
    }
}

// The two (or three) launches of a fused scan over n_fixed item slots.
template <int N, class F, class G>
inline void tile_scan(F f, G g, const uint32_t* d_n, uint32_t n_fixed, Vec<N>* blk, hipStream_t s)
{
    const uint32_t nt = ts_tiles(n_fixed);
    const bool scanned = nt > kTsDirectTiles;
    k_tile_reduce<N><<<nt, kBlock, 0, s>>>(f, d_n, n_fixed, blk);
    if (scanned) k_tile_totals<N><<<1, kBlock, 0, s>>>(blk, nt);
    k_tile_down<N><<<nt, kBlock, 0, s>>>(f, g, d_n, n_fixed, blk, scanned);
}

}  // namespace vm

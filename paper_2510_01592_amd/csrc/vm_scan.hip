// vm_scan.hip -- device-wide exclusive scan and stable LSD radix sort of
// (key, value) pairs, with element counts read on the device so that no
// stage of a frame waits for the host.
#include "vm_common.h"

namespace vm {
namespace {

constexpr int kScanItems = 16;                      // per thread
constexpr int kScanTile = kBlock * kScanItems;      // 4096 values per block

// 10-bit digits: cluster ids below 1024 (the usual case) sort in one pass
// that runs, and ids up to 2^20 in two
constexpr int kRadixBits = 10;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kBinsPerThread = kRadixBins / kBlock;
static_assert(kRadixBins % kBlock == 0, "bins are spread evenly over the threads");
constexpr int kRadixIters = 8;
constexpr int kRadixTile = kBlock * kRadixIters;    // 2048 pairs per block

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, kWave);
        if (lane >= d) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the prefix and
// writes the block total to *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lds4, uint32_t* total)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v, lane);
    if (lane == kWave - 1) lds4[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        const uint32_t t = lds4[w];
        off += (w < wave) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const uint32_t* __restrict__ in, const uint32_t* d_n,
                                                        uint32_t n_fixed, uint32_t* __restrict__ blk)
{
    __shared__ uint32_t lds[kBlock / kWave];
    const uint32_t n = d_n ? min(*d_n, n_fixed) : n_fixed;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    if (base >= n) {
        if (threadIdx.x == 0) blk[blockIdx.x] = 0;
        return;
    }
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

// Down-sweep: each tile adds up the totals of the tiles before it (a block-
// wide sum over at most a few thousand words, read from L2), so the scan
// needs no pass over the totals of its own and no workgroup waits on another.
__global__ void __launch_bounds__(kBlock) k_scan_down(const uint32_t* in, uint32_t* out, const uint32_t* d_n,
                                                      uint32_t n_fixed, const uint32_t* __restrict__ blk,
                                                      uint32_t* d_total)
{
    __shared__ uint32_t lds[kBlock / kWave];
    const uint32_t n = d_n ? min(*d_n, n_fixed) : n_fixed;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    if (base >= n) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && d_total) *d_total = 0;   // n == 0
        return;
    }
    uint32_t pre = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kBlock) pre += blk[i];
    // blocked arrangement: thread t owns values [t*I, t*I + I) of the tile
    uint32_t v[kScanItems];
    uint32_t s = 0;
    const uint64_t mine = base + (uint64_t)threadIdx.x * kScanItems;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t i = mine + j;
        v[j] = i < n ? in[i] : 0u;
        s += v[j];
    }
    uint32_t prefix;
    block_excl_scan(pre, lds, &prefix);   // block total of the partial sums = prefix of this tile
    uint32_t tot;
    uint32_t run = block_excl_scan(s, lds, &tot) + prefix;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const uint64_t i = mine + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
    if (d_total && threadIdx.x == 0 && base + kScanTile >= n) *d_total = prefix + tot;
}

// Short arrays (per-cluster counts) are scanned by one workgroup in one
// launch; a two-kernel scan would cost a second launch, which is most of its
// time at these sizes.
__global__ void __launch_bounds__(kOneBlockThreads) k_scan_small(const uint32_t* in, uint32_t* out,
                                                                 const uint32_t* d_n, uint32_t n_fixed,
                                                                 uint32_t* d_total)
{
    const uint32_t n = d_n ? min(*d_n, n_fixed) : n_fixed;
    uint32_t total[1];
    one_block_scan<kOneBlockThreads, 4, 1>(
        n, [&](uint32_t i, uint32_t(&v)[1]) { v[0] = in[i]; }, [&](uint32_t i, const uint32_t(&e)[1]) { out[i] = e[0]; },
        total);
    if (threadIdx.x == 0 && d_total) *d_total = total[0];
}

// ---- radix sort ---------------------------------------------------------------
// A pass runs if it is the first or the bound's digits from `shift` up are
// not all zero (keys are at most the bound).
__device__ __forceinline__ bool radix_pass_runs(const uint32_t* d_max_key, int shift)
{
    return shift == 0 || ((*d_max_key) >> shift) != 0u;
}

// Tiles holding keys: the histograms are laid out digit-major over these
// only, so a sort sized for a large capacity scans and scatters only what
// the device-side count holds.
__device__ __forceinline__ uint32_t radix_tiles(uint32_t n, uint32_t nblk)
{
    const uint32_t t = (uint32_t)(((uint64_t)n + kRadixTile - 1) / kRadixTile);
    return t < nblk ? t : nblk;
}

__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint32_t* __restrict__ keys, const uint32_t* d_n,
                                                       int shift, int passes, const uint32_t* d_max_key, uint32_t nblk,
                                                       uint32_t* __restrict__ hist, uint32_t* __restrict__ scan_n,
                                                       uint32_t* __restrict__ d_sel)
{
    __shared__ uint32_t cnt[kRadixBins];
    const bool runs = radix_pass_runs(d_max_key, shift);
    const uint32_t n = *d_n;
    const uint32_t nt = radix_tiles(n, nblk);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the scan of this pass's histograms covers nothing if the pass is skipped
        *scan_n = runs ? (uint32_t)kRadixBins * nt : 0u;
        if (shift == 0) {
            int ran = 1;
            for (int p = 1; p < passes; ++p) ran += radix_pass_runs(d_max_key, p * kRadixBits) ? 1 : 0;
            *d_sel = (uint32_t)(ran & 1);
        }
    }
    if (!runs || blockIdx.x >= nt) return;
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) cnt[q * kBlock + threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
    for (int j = 0; j < kRadixIters; ++j) {
        const uint64_t i = base + (uint64_t)j * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kRadixBins - 1)], 1u);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) {
        const uint32_t d = q * kBlock + threadIdx.x;
        hist[(uint64_t)d * nt + blockIdx.x] = cnt[d];
    }
}

__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          const uint32_t* d_n, int shift, const uint32_t* d_max_key,
                                                          uint32_t nblk, const uint32_t* __restrict__ hist)
{
    __shared__ uint32_t base[kRadixBins];
    __shared__ uint32_t wcnt[kBlock / kWave][kRadixBins];
    if (!radix_pass_runs(d_max_key, shift)) return;
    const uint32_t n = *d_n;
    const uint32_t nt = radix_tiles(n, nblk);
    const uint64_t tile = (uint64_t)blockIdx.x * kRadixTile;
    if (blockIdx.x >= nt) return;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < kBinsPerThread; ++q) {
        const uint32_t d = q * kBlock + threadIdx.x;
        base[d] = hist[(uint64_t)d * nt + blockIdx.x];
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) wcnt[w][d] = 0;
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int j = 0; j < kRadixIters; ++j) {
        const uint64_t i = tile + (uint64_t)j * kBlock + threadIdx.x;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u;
        const uint32_t v = valid ? vin[i] : 0u;
        const uint32_t dig = (k >> shift) & (kRadixBins - 1);
        // lanes of this wave holding the same digit
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t bb = __ballot(valid && bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t r = (uint32_t)__popcll(m & lt);
        if (valid && r == 0) wcnt[wave][dig] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[dig] + r;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][dig];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kBinsPerThread; ++q) {
            const uint32_t d = q * kBlock + threadIdx.x;
            uint32_t add = 0;
#pragma unroll
            for (int w = 0; w < kBlock / kWave; ++w) { add += wcnt[w][d]; wcnt[w][d] = 0; }
            base[d] += add;
        }
        __syncthreads();
    }
}

}  // namespace

size_t scan_blk_words(uint64_t n_cap)
{
    return (size_t)((n_cap + kScanTile - 1) / kScanTile) + 64;
}

hipError_t scan_exclusive_dev(const uint32_t* in, uint32_t* out, const uint32_t* d_n, uint32_t n_cap,
                              uint32_t* d_total, uint32_t* blk, hipStream_t s)
{
    if (n_cap <= kOneBlockMax) {
        k_scan_small<<<1, kOneBlockThreads, 0, s>>>(in, out, d_n, n_cap, d_total);
        return hipGetLastError();
    }
    uint32_t nblk = (uint32_t)((uint64_t(n_cap) + kScanTile - 1) / kScanTile);
    if (nblk == 0) nblk = 1;   // still writes the total (0)
    k_scan_reduce<<<nblk, kBlock, 0, s>>>(in, d_n, n_cap, blk);
    k_scan_down<<<nblk, kBlock, 0, s>>>(in, out, d_n, n_cap, blk, d_total);
    return hipGetLastError();
}

size_t radix_hist_words(uint64_t n_cap)
{
    return (size_t)kRadixBins * ((n_cap + kRadixTile - 1) / kRadixTile + 1) + 64;
}

hipError_t radix_sort_pairs_dev(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* d_n, uint32_t n_cap,
                                int bits, const uint32_t* d_max_key, uint32_t* hist, uint32_t* blk,
                                uint32_t* d_sel, hipStream_t s)
{
    uint32_t nblk = (uint32_t)((uint64_t(n_cap) + kRadixTile - 1) / kRadixTile);
    if (nblk == 0) nblk = 1;   // still writes *d_sel
    int passes = (bits + kRadixBits - 1) / kRadixBits;
    if (passes < 1) passes = 1;
    const uint32_t hn = (uint32_t)kRadixBins * nblk;
    // per-pass scan lengths live past the histograms (radix_hist_words leaves room)
    uint32_t* scan_n = hist + hn + 8;
    hipError_t e = hipSuccess;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        const int src = p & 1;
        k_radix_hist<<<nblk, kBlock, 0, s>>>(keys[src], d_n, shift, passes, d_max_key, nblk, hist, scan_n + p, d_sel);
        e = scan_exclusive_dev(hist, hist, scan_n + p, hn, nullptr, blk, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<nblk, kBlock, 0, s>>>(keys[src], vals[src], keys[src ^ 1], vals[src ^ 1], d_n, shift,
                                                 d_max_key, nblk, hist);
    }
    return hipGetLastError();
}

}  // namespace vm

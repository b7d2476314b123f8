// vm_peaks.hip -- microbenchmarks for the measured roofline denominators
// (libvm_peaks.so, separate from the segmentation library): a plain fp32
// fused multiply-add loop, a loop of the inlier test in the exact instruction
// form the counting kernels use, and a streaming copy.  Each kernel does a
// fixed, host-known amount of work, so the caller divides it by the time its
// own events measure on `stream`.
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace {

constexpr int kThreads = 256;
constexpr int kChains = 8;   // independent dependency chains per lane

// kChains * iters fmas per lane; the chains are independent so the loop is
// issue-bound, not latency-bound
__global__ void __launch_bounds__(kThreads) k_fma_loop(uint32_t iters, float b, float c, float* __restrict__ sink)
{
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = (float)(threadIdx.x + j) * 1e-3f;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = fmaf(a[j], b, c);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    if (s == 12345.678f) sink[blockIdx.x] = s;   // keeps the loop; practically never stores
}

// iters planes against 16 points per lane, each test the fp32 chain
// |fma(nz, z, fma(ny, y, fma(nx, x, d)))| < eps with a wave ballot and a
// scalar popcount, as in the counting kernels (the plane is wave-uniform)
__global__ void __launch_bounds__(kThreads) k_test_loop(uint32_t iters, float eps, uint32_t* __restrict__ sink)
{
    constexpr int kP = 16;
    float px[kP], py[kP], pz[kP];
#pragma unroll
    for (int j = 0; j < kP; ++j) {
        const float t = (float)(threadIdx.x * kP + j) * 1e-4f;
        px[j] = t;
        py[j] = 0.5f * t;
        pz[j] = 1e-3f * t;
    }
    uint32_t acc = 0;
    float nx = 0.01f, ny = 0.02f, nz = 0.9997f, d = -1e-3f;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kP; ++j) {
            const float dd = fmaf(nz, pz[j], fmaf(ny, py[j], fmaf(nx, px[j], d)));
            acc += (uint32_t)__popcll(__ballot(fabsf(dd) < eps));
        }
        // a new (wave-uniform) plane each iteration, so nothing is hoisted
        d = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(d - 1e-7f)));
    }
    if (acc == 0xFFFFFFFFu) sink[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kThreads) k_copy(const float4* __restrict__ src, float4* __restrict__ dst, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// fp32 fmas: blocks * 256 lanes * 8 chains * iters (2 flops each)
int vmp_fma_loop(uint32_t blocks, uint32_t iters, float* d_sink, void* stream)
{
    if (blocks < 1 || !d_sink) return -1;
    k_fma_loop<<<blocks, kThreads, 0, (hipStream_t)stream>>>(iters, 0.999999f, 1e-6f, d_sink);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// inlier tests: blocks * 256 lanes * 16 points * iters
int vmp_test_loop(uint32_t blocks, uint32_t iters, float eps, uint32_t* d_sink, void* stream)
{
    if (blocks < 1 || !d_sink) return -1;
    k_test_loop<<<blocks, kThreads, 0, (hipStream_t)stream>>>(iters, eps, d_sink);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// n16 16-byte elements read and written
int vmp_copy(const void* d_src, void* d_dst, uint64_t n16, uint32_t blocks, void* stream)
{
    if (!d_src || !d_dst || blocks < 1) return -1;
    k_copy<<<blocks, kThreads, 0, (hipStream_t)stream>>>((const float4*)d_src, (float4*)d_dst, n16);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"

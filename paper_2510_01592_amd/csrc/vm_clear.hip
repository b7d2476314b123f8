// vm_clear.hip -- free space along the sensor rays (Sec. III-B, Eq. (2)).
//
//   k_clear_cast:  a wave per point transforms it as the insert does, marks
//                  its voxel in the `keep` bitmap when that voxel is
//                  occupied, and walks the 3D Bresenham line from the
//                  sensor's voxel towards it (its own voxel excluded, cut at
//                  the grid's faces) with its lanes over the steps, marking
//                  every occupied voxel it passes in the `ray` bitmap.  A
//                  mark is an atomic OR only when a plain read shows the bit
//                  still clear.
//   k_clear_apply: a thread per 32-cell word frees the cells marked on a ray
//                  and not kept (count and sums zeroed in the hash slot, the
//                  occupancy bit cleared), and leaves both bitmaps zero for
//                  the next call.
// The two bitmaps deduplicate the removal set: whatever the number of rays
// through a voxel, its slot is written once, by the one thread that owns its
// word, after every ray has been cast.
#include "vm_common.h"

namespace vm {
namespace {

__device__ __forceinline__ void mark_bit(uint32_t* __restrict__ bm, uint32_t key)
{
    const uint32_t bit = 1u << (key & 31);
    uint32_t* w = &bm[key >> 5];
    if (!(__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit)) atomicOr(w, bit);
}

struct CastArgs {
    Pose pose;
    Geom g;
    int32_t s[3];            // the sensor's voxel
    const uint32_t* bits;    // occupancy
    uint32_t* ray;           // cells on a ray (occupied ones only)
    uint32_t* keep;          // cells holding a point of the frame (occupied ones only)
};

// One wave per ray.  The Bresenham walk has a closed form: after k steps
// along the driving axis m, a minor axis with extent d has moved
// floor((2 d k + dm) / (2 dm)) times (the error-term rule, a step when the
// term reaches zero, unrolled), so lane l takes steps l, l + 64, ... and
// keeps each minor coordinate as a quotient and remainder, advanced by the
// constant increments of 64 steps.  The walk leaves the grid at the first
// step where some coordinate does (each moves one way only); that step is
// computed up front per axis, so every lane knows where to stop.
template <typename T>
__device__ __forceinline__ void walk_lanes(const CastArgs& a, int lane, T dm, T du, T dw, T nsteps, uint32_t key0,
                                           uint32_t Sm, uint32_t Su, uint32_t Sw)
{
    const T two_dm = 2 * dm;
    T k = (T)lane;
    // the minor axes' moves after k steps: quotient and remainder of 2 d k + dm by 2 dm
    int64_t nu = 2 * (int64_t)du * (int64_t)lane + (int64_t)dm, nw = 2 * (int64_t)dw * (int64_t)lane + (int64_t)dm;
    T U = (T)(nu / (int64_t)two_dm), ru = (T)(nu % (int64_t)two_dm);
    T W = (T)(nw / (int64_t)two_dm), rw = (T)(nw % (int64_t)two_dm);
    // their increments over 64 steps
    const int64_t iu = 2 * (int64_t)du * kWave, iw = 2 * (int64_t)dw * kWave;
    const T qu = (T)(iu / (int64_t)two_dm), pu = (T)(iu % (int64_t)two_dm);
    const T qw = (T)(iw / (int64_t)two_dm), pw = (T)(iw % (int64_t)two_dm);
    for (; k < nsteps; k += kWave) {
        const uint32_t key = key0 + Sm * (uint32_t)k + Su * (uint32_t)U + Sw * (uint32_t)W;
        if ((a.bits[key >> 5] >> (key & 31)) & 1u) mark_bit(a.ray, key);
        U += qu;
        ru += pu;
        if (ru >= two_dm) {
            ++U;
            ru -= two_dm;
        }
        W += qw;
        rw += pw;
        if (rw >= two_dm) {
            ++W;
            rw -= two_dm;
        }
    }
}

// first step at which a coordinate starting at c and moving by g per move
// leaves [0, D), in steps of the driving axis: moves = floor((2 d k + dm) / (2 dm))
__device__ __forceinline__ int64_t exit_step(int64_t c, int32_t g, int64_t D, int64_t d, int64_t dm)
{
    const int64_t L = g > 0 ? D - c : c + 1;   // moves that stay inside
    if (d == 0) return (int64_t)0x7FFFFFFFFFFFFFFFll;
    return (2 * dm * L - dm + 2 * d - 1) / (2 * d);
}

__global__ void __launch_bounds__(kBlock) k_clear_cast(const float* __restrict__ xyz, int64_t n, CastArgs a)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const int32_t NX = a.g.dims[0], NY = a.g.dims[1], NZ = a.g.dims[2];
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < n; i += nwaves) {
        // the point (every lane of the wave computes the same values)
        const double px = (double)xyz[3 * i + 0];
        const double py = (double)xyz[3 * i + 1];
        const double pz = (double)xyz[3 * i + 2];
        const double wx = fma(a.pose.R[2], pz, fma(a.pose.R[1], py, fma(a.pose.R[0], px, a.pose.t[0])));
        const double wy = fma(a.pose.R[5], pz, fma(a.pose.R[4], py, fma(a.pose.R[3], px, a.pose.t[1])));
        const double wz = fma(a.pose.R[8], pz, fma(a.pose.R[7], py, fma(a.pose.R[6], px, a.pose.t[2])));
        const double fx = floor((wx - a.g.origin[0]) * a.g.inv_q);
        const double fy = floor((wy - a.g.origin[1]) * a.g.inv_q);
        const double fz = floor((wz - a.g.origin[2]) * a.g.inv_q);
        // no ray for non-finite points or points absurdly far away (the
        // negated test also rejects NaN)
        if (!(fx >= -1e15 && fx <= 1e15 && fy >= -1e15 && fy <= 1e15 && fz >= -1e15 && fz <= 1e15)) continue;
        // the point's voxel: floor division of the fixed-point coordinate
        const int64_t e0 = (int64_t)fx >> 20, e1 = (int64_t)fy >> 20, e2 = (int64_t)fz >> 20;
        if (lane == 0 && e0 >= 0 && e1 >= 0 && e2 >= 0 && e0 < NX && e1 < NY && e2 < NZ) {
            const uint32_t k = (uint32_t)e0 + (uint32_t)NX * ((uint32_t)e1 + (uint32_t)NY * (uint32_t)e2);
            if ((a.bits[k >> 5] >> (k & 31)) & 1u) mark_bit(a.keep, k);
        }
        // Bresenham on (driving axis m, minor axes u = m+1, w = m+2 mod 3)
        const int64_t d0 = e0 - a.s[0], d1 = e1 - a.s[1], d2 = e2 - a.s[2];
        const int64_t ad0 = d0 < 0 ? -d0 : d0, ad1 = d1 < 0 ? -d1 : d1, ad2 = d2 < 0 ? -d2 : d2;
        int m = 0;
        if (ad1 > ad0) m = 1;
        if (ad2 > (m == 0 ? ad0 : ad1)) m = 2;
        const int64_t dm = m == 0 ? ad0 : (m == 1 ? ad1 : ad2);
        if (dm == 0) continue;
        const int64_t du = m == 0 ? ad1 : (m == 1 ? ad2 : ad0);
        const int64_t dw = m == 0 ? ad2 : (m == 1 ? ad0 : ad1);
        const int32_t gm = (m == 0 ? d0 : (m == 1 ? d1 : d2)) < 0 ? -1 : 1;
        const int32_t gu = (m == 0 ? d1 : (m == 1 ? d2 : d0)) < 0 ? -1 : 1;
        const int32_t gw = (m == 0 ? d2 : (m == 1 ? d0 : d1)) < 0 ? -1 : 1;
        const int64_t Dm = m == 0 ? NX : (m == 1 ? NY : NZ);
        const int64_t Du = m == 0 ? NY : (m == 1 ? NZ : NX);
        const int64_t Dw = m == 0 ? NZ : (m == 1 ? NX : NY);
        const int64_t cm = m == 0 ? a.s[0] : (m == 1 ? a.s[1] : a.s[2]);
        const int64_t cu = m == 0 ? a.s[1] : (m == 1 ? a.s[2] : a.s[0]);
        const int64_t cw = m == 0 ? a.s[2] : (m == 1 ? a.s[0] : a.s[1]);
        int64_t nsteps = dm;
        const int64_t xm = gm > 0 ? Dm - cm : cm + 1;
        nsteps = nsteps < xm ? nsteps : xm;
        const int64_t xu = exit_step(cu, gu, Du, du, dm), xw = exit_step(cw, gw, Dw, dw, dm);
        nsteps = nsteps < xu ? nsteps : xu;
        nsteps = nsteps < xw ? nsteps : xw;
        // key strides, applied with the step's sign in modulo-2^32 arithmetic
        // (the grid has fewer than 2^32 cells, so keys inside it are exact)
        const uint32_t sx = 1u, sy = (uint32_t)NX, sz = (uint32_t)NX * (uint32_t)NY;
        const uint32_t Sm = (m == 0 ? sx : (m == 1 ? sy : sz)) * (uint32_t)gm;
        const uint32_t Su = (m == 0 ? sy : (m == 1 ? sz : sx)) * (uint32_t)gu;
        const uint32_t Sw = (m == 0 ? sz : (m == 1 ? sx : sy)) * (uint32_t)gw;
        const uint32_t key0 = (uint32_t)a.s[0] + (uint32_t)NX * ((uint32_t)a.s[1] + (uint32_t)NY * (uint32_t)a.s[2]);
        // 32-bit walk state while 2 dm fits comfortably (quotients < dm, remainders < 2 dm)
        if (dm < ((int64_t)1 << 29))
            walk_lanes<int32_t>(a, lane, (int32_t)dm, (int32_t)du, (int32_t)dw, (int32_t)nsteps, key0, Sm, Su, Sw);
        else
            walk_lanes<int64_t>(a, lane, dm, du, dw, nsteps, key0, Sm, Su, Sw);
    }
}

__global__ void __launch_bounds__(kBlock) k_clear_apply(Hash h, uint32_t* __restrict__ bits, uint32_t nwords,
                                                        uint32_t* __restrict__ ray, uint32_t* __restrict__ keep,
                                                        DevCounters* __restrict__ ctr)
{
    uint32_t removed = 0;
    for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += gridDim.x * blockDim.x) {
        const uint32_t r = ray[w], k = keep[w];
        if (r) ray[w] = 0u;
        if (k) keep[w] = 0u;
        const uint32_t b = bits[w];
        uint32_t c = r & ~k & b;
        if (!c) continue;
        bits[w] = b & ~c;
        removed += (uint32_t)__popc(c);
        while (c) {
            const int j = __ffs(c) - 1;
            c &= c - 1u;
            const uint32_t s = hash_find(h, w * 32u + (uint32_t)j);
            if (s == kEmpty) continue;   // cannot happen for an occupied cell
            Slot* sl = &h.slot[s];
            sl->cnt = 0u;
            sl->sum[0] = 0ull;
            sl->sum[1] = 0ull;
            sl->sum[2] = 0ull;
        }
    }
    // one pair of atomics per block: occupied -= removed, cleared += removed
    __shared__ uint32_t part[kBlock / kWave];
    uint32_t t = removed;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) t += __shfl_xor(t, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) tot += part[q];
        if (tot) {
            atomicAdd(&ctr->occupied, 0ull - tot);
            atomicAdd(&ctr->cleared, tot);
        }
    }
}

}  // namespace

hipError_t launch_clear_rays(const float* xyz, int64_t n, const Pose& pose, const Geom& g, const int32_t sensor[3],
                             const Hash& h, uint32_t* bits, uint32_t* ray, uint32_t* keep, DevCounters* ctr,
                             hipStream_t s)
{
    if (n > 0) {
        CastArgs a;
        a.pose = pose;
        a.g = g;
        a.s[0] = sensor[0];
        a.s[1] = sensor[1];
        a.s[2] = sensor[2];
        a.bits = bits;
        a.ray = ray;
        a.keep = keep;
        k_clear_cast<<<grid_for((uint64_t)n), kBlock, 0, s>>>(xyz, n, a);
    }
    k_clear_apply<<<grid_for(g.nwords), kBlock, 0, s>>>(h, bits, g.nwords, ray, keep, ctr);
    return hipGetLastError();
}

}  // namespace vm

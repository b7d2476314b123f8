// vm_hull.hip -- boundary polygons (Sec. III-C, "Boundary polygon
// generation"): the convex hull of each plane's inliers, in the plane.
//
// The paper filters most points on the GPU and finishes the hull on the CPU
// from the few candidates left.  Here the whole hull stays on the device, one
// workgroup per cluster:
//   1. project the inliers onto an orthonormal in-plane basis (fp64);
//   2. find the extreme inlier in each of 8 directions (every 45 degrees);
//      these are hull points, and the convex polygon through them lies inside
//      the hull, so any point strictly inside it (by a margin far above the
//      fp64 rounding of the test) cannot be a hull vertex and is dropped;
//   3. sort the survivors by (u, v, inlier index) -- bitonic in LDS, or in
//      global memory for very large survivor sets;
//   4. Andrew's monotone chain over the survivors, popping on every non-left
//      turn (strictly convex output, counter-clockwise from the smallest point).
// A second pass packs the polygons into the caller's CSR and projects each
// vertex onto the plane.
#include "vm_common.h"

#include <math.h>

namespace vm {
namespace {

constexpr int kHullBlock = 512;
constexpr int kLdsCap = 2048;   // survivors sorted in LDS; more go through global memory

struct P2 {
    double u, v;
    uint32_t i;
};

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
    double u[3], v[3], n[3];
};

__device__ __forceinline__ Basis plane_basis(float4 pl)
{
    Basis b;
    b.n[0] = pl.x;
    b.n[1] = pl.y;
    b.n[2] = pl.z;
    double a[3] = {0.0, 0.0, 0.0};
    if (fabs(b.n[0]) < 0.9) a[0] = 1.0;
    else a[1] = 1.0;
    const double c0 = a[1] * b.n[2] - a[2] * b.n[1];
    const double c1 = a[2] * b.n[0] - a[0] * b.n[2];
    const double c2 = a[0] * b.n[1] - a[1] * b.n[0];
    const double inv = 1.0 / sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    b.u[0] = c0 * inv;
    b.u[1] = c1 * inv;
    b.u[2] = c2 * inv;
    b.v[0] = b.n[1] * b.u[2] - b.n[2] * b.u[1];
    b.v[1] = b.n[2] * b.u[0] - b.n[0] * b.u[2];
    b.v[2] = b.n[0] * b.u[1] - b.n[1] * b.u[0];
    return b;
}

// directional functional of direction d (0..7, every 45 degrees, CCW from +u)
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

__global__ void __launch_bounds__(kBlock) k_hull_k(const uint32_t* __restrict__ meta, uint32_t kc, uint32_t n_cap,
                                                   const uint32_t* __restrict__ off, uint32_t* small,
                                                   uint32_t* status)
{
    __shared__ int bad;
    const uint32_t K = validate_clusters(meta, off, kc, n_cap, status, &bad);
    if (threadIdx.x == 0) small[4] = K;
}

__global__ void __launch_bounds__(kHullBlock) k_hull(const uint32_t* __restrict__ small,
                                                     const uint32_t* __restrict__ off, const float* __restrict__ X,
                                                     const float* __restrict__ Y, const float* __restrict__ Z,
                                                     const int32_t* __restrict__ best, const float4* __restrict__ plane,
                                                     const uint32_t* __restrict__ in_off,
                                                     const uint32_t* __restrict__ in_idx, uint32_t in_cap,
                                                     uint32_t* __restrict__ hull_cnt, uint32_t* __restrict__ hull_tmp,
                                                     double* __restrict__ gu, double* __restrict__ gv,
                                                     uint32_t* __restrict__ gi, double* __restrict__ area_out,
                                                     uint32_t* __restrict__ status)
{
    __shared__ double su[kLdsCap];
    __shared__ double sv[kLdsCap];
    __shared__ uint32_t si[kLdsCap];
    __shared__ uint16_t stk[kLdsCap + 2];
    __shared__ double red_val[kHullBlock / kWave][8];
    __shared__ uint32_t red_idx[kHullBlock / kWave][8];
    __shared__ double poly_u[8], poly_v[8];
    __shared__ int npoly;
    __shared__ uint32_t nsurv;
    __shared__ double margin;

    const uint32_t K = small[4];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;

    for (uint32_t k = blockIdx.x; k < K; k += gridDim.x) {
        const uint32_t ib = in_off[k], ie = in_off[k + 1];
        if (best[k] < 0 || ie <= ib || ie > in_cap) {
            if (threadIdx.x == 0) {
                hull_cnt[k] = 0;
                area_out[k] = 0.0;
                if (best[k] >= 0 && ie > in_cap) atomicOr(status, (uint32_t)VM_FLAG_INLIERS_CAP);
            }
            continue;
        }
        const uint32_t m = ie - ib;
        const uint32_t pb = off[k];
        const uint32_t nk = off[k + 1] - pb;
        if (in_idx[ib] >= nk) {   // inlier lists must index the cluster's own points
            if (threadIdx.x == 0) {
                hull_cnt[k] = 0;
                area_out[k] = 0.0;
            }
            continue;
        }
        const Basis B = plane_basis(plane[k]);
        const uint32_t i0 = pb + in_idx[ib];
        const double ox = X[i0], oy = Y[i0], oz = Z[i0];

        // ---- 1+2a: extreme points in 8 directions --------------------------------
        double bv[8];
        uint32_t bi[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) { bv[d] = -INFINITY; bi[d] = 0xFFFFFFFFu; }
        for (uint32_t j = threadIdx.x; j < m; j += kHullBlock) {
            const uint32_t li = in_idx[ib + j];
            if (li >= nk) continue;
            const uint32_t i = pb + li;
            const double dx = (double)X[i] - ox, dy = (double)Y[i] - oy, dz = (double)Z[i] - oz;
            const double pu = B.u[0] * dx + B.u[1] * dy + B.u[2] * dz;
            const double pv = B.v[0] * dx + B.v[1] * dy + B.v[2] * dz;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const double f = dir_val(d, pu, pv);
                if (f > bv[d] || (f == bv[d] && j < bi[d])) { bv[d] = f; bi[d] = j; }
            }
        }
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            for (int s = kWave / 2; s >= 1; s >>= 1) {
                const double ov = __shfl_xor(bv[d], s, kWave);
                const uint32_t oi = __shfl_xor(bi[d], s, kWave);
                if (ov > bv[d] || (ov == bv[d] && oi < bi[d])) { bv[d] = ov; bi[d] = oi; }
            }
            if (lane == 0) { red_val[wave][d] = bv[d]; red_idx[wave][d] = bi[d]; }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t e[8];
            for (int d = 0; d < 8; ++d) {
                double v = red_val[0][d];
                uint32_t ix = red_idx[0][d];
                for (int w = 1; w < kHullBlock / kWave; ++w)
                    if (red_val[w][d] > v || (red_val[w][d] == v && red_idx[w][d] < ix)) { v = red_val[w][d]; ix = red_idx[w][d]; }
                e[d] = ix;
            }
            // distinct extreme points in CCW order
            int np = 0;
            uint32_t q[8];
            bool found = true;
            for (int d = 0; d < 8; ++d) found = found && e[d] < m;
            for (int d = 0; found && d < 8; ++d)
                if (np == 0 || q[np - 1] != e[d]) q[np++] = e[d];
            while (np > 1 && q[np - 1] == q[0]) --np;
            double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
            for (int a = 0; a < np; ++a) {
                const uint32_t i = pb + in_idx[ib + q[a]];
                const double dx = (double)X[i] - ox, dy = (double)Y[i] - oy, dz = (double)Z[i] - oz;
                poly_u[a] = B.u[0] * dx + B.u[1] * dy + B.u[2] * dz;
                poly_v[a] = B.v[0] * dx + B.v[1] * dy + B.v[2] * dz;
                umin = fmin(umin, poly_u[a]); umax = fmax(umax, poly_u[a]);
                vmin = fmin(vmin, poly_v[a]); vmax = fmax(vmax, poly_v[a]);
            }
            const double span = fmax(umax - umin, vmax - vmin);
            // margin: far above fp64 rounding of a cross product at this scale
            margin = 1e-9 * span * span + 1e-300;
            bool convex = np >= 3;
            for (int a = 0; convex && a < np; ++a) {
                const int b2 = (a + 1) % np, c2 = (a + 2) % np;
                if (cross3(poly_u[a], poly_v[a], poly_u[b2], poly_v[b2], poly_u[c2], poly_v[c2]) <= margin) convex = false;
            }
            npoly = convex ? np : 0;
            nsurv = 0;
        }
        __syncthreads();

        // ---- 2b: survivors (not strictly inside the extreme polygon) ------------------
        const int np = npoly;
        const double mg = margin;
        for (uint32_t j = threadIdx.x; j < m; j += kHullBlock) {
            const uint32_t li = in_idx[ib + j];
            if (li >= nk) continue;
            const uint32_t i = pb + li;
            const double dx = (double)X[i] - ox, dy = (double)Y[i] - oy, dz = (double)Z[i] - oz;
            const double pu = B.u[0] * dx + B.u[1] * dy + B.u[2] * dz;
            const double pv = B.v[0] * dx + B.v[1] * dy + B.v[2] * dz;
            bool inside = np >= 3;
            for (int a = 0; inside && a < np; ++a) {
                const int b2 = (a + 1 == np) ? 0 : a + 1;
                inside = cross3(poly_u[a], poly_v[a], poly_u[b2], poly_v[b2], pu, pv) > mg;
            }
            if (!inside) {
                const uint32_t slot = atomicAdd(&nsurv, 1u);
                gu[ib + slot] = pu;
                gv[ib + slot] = pv;
                gi[ib + slot] = j;
            }
        }
        __syncthreads();
        const uint32_t ns = nsurv;

        // ---- 3: sort survivors by (u, v, index) -------------------------------------------
        double* Su;
        double* Sv;
        uint32_t* Si;
        if (ns <= (uint32_t)kLdsCap) {
            uint32_t N = 1;
            while (N < ns) N <<= 1;
            for (uint32_t t = threadIdx.x; t < N; t += kHullBlock) {
                if (t < ns) { su[t] = gu[ib + t]; sv[t] = gv[ib + t]; si[t] = gi[ib + t]; }
                else { su[t] = INFINITY; sv[t] = INFINITY; si[t] = 0xFFFFFFFFu; }
            }
            __syncthreads();
            for (uint32_t size = 2; size <= N; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t t = threadIdx.x; t < N / 2; t += kHullBlock) {
                        const uint32_t a = 2 * t - (t & (stride - 1));
                        const uint32_t b2 = a + stride;
                        const bool up = (a & size) == 0;
                        const bool lt = p2_less(su[b2], sv[b2], si[b2], su[a], sv[a], si[a]);
                        if (lt == up) {
                            const double tu = su[a], tv = sv[a];
                            const uint32_t ti = si[a];
                            su[a] = su[b2]; sv[a] = sv[b2]; si[a] = si[b2];
                            su[b2] = tu; sv[b2] = tv; si[b2] = ti;
                        }
                    }
                    __syncthreads();
                }
            }
            Su = su; Sv = sv; Si = si;
        } else {
            // bitonic network on the survivors in global memory; partners beyond
            // ns are +infinity and never move
            uint32_t N = 1;
            while (N < ns) N <<= 1;
            double* U = gu + ib;
            double* Vv = gv + ib;
            uint32_t* I = gi + ib;
            for (uint32_t size = 2; size <= N; size <<= 1) {
                for (uint32_t t = threadIdx.x; t < N / 2; t += kHullBlock) {
                    const uint32_t blk = t / (size >> 1), r = t % (size >> 1);
                    const uint32_t a = blk * size + r, b2 = blk * size + size - 1 - r;
                    if (b2 < ns && p2_less(U[b2], Vv[b2], I[b2], U[a], Vv[a], I[a])) {
                        const double tu = U[a], tv = Vv[a];
                        const uint32_t ti = I[a];
                        U[a] = U[b2]; Vv[a] = Vv[b2]; I[a] = I[b2];
                        U[b2] = tu; Vv[b2] = tv; I[b2] = ti;
                    }
                }
                __syncthreads();
                for (uint32_t stride = size >> 2; stride > 0; stride >>= 1) {
                    for (uint32_t t = threadIdx.x; t < N / 2; t += kHullBlock) {
                        const uint32_t a = 2 * t - (t & (stride - 1));
                        const uint32_t b2 = a + stride;
                        if (b2 < ns && p2_less(U[b2], Vv[b2], I[b2], U[a], Vv[a], I[a])) {
                            const double tu = U[a], tv = Vv[a];
                            const uint32_t ti = I[a];
                            U[a] = U[b2]; Vv[a] = Vv[b2]; I[a] = I[b2];
                            U[b2] = tu; Vv[b2] = tv; I[b2] = ti;
                        }
                    }
                    __syncthreads();
                }
            }
            Su = U; Sv = Vv; Si = I;
        }

        // ---- 4: monotone chain (one lane) ------------------------------------------------
        if (threadIdx.x == 0) {
            const bool lds_stack = ns <= (uint32_t)kLdsCap;
            // cluster k owns hull_tmp[ib + k, ib + k + m + 1): the chain's stack never
            // holds more than (survivors + 1) <= m + 1 entries
            uint32_t* gst = hull_tmp + ib + k;
            auto st_get = [&](uint32_t q) -> uint32_t { return lds_stack ? (uint32_t)stk[q] : gst[q]; };
            auto st_set = [&](uint32_t q, uint32_t v) {
                if (lds_stack) stk[q] = (uint16_t)v;
                else gst[q] = v;
            };
            uint32_t h = 0;
            if (ns == 1) {
                st_set(h++, 0);
            } else {
                for (uint32_t i = 0; i < ns; ++i) {
                    while (h >= 2) {
                        const uint32_t a = st_get(h - 2), b2 = st_get(h - 1);
                        if (cross3(Su[a], Sv[a], Su[b2], Sv[b2], Su[i], Sv[i]) <= 0.0) --h;
                        else break;
                    }
                    st_set(h++, i);
                }
                const uint32_t lower = h + 1;
                for (int32_t i = (int32_t)ns - 2; i >= 0; --i) {
                    while (h >= lower) {
                        const uint32_t a = st_get(h - 2), b2 = st_get(h - 1);
                        if (cross3(Su[a], Sv[a], Su[b2], Sv[b2], Su[i], Sv[i]) <= 0.0) --h;
                        else break;
                    }
                    st_set(h++, (uint32_t)i);
                }
                --h;
            }
            double s = 0.0;
            if (h >= 3) {
                for (uint32_t q = 0; q < h; ++q) {
                    const uint32_t a = st_get(q), b2 = st_get(q + 1 == h ? 0 : q + 1);
                    s = s + (Su[a] * Sv[b2] - Su[b2] * Sv[a]);
                }
            }
            area_out[k] = h >= 3 ? 0.5 * s : 0.0;
            // vertex list: cluster-local point indices (the stack is read before
            // hull_tmp is overwritten, entry by entry in increasing order)
            for (uint32_t q = 0; q < h; ++q) {
                const uint32_t j = Si[st_get(q)];
                hull_tmp[ib + k + q] = in_idx[ib + j];
            }
            hull_cnt[k] = h;
        }
        __syncthreads();
    }
}

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
            if (pos >= v_cap) { over = true; continue; }
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

vm_status hulls(const vm_clusters& cl, const vm_planes& planes, const vm_hulls_out& out, const WorkLayout& w,
                hipStream_t s)
{
    uint32_t kc = cl.k_cap;
    if (planes.k_cap < kc) kc = planes.k_cap;
    if (out.k_cap < kc) kc = out.k_cap;
    StageScope t(VM_STAGE_HULL, s);
    k_hull_k<<<1, kBlock, 0, s>>>(cl.d_meta, kc, cl.n_cap, cl.d_off, w.small, out.d_status);
    const int grid = kc < 4096 ? (int)(kc ? kc : 1) : 4096;
    k_hull<<<grid, kHullBlock, 0, s>>>(w.small, cl.d_off, cl.d_x, cl.d_y, cl.d_z, planes.d_best_h,
                                       (const float4*)planes.d_plane, planes.d_in_off, planes.d_in_idx, planes.in_cap,
                                       w.hull_cnt, w.hull_tmp, w.hull_u, w.hull_v, w.hull_i, out.d_area, out.d_status);
    VM_HIP(hipGetLastError());
    VM_HIP(scan_exclusive_dev(w.hull_cnt, w.hull_off, w.small + 4, kc, w.small + 5, w.blk, s));
    k_hull_pack<<<grid, kBlock, 0, s>>>(w.small, cl.d_off, cl.d_x, cl.d_y, cl.d_z, (const float4*)planes.d_plane,
                                         planes.d_in_off, w.hull_cnt, w.hull_tmp, w.hull_off, out.v_cap, out.d_v_off,
                                         out.d_v_idx, out.d_v_xyz, out.d_status);
    VM_HIP(hipGetLastError());
    return VM_OK;
}

}  // namespace vm

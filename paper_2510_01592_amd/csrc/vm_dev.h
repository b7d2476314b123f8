// vm_dev.h -- device functions shared by the library's kernels (gfx950):
// the counter-based generator and the hypothesis plane of Sec. III-C (a), the
// inlier test of (b), and the in-plane projection, orientation test and
// monotone-chain building blocks of the boundary polygons.
#pragma once
#include "vm_common.h"

#include <math.h>

namespace vm {
namespace dev {

// The 128-bit product of two 64-bit words from four 32 x 32 -> 64 bit
// multiply-adds (the high and the low half of one product; computing them
// as separate 64-bit operations repeats partial products).
__device__ __forceinline__ void mul_64x64_128(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t t = (uint64_t)a0 * b1 + (p00 >> 32);             // < 2^64
    const uint64_t t2 = (uint64_t)a1 * b0 + (uint32_t)t;            // < 2^64
    lo = (t2 << 32) | (uint32_t)p00;
    hi = (uint64_t)a1 * b1 + (t >> 32) + (t2 >> 32);
}

__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1, uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mul_64x64_128(M0, c0, hi0, lo0);
        mul_64x64_128(M1, c2, hi1, lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Sec. III-C (a): hypothesis h of a cluster of n points (pointers at its
// first point): three distinct points drawn with Philox4x64-10, key (seed, 0)
// and counter (h, tag, frame, 0); the plane through them in fp64 (unit
// normal with +z first, then +y, then +x; offset from the first point),
// rounded to float32.  Degenerate triples (and n < 3) give a NaN plane.
__device__ __forceinline__ float4 hyp_plane(const float* __restrict__ X, const float* __restrict__ Y,
                                            const float* __restrict__ Z, uint64_t n, uint32_t h, uint32_t tag,
                                            uint32_t frame, uint64_t seed)
{
    const float qnan = __builtin_nanf("");
    float4 pl = make_float4(qnan, qnan, qnan, qnan);
    if (n >= 3) {
        uint64_t r[4];
        philox4x64_10(h, tag, frame, 0, seed, 0, r);
        const uint64_t u0 = r[0] >> 32, u1 = r[1] >> 32, u2 = r[2] >> 32;
        const uint64_t ia = (u0 * n) >> 32;
        uint64_t ib = (u1 * (n - 1)) >> 32;
        if (ib >= ia) ib += 1;
        uint64_t ic = (u2 * (n - 2)) >> 32;
        const uint64_t lo = ia < ib ? ia : ib, hi = ia < ib ? ib : ia;
        if (ic >= lo) ic += 1;
        if (ic >= hi) ic += 1;
        const double ax = X[ia], ay = Y[ia], az = Z[ia];
        const double e1x = (double)X[ib] - ax, e1y = (double)Y[ib] - ay, e1z = (double)Z[ib] - az;
        const double e2x = (double)X[ic] - ax, e2y = (double)Y[ic] - ay, e2z = (double)Z[ic] - az;
        double nx = e1y * e2z - e1z * e2y;
        double ny = e1z * e2x - e1x * e2z;
        double nz = e1x * e2y - e1y * e2x;
        const double nn = nx * nx + ny * ny + nz * nz;
        if (nn >= 1e-24) {
            const double inv = 1.0 / sqrt(nn);
            nx = nx * inv;
            ny = ny * inv;
            nz = nz * inv;
            if (nz < 0.0 || (nz == 0.0 && (ny < 0.0 || (ny == 0.0 && nx < 0.0)))) {
                nx = -nx;
                ny = -ny;
                nz = -nz;
            }
            const double d = -(nx * ax + ny * ay + nz * az);
            pl = make_float4((float)nx, (float)ny, (float)nz, (float)d);
        }
    }
    return pl;
}

// Sec. III-C (b): the inlier test of a point against a plane, as specified
__device__ __forceinline__ bool inlier_test(const float4 pl, float x, float y, float z, float eps)
{
    return fabsf(fmaf(pl.z, z, fmaf(pl.y, y, fmaf(pl.x, x, pl.w)))) < eps;
}

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

__device__ __forceinline__ void project(const ClusterFrame& f, float x, float y, float z, double* pu, double* pv)
{
    const double dx = (double)x - f.ox, dy = (double)y - f.oy, dz = (double)z - f.oz;
    *pu = f.B.u[0] * dx + f.B.u[1] * dy + f.B.u[2] * dz;
    *pv = f.B.v[0] * dx + f.B.v[1] * dy + f.B.v[2] * dz;
}

// The convex polygon through a cluster's extreme inliers e[0..kDirs) (their
// positions in the inlier list, m entries; repeated ones merged), projected
// by point(j, &u, &v).  Corners that do not turn left by more than a margin
// (far above the fp64 rounding of a cross product at the polygon's scale)
// are pruned until every corner is strictly convex; the rest bound a convex
// polygon inside the hull.  P receives u[kDirs], v[kDirs], the margin and
// the vertex count (0: fewer than 3 corners, no filtering).
template <class PointOf>
__device__ __forceinline__ void extreme_polygon(const uint32_t (&e)[kDirs], uint32_t m, double* P, PointOf point)
{
    int np = 0;
    uint32_t q[kDirs];
    bool found = true;
    for (int d = 0; d < kDirs; ++d) found = found && e[d] < m;
    for (int d = 0; found && d < kDirs; ++d)
        if (np == 0 || q[np - 1] != e[d]) q[np++] = e[d];
    while (np > 1 && q[np - 1] == q[0]) --np;
    double pu[kDirs], pv[kDirs];
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    for (int a = 0; a < np; ++a) {
        point(q[a], &pu[a], &pv[a]);
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


// One wave's hull of at most 64 points, one per lane (u, v and i = the
// point's position in its list; lanes >= ns hold +inf and 0xFFFFFFFF): the
// points are sorted across the lanes by (u, v, i) with a bitonic network on
// shuffles, then lane 0 builds the lower and lane 1 at the same time the
// upper chain, each with its two top points in registers.  su/sv/si (64
// entries) and st (2*64+2) are this wave's LDS scratch.  Returns the vertex
// count h and the shoelace area (on every lane) and, for lane < h, the
// sorted position vi of vertex `lane` (counter-clockwise from the smallest
// point): its list position is si[vi].
struct WaveHull {
    uint32_t h, vi;
    double area;
};

__device__ __forceinline__ WaveHull wave_hull(double u, double v, uint32_t i, uint32_t ns, int lane, double* su,
                                              double* sv, uint32_t* si, uint8_t* st)
{
    WaveHull r;
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
    su[lane] = u;
    sv[lane] = v;
    si[lane] = i;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // lane 0 builds the lower chain (points in sorted order), lane 1 at
    // the same time the upper one (reverse order), each with the two top
    // points of its stack held in registers
    uint32_t h = 0;
    if (lane < 2) {
        const double* U = su;
        const double* V = sv;
        uint8_t* S = st + (lane ? kWave + 1 : 0);
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
        return p < hl ? st[p] : st[kWave + 1 + (p - hl + 1)];
    };
    double term = 0.0;
    uint32_t vi = 0;
    if ((uint32_t)lane < h) {
        vi = vertex((uint32_t)lane);
        const uint32_t v1 = vertex((uint32_t)lane + 1 == h ? 0u : (uint32_t)lane + 1);
        term = su[vi] * sv[v1] - su[v1] * sv[vi];
    }
    // shoelace sum over the vertices (a wave reduction)
#pragma unroll
    for (int dd = kWave / 2; dd >= 1; dd >>= 1) term += __shfl_xor(term, dd, kWave);
    r.h = h;
    r.vi = vi;
    r.area = h >= 3 ? 0.5 * term : 0.0;
    return r;
}

constexpr int kChainBlock = 256;   // threads of block_chain

// LDS scratch of block_chain for up to Cap points.
template <int Cap>
struct ChainLds {
    double su[Cap];
    double sv[Cap];
    uint32_t si[Cap];
    uint16_t st_lo[2 * Cap];
    uint16_t st_up[Cap + 1];
    uint16_t tmp_lo[Cap];
    uint16_t tmp_up[Cap];
    uint16_t seq_lo[Cap];
    uint16_t seq_up[Cap];
    uint32_t offs_lo[kWave + 1], offs_up[kWave + 1];
    uint32_t len2_lo[kChainL2], len2_up[kChainL2];
    uint32_t hlo, hup;
    double red[kChainBlock / kWave];
};

// The hull of ns <= Cap points by one workgroup of kChainBlock threads: the
// points (load(t, &u, &v, &i) gives point t) are sorted in L by (u, v, i)
// -- one point per thread with shuffles for short distances, or a bitonic
// network in LDS -- then the lower chain runs on wave 0 and the upper one on
// wave 1 in the three levels of chain_level1/2 and chain_run.  emit(q, p)
// receives vertex q (counter-clockwise from the smallest point) as sorted
// position p (list position L.si[p]); thread 0 gets the shoelace area.
// Returns the vertex count.
template <int Cap, class Load, class Emit>
__device__ __forceinline__ uint32_t block_chain(ChainLds<Cap>& L, uint32_t ns, Load load, Emit emit, double* area)
{
    uint32_t N = 1;
    while (N < ns) N <<= 1;
    if (N <= (uint32_t)kChainBlock) {
        // one point per thread: bitonic stages over distances below 64
        // are shuffles inside a wave, the others go through LDS
        const uint32_t t = threadIdx.x;
        double u = INFINITY, v = INFINITY;
        uint32_t id = 0xFFFFFFFFu;
        if (t < ns) load(t, &u, &v, &id);
        for (uint32_t size = 2; size <= N; size <<= 1) {
            for (uint32_t j = size >> 1; j > 0; j >>= 1) {
                double ou, ov;
                uint32_t oi;
                if (j >= (uint32_t)kWave) {
                    L.su[t] = u;
                    L.sv[t] = v;
                    L.si[t] = id;
                    __syncthreads();
                    ou = L.su[t ^ j];
                    ov = L.sv[t ^ j];
                    oi = L.si[t ^ j];
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
        L.su[t] = u;
        L.sv[t] = v;
        L.si[t] = id;
        __syncthreads();
    } else {
        for (uint32_t t = threadIdx.x; t < N; t += kChainBlock) {
            if (t < ns) {
                load(t, &L.su[t], &L.sv[t], &L.si[t]);
            } else {
                L.su[t] = INFINITY;
                L.sv[t] = INFINITY;
                L.si[t] = 0xFFFFFFFFu;
            }
        }
        __syncthreads();
        for (uint32_t size = 2; size <= N; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t t = threadIdx.x; t < N / 2; t += kChainBlock) {
                    const uint32_t a = 2 * t - (t & (stride - 1)), b = a + stride;
                    const bool upw = (a & size) == 0;
                    if (p2_less(L.su[b], L.sv[b], L.si[b], L.su[a], L.sv[a], L.si[a]) == upw) swap3(L.su, L.sv, L.si, a, b);
                }
                __syncthreads();
            }
        }
    }
    // lower chain on wave 0, upper chain on wave 1
    if (threadIdx.x < kWave) chain_level1(L.su, L.sv, ns, true, L.tmp_lo, L.seq_lo, L.offs_lo);
    else if (threadIdx.x < 2 * kWave) chain_level1(L.su, L.sv, ns, false, L.tmp_up, L.seq_up, L.offs_up);
    __syncthreads();
    if (threadIdx.x < kChainL2) L.len2_lo[threadIdx.x] = chain_level2(L.su, L.sv, L.seq_lo, L.offs_lo, threadIdx.x);
    else if (threadIdx.x >= kWave && threadIdx.x < kWave + kChainL2)
        L.len2_up[threadIdx.x - kWave] = chain_level2(L.su, L.sv, L.seq_up, L.offs_up, threadIdx.x - kWave);
    __syncthreads();
    // level 3: the plain chain over the level-2 results, made contiguous
    // (the level-1 scratch is free again)
    const uint32_t l2lo = chain_gather2(L.seq_lo, L.offs_lo, L.len2_lo, L.tmp_lo);
    const uint32_t l2up = chain_gather2(L.seq_up, L.offs_up, L.len2_up, L.tmp_up);
    __syncthreads();
    if (threadIdx.x == 0) L.hlo = chain_run<false>(L.su, L.sv, L.tmp_lo, l2lo, L.st_lo);
    if (threadIdx.x == kWave) L.hup = chain_run<false>(L.su, L.sv, L.tmp_up, l2up, L.st_up);
    __syncthreads();
    // hull = lower chain, then the upper chain without its end points
    // (they are the lower chain's last and first points); the
    // vertices and the shoelace terms are taken in parallel
    {
        const uint32_t hl = L.hlo, hu = L.hup;
        const uint32_t h = hl + (hu >= 2 ? hu - 2 : 0u);
        auto vertex = [&](uint32_t q) -> uint32_t { return q < hl ? L.st_lo[q] : L.st_up[q - hl + 1]; };
        double term = 0.0;
        for (uint32_t q = threadIdx.x; q < h; q += kChainBlock) {
            const uint32_t p0 = vertex(q), p1 = vertex(q + 1 == h ? 0u : q + 1);
            term += L.su[p0] * L.sv[p1] - L.su[p1] * L.sv[p0];
            emit(q, p0);   // vertex q is sorted point p0
        }
#pragma unroll
        for (int dd = kWave / 2; dd >= 1; dd >>= 1) term += __shfl_xor(term, dd, kWave);
        if ((threadIdx.x & (kWave - 1)) == 0) L.red[threadIdx.x / kWave] = term;
        __syncthreads();
        if (threadIdx.x == 0) {
            double tot = 0.0;
            for (int w2 = 0; w2 < kChainBlock / kWave; ++w2) tot += L.red[w2];
            *area = h >= 3 ? 0.5 * tot : 0.0;
        }
        return h;
    }
}

}  // namespace dev
}  // namespace vm

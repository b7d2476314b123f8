// vm_step.hip -- steppable point classification (Sec. III-C, Eq. (3)-(4))
// and the clustering of steppable points with Alg. 1's distance and
// normal-angle gates.
//
//   k_step_means:    the Eq. (1) mean of every occupied voxel, by rank
//                    (one hash lookup each);
//   k_step_classify: a thread per voxel gathers the means of the occupied
//                    voxels within `radius` cells (occupancy bits and ranks,
//                    no hash), in ascending key order: their mean, then their
//                    scatter matrix (fp64), its cyclic Jacobi eigenvectors,
//                    the unit normal of the smallest eigenvalue oriented to
//                    +z, and the Eq. (4) test;
//   k_step_hook:     union-find over the steppable voxels: each unites with
//                    its 13 neighbours of smaller key that pass both gates
//                    (the gates are symmetric, so every edge is seen once);
//                    hooks put the larger root under the smaller, so each
//                    root is its component's smallest key, Alg. 1's fixed
//                    point from L_i = i;
//   k_step_flatten:  every voxel takes its root; steppable roots count their
//                    voxels (the grouping then keeps components of at least
//                    min_cluster voxels; voxels that are not steppable count
//                    nothing and join no cluster).
// The fp64 arithmetic is written operation by operation (no contraction), so
// the normals and decisions are the same bits as the definition computes.
#include "vm_common.h"
#include "vm_dev.h"

#include <math.h>

namespace vm {
namespace {

__device__ __forceinline__ uint32_t ld_rel(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// path-halving and flattening stores are device-scope (written through to
// memory), as in the unconditional labelling's union-find
__device__ __forceinline__ void st_rel(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// root of x with path halving (parents only ever move to ancestors)
__device__ __forceinline__ uint32_t find_root(uint32_t* parent, uint32_t x)
{
    uint32_t p = ld_rel(&parent[x]);
    while (p != x) {
        const uint32_t g = ld_rel(&parent[p]);
        if (g == p) return p;
        st_rel(&parent[x], g);
        x = g;
        p = ld_rel(&parent[x]);
    }
    return x;
}

// union of the sets of a and b: the larger root is hooked under the smaller
__device__ __forceinline__ void unite(uint32_t* parent, uint32_t a, uint32_t b)
{
    a = find_root(parent, a);
    b = find_root(parent, b);
    while (a != b) {
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicCAS(&parent[a], a, b);
        if (old == a) return;
        a = find_root(parent, old);
        b = find_root(parent, b);
    }
}

__device__ __forceinline__ bool occupied(const uint32_t* __restrict__ bits, uint32_t key)
{
    return (bits[key >> 5] >> (key & 31)) & 1u;
}

__device__ __forceinline__ uint32_t rank_of_key(const uint32_t* __restrict__ bits, const uint32_t* __restrict__ wrank,
                                                uint32_t key)
{
    return wrank[key >> 5] + __popc(bits[key >> 5] & ((1u << (key & 31)) - 1u));
}

__global__ void __launch_bounds__(kBlock) k_step_means(Geom g, Hash h, const DevCounters* __restrict__ ctr,
                                                       const uint32_t* __restrict__ occ_key, float4* __restrict__ mean)
{
    const uint32_t V = ctr->n_occ;
    const uint32_t nx = (uint32_t)g.dims[0], ny = (uint32_t)g.dims[1];
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t k = occ_key[r];
        const uint32_t s = hash_find(h, k);
        float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
        if (s != kEmpty) {
            const Slot sl = h.slot[s];
            m.x = voxel_mean_axis(k % nx, sl.sum[0], sl.cnt, g.voxel_size, g.origin[0]);
            m.y = voxel_mean_axis((k / nx) % ny, sl.sum[1], sl.cnt, g.voxel_size, g.origin[1]);
            m.z = voxel_mean_axis(k / (nx * ny), sl.sum[2], sl.cnt, g.voxel_size, g.origin[2]);
        }
        mean[r] = m;
    }
}

// the cyclic Jacobi method on a symmetric 3x3 matrix: rotations in the planes
// (0,1), (0,2), (1,2) in turn, sweeps until the off-diagonal part is
// negligible against the diagonal (at most 16); V receives the eigenvectors
__device__ __forceinline__ void jacobi3(double A[3][3], double V[3][3])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 16; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-30 * dia) break;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int p = r < 2 ? 0 : 1, q = r == 0 ? 1 : 2;
            const double apq = A[p][q];
            if (apq == 0.0) continue;
            const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double s = t * c;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double akp = A[k][p], akq = A[k][q];
                A[k][p] = c * akp - s * akq;
                A[k][q] = s * akp + c * akq;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double apk = A[p][k], aqk = A[q][k];
                A[p][k] = c * apk - s * aqk;
                A[q][k] = s * apk + c * aqk;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double vkp = V[k][p], vkq = V[k][q];
                V[k][p] = c * vkp - s * vkq;
                V[k][q] = s * vkp + c * vkq;
            }
        }
    }
}

struct StepArgs {
    const uint32_t* bits;
    const uint32_t* wrank;
    const uint32_t* occ_key;
    const float4* mean;
    int32_t nx, ny, nz;
    int32_t radius;
    uint32_t n_th;
    double cos_th;
    double d_th;
    float4* normal;       // [cap] xyz + pad
    uint8_t* step;        // [cap]
};

// Eq. (3)-(4) for every occupied voxel
__global__ void __launch_bounds__(kBlock) k_step_classify(StepArgs a, const DevCounters* __restrict__ ctr)
{
    const uint32_t V = ctr->n_occ;
    const int R = a.radius;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t key = a.occ_key[r];
        const int x = (int)(key % (uint32_t)a.nx), y = (int)((key / (uint32_t)a.nx) % (uint32_t)a.ny),
                  z = (int)(key / ((uint32_t)a.nx * (uint32_t)a.ny));
        // pass 1: the neighbours' mean (in ascending key order)
        double sx = 0.0, sy = 0.0, sz = 0.0;
        uint32_t cnt = 0;
        for (int dz = -R; dz <= R; ++dz)
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx) {
                    const int xx = x + dx, yy = y + dy, zz = z + dz;
                    if (xx < 0 || yy < 0 || zz < 0 || xx >= a.nx || yy >= a.ny || zz >= a.nz) continue;
                    const uint32_t k2 = (uint32_t)xx + (uint32_t)a.nx * ((uint32_t)yy + (uint32_t)a.ny * (uint32_t)zz);
                    if (!occupied(a.bits, k2)) continue;
                    const float4 p = a.mean[rank_of_key(a.bits, a.wrank, k2)];
                    sx += (double)p.x;
                    sy += (double)p.y;
                    sz += (double)p.z;
                    ++cnt;
                }
        const double mx = sx / (double)cnt, my = sy / (double)cnt, mz = sz / (double)cnt;
        // pass 2: their scatter matrix about that mean (same order)
        double A[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        for (int dz = -R; dz <= R; ++dz)
            for (int dy = -R; dy <= R; ++dy)
                for (int dx = -R; dx <= R; ++dx) {
                    const int xx = x + dx, yy = y + dy, zz = z + dz;
                    if (xx < 0 || yy < 0 || zz < 0 || xx >= a.nx || yy >= a.ny || zz >= a.nz) continue;
                    const uint32_t k2 = (uint32_t)xx + (uint32_t)a.nx * ((uint32_t)yy + (uint32_t)a.ny * (uint32_t)zz);
                    if (!occupied(a.bits, k2)) continue;
                    const float4 p = a.mean[rank_of_key(a.bits, a.wrank, k2)];
                    const double ex = (double)p.x - mx, ey = (double)p.y - my, ez = (double)p.z - mz;
                    A[0][0] += ex * ex;
                    A[0][1] += ex * ey;
                    A[0][2] += ex * ez;
                    A[1][1] += ey * ey;
                    A[1][2] += ey * ez;
                    A[2][2] += ez * ez;
                }
        A[1][0] = A[0][1];
        A[2][0] = A[0][2];
        A[2][1] = A[1][2];
        double Vv[3][3];
        jacobi3(A, Vv);
        int m = 0;
        if (A[1][1] < A[m][m]) m = 1;
        if (A[2][2] < A[m][m]) m = 2;
        double nx = m == 0 ? Vv[0][0] : (m == 1 ? Vv[0][1] : Vv[0][2]);
        double ny = m == 0 ? Vv[1][0] : (m == 1 ? Vv[1][1] : Vv[1][2]);
        double nz = m == 0 ? Vv[2][0] : (m == 1 ? Vv[2][1] : Vv[2][2]);
        const double len = sqrt(nx * nx + ny * ny + nz * nz);
        nx /= len;
        ny /= len;
        nz /= len;
        // the orientation as one flag and a product with -1 or +1 (exact; +0
        // becomes -0 as under negation): no branches, whose nested short
        // circuits the device compiler has been seen to resolve for nz >= 0
        // without the inner tests
        const bool flip = (nz < 0.0) | ((nz == 0.0) & ((ny < 0.0) | ((ny == 0.0) & (nx < 0.0))));
        const double sg = flip ? -1.0 : 1.0;
        nx *= sg;
        ny *= sg;
        nz *= sg;
        a.normal[r] = make_float4((float)nx, (float)ny, (float)nz, 0.f);
        a.step[r] = (cnt >= a.n_th && nz >= a.cos_th) ? 1 : 0;
    }
}

// union-find over the steppable voxels with Alg. 1's gates (parent = rank)
__global__ void __launch_bounds__(kBlock) k_step_hook(StepArgs a, const DevCounters* __restrict__ ctr,
                                                      uint32_t* parent)
{
    const uint32_t V = ctr->n_occ;
    const double d2_th = a.d_th * a.d_th;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        if (!a.step[r]) continue;
        const uint32_t key = a.occ_key[r];
        const int x = (int)(key % (uint32_t)a.nx), y = (int)((key / (uint32_t)a.nx) % (uint32_t)a.ny),
                  z = (int)(key / ((uint32_t)a.nx * (uint32_t)a.ny));
        const float4 pi = a.mean[r], ni = a.normal[r];
        // the 13 neighbours with smaller keys: dz = -1 (any dy, dx), dz = 0 and
        // dy = -1 (any dx), and dz = dy = 0, dx = -1
        for (int q = 0; q < 13; ++q) {
            const int dz = q < 9 ? -1 : 0;
            const int dy = q < 9 ? q / 3 - 1 : (q < 12 ? -1 : 0);
            const int dx = q < 12 ? q % 3 - 1 : -1;
            const int xx = x + dx, yy = y + dy, zz = z + dz;
            if (xx < 0 || yy < 0 || zz < 0 || xx >= a.nx || yy >= a.ny || zz >= a.nz) continue;
            const uint32_t k2 = (uint32_t)xx + (uint32_t)a.nx * ((uint32_t)yy + (uint32_t)a.ny * (uint32_t)zz);
            if (!occupied(a.bits, k2)) continue;
            const uint32_t r2 = rank_of_key(a.bits, a.wrank, k2);
            if (!a.step[r2]) continue;
            const float4 pj = a.mean[r2], nj = a.normal[r2];
            const double ddx = (double)pi.x - (double)pj.x, ddy = (double)pi.y - (double)pj.y,
                         ddz = (double)pi.z - (double)pj.z;
            if (!(ddx * ddx + ddy * ddy + ddz * ddz < d2_th)) continue;
            const double dot = (double)ni.x * (double)nj.x + (double)ni.y * (double)nj.y + (double)ni.z * (double)nj.z;
            if (!(dot > a.cos_th)) continue;
            unite(parent, r, r2);
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_step_init(const DevCounters* __restrict__ ctr, uint32_t* __restrict__ parent)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) parent[r] = r;
}

// every voxel takes its root (a read-only walk, then its own store); steppable
// voxels add one to their root's count, one atomic per distinct root per wave
__global__ void __launch_bounds__(kBlock) k_step_flatten(const DevCounters* __restrict__ ctr,
                                                         const uint8_t* __restrict__ step, uint32_t* parent,
                                                         uint32_t* csize)
{
    const uint32_t V = ctr->n_occ;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t b0 = blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1)); b0 < V; b0 += stride) {
        const uint32_t r = b0 + (uint32_t)lane;
        uint32_t x = r, cs = 0;
        if (r < V) {
            uint32_t p = ld_rel(&parent[r]);
            while (p != x) {
                x = p;
                p = ld_rel(&parent[x]);
            }
            st_rel(&parent[r], x);
            cs = step[r] ? 1u : 0u;
        }
        uint64_t pending = __ballot(cs != 0);
        while (pending) {
            const int leader = __ffsll((long long)pending) - 1;
            const uint32_t root = __shfl(x, leader, kWave);
            const bool same = cs != 0 && x == root;
            uint32_t v = same ? cs : 0u;
#pragma unroll
            for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
            if (lane == leader) atomicAdd(&csize[root], v);
            pending &= ~__ballot(same);
        }
    }
}

// labels in ascending key order: the root's key, kEmpty where not steppable
__global__ void __launch_bounds__(kBlock) k_step_labels(const DevCounters* __restrict__ ctr,
                                                        const uint32_t* __restrict__ parent,
                                                        const uint8_t* __restrict__ step,
                                                        const uint32_t* __restrict__ occ_key, uint32_t* __restrict__ labels)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x)
        labels[r] = step[r] ? occ_key[parent[r]] : kEmpty;
}

// the classification as three floats and one byte per voxel (caller's buffers)
__global__ void __launch_bounds__(kBlock) k_step_export(const DevCounters* __restrict__ ctr,
                                                        const float4* __restrict__ normal,
                                                        const uint8_t* __restrict__ step, float* __restrict__ n_out,
                                                        uint8_t* __restrict__ s_out)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        if (n_out) {
            const float4 n = normal[r];
            n_out[3 * (size_t)r + 0] = n.x;
            n_out[3 * (size_t)r + 1] = n.y;
            n_out[3 * (size_t)r + 2] = n.z;
        }
        if (s_out) s_out[r] = step[r];
    }
}

}  // namespace

hipError_t launch_steppable(const Geom& g, const Hash& h, const uint32_t* bits, SegBuffers& b, uint32_t cap,
                            const StepBuffers& sb, uint32_t radius, uint32_t n_th, double cos_th, double d_th,
                            float* d_normal, uint8_t* d_steppable, DevCounters* ctr, hipStream_t s)
{
    const int grid = grid_for(cap);
    k_step_means<<<grid, kBlock, 0, s>>>(g, h, ctr, b.occ_key, sb.mean);
    StepArgs a;
    a.bits = bits;
    a.wrank = b.wrank;
    a.occ_key = b.occ_key;
    a.mean = sb.mean;
    a.nx = g.dims[0];
    a.ny = g.dims[1];
    a.nz = g.dims[2];
    a.radius = (int32_t)radius;
    a.n_th = n_th;
    a.cos_th = cos_th;
    a.d_th = d_th;
    a.normal = sb.normal;
    a.step = sb.step;
    k_step_classify<<<grid, kBlock, 0, s>>>(a, ctr);
    k_step_init<<<grid, kBlock, 0, s>>>(ctr, b.parent);
    k_step_hook<<<grid, kBlock, 0, s>>>(a, ctr, b.parent);
    k_step_flatten<<<grid, kBlock, 0, s>>>(ctr, sb.step, b.parent, b.csize);
    if (d_normal || d_steppable) k_step_export<<<grid, kBlock, 0, s>>>(ctr, sb.normal, sb.step, d_normal, d_steppable);
    return hipGetLastError();
}

hipError_t launch_step_labels(const SegBuffers& b, const StepBuffers& sb, uint32_t cap, DevCounters* ctr,
                              uint32_t* d_labels, hipStream_t s)
{
    k_step_labels<<<grid_for(cap), kBlock, 0, s>>>(ctr, b.parent, sb.step, b.occ_key, d_labels);
    return hipGetLastError();
}

}  // namespace vm

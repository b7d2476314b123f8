// vm_ccl.hip -- connected-component labelling of the occupied voxels and the
// grouping of voxels into clusters (Sec. III-C, "Clustering", Alg. 1).
//
// Alg. 1 propagates the smaller label over every adjacency until nothing
// changes; from L_i = i its fixed point is the smallest index of each
// connected component.  That fixed point is reached here with a lock-free
// union-find over the occupied ranks (rank order == key order, so the
// smallest rank of a component is its smallest key):
//   * init:    every voxel points at the start of its run along x (runs of
//              consecutive occupied cells share a component trivially);
//   * merge:   runs in the four neighbouring rows with smaller keys
//              (dz = -1, any dy; dz = 0, dy = -1) are hooked together; a
//              voxel only hooks where an overlap between its run and a run of
//              the other row begins, plus the diagonal end cells, so each
//              pair of touching runs is hooked about once;
//   * flatten: every voxel takes its root.
// Hooks always put the larger root under the smaller one with a CAS on the
// root, so every root ends as the minimum of its tree and the labels are
// exact whatever the interleaving.  Path halving keeps trees shallow.  The
// 26-neighbourhood never needs the hash: occupancy and ranks come from the
// 1-bit-per-cell index.
#include "vm_common.h"

namespace vm {
namespace {

// Parent pointers are read and path-halved through the ordinary caches.  A
// stale value is still an ancestor (parents only ever move to smaller ranks
// of the same component), so finds stay correct; only the hook itself needs a
// device-coherent CAS.  Relaxed atomics keep the compiler from caching or
// tearing the accesses.
__device__ __forceinline__ uint32_t ld_parent(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ void st_parent(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ bool occ(const uint32_t* __restrict__ bits, uint32_t key)
{
    return (bits[key >> 5] >> (key & 31)) & 1u;
}

__device__ __forceinline__ uint32_t rank_of(const uint32_t* __restrict__ bits, const uint32_t* __restrict__ wrank,
                                            uint32_t key)
{
    const uint32_t b = key & 31;
    return wrank[key >> 5] + __popc(bits[key >> 5] & ((1u << b) - 1u));
}

// Root of x with path halving (each visited node is re-pointed at its
// grandparent; concurrent writes only ever store an ancestor).
__device__ __forceinline__ uint32_t uf_find(uint32_t* parent, uint32_t x)
{
    uint32_t p = ld_parent(&parent[x]);
    while (p != x) {
        const uint32_t g = ld_parent(&parent[p]);
        if (g == p) return p;
        st_parent(&parent[x], g);
        x = g;
        p = ld_parent(&parent[x]);
    }
    return x;
}

__device__ __forceinline__ void uf_unite(uint32_t* parent, uint32_t a, uint32_t b)
{
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    while (a != b) {
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        const uint32_t old = atomicCAS(&parent[a], a, b);   // hook root a under b
        if (old == a) return;
        a = uf_find(parent, old);
        b = uf_find(parent, b);
    }
}

struct Dims {
    uint32_t nx, ny, nz, nxy;
};

__global__ void __launch_bounds__(kBlock) k_ccl_init(const uint32_t* __restrict__ bits,
                                                     const uint32_t* __restrict__ occ_key,
                                                     const DevCounters* __restrict__ ctr, Dims d,
                                                     uint32_t* __restrict__ parent, uint32_t* __restrict__ linked)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t key = occ_key[r];
        const uint32_t x = key % d.nx;
        const uint32_t rowstart = key - x;
        // smallest key of the run of occupied cells ending at `key`
        const uint32_t w = key >> 5, b = key & 31;
        uint32_t start;
        const uint32_t zeros = (~bits[w]) & ((1u << b) - 1u);
        if (zeros) {
            start = (w << 5) + 32u - __clz(zeros);
        } else {
            start = w << 5;
            uint32_t ww = w;
            while (start > rowstart && ww > 0) {
                --ww;
                const uint32_t z = ~bits[ww];
                if (z) { start = (ww << 5) + 32u - __clz(z); break; }
                start = ww << 5;
            }
        }
        if (start < rowstart) start = rowstart;
        parent[r] = r - (key - start);
        // part of a run of two or more voxels along x?
        const bool next = (x + 1 < d.nx) && occ(bits, key + 1);
        linked[r] = (start < key || next) ? 1u : 0u;
    }
}

// a voxel joined to another across rows: both ends are marked (stores of 1
// only, so concurrent marks cannot conflict)
__device__ __forceinline__ void link(uint32_t* parent, uint32_t* linked, uint32_t a, uint32_t b)
{
    linked[a] = 1u;
    linked[b] = 1u;
    uf_unite(parent, a, b);
}

__global__ void __launch_bounds__(kBlock) k_ccl_merge(const uint32_t* __restrict__ bits,
                                                      const uint32_t* __restrict__ wrank,
                                                      const uint32_t* __restrict__ occ_key,
                                                      const DevCounters* __restrict__ ctr, Dims d,
                                                      uint32_t* parent, uint32_t* linked)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t key = occ_key[r];
        const uint32_t x = key % d.nx;
        const uint32_t y = (key / d.nx) % d.ny;
        const uint32_t z = key / d.nxy;
        const bool run_start = (x == 0) || !occ(bits, key - 1);
        const bool run_end = (x + 1 == d.nx) || !occ(bits, key + 1);
        // the four rows with smaller keys: (dy, dz) = (-1,0), (-1,-1), (0,-1), (+1,-1)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int dy = (j == 0) ? -1 : (j - 2);
            const int dz = (j == 0) ? 0 : -1;
            if ((dz < 0 && z == 0) || (dy < 0 && y == 0) || (dy > 0 && y + 1 == d.ny)) continue;
            const uint32_t nk = (uint32_t)((int64_t)key + (int64_t)dy * d.nx + (int64_t)dz * d.nxy);
            if (occ(bits, nk) && (run_start || !occ(bits, nk - 1)))
                link(parent, linked, r, rank_of(bits, wrank, nk));
            if (run_start && x > 0 && occ(bits, nk - 1))
                link(parent, linked, r, rank_of(bits, wrank, nk - 1));
            if (run_end && x + 1 < d.nx && occ(bits, nk + 1))
                link(parent, linked, r, rank_of(bits, wrank, nk + 1));
        }
    }
}

// After the merge every tree is final.  Each voxel walks to its root without
// writing anything on the way (a path-halving store here could overwrite the
// root another thread has just stored for that node) and stores only its own
// entry; every value a walk can read is an ancestor, so walks stay correct.
__global__ void __launch_bounds__(kBlock) k_ccl_flatten(const DevCounters* __restrict__ ctr, uint32_t* parent)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        uint32_t x = r, p = ld_parent(&parent[r]);
        while (p != x) {
            x = p;
            p = ld_parent(&parent[x]);
        }
        st_parent(&parent[r], x);
    }
}

// Component sizes at the roots.  A voxel never linked to another is a
// component of its own: size 1, a plain store.  For the rest, consecutive
// ranks mostly share a root: a wave first sums each run of equal roots, then
// the block merges its runs in an LDS table and adds one count per distinct
// root (a large component's root would otherwise take an atomic from every
// wave that holds part of it).
constexpr int kSizeItems = 8;
constexpr int kSizeSpan = kBlock * kSizeItems;   // ranks per block pass
constexpr int kSizeTab = kSizeSpan;              // one slot per possible root
static_assert(kSizeTab == 1 << 11, "the table hash below indexes 2^11 slots");

__global__ void __launch_bounds__(kBlock) k_ccl_sizes(const DevCounters* __restrict__ ctr,
                                                      const uint32_t* __restrict__ parent,
                                                      const uint32_t* __restrict__ linked, uint32_t* csize)
{
    __shared__ uint32_t tkey[kSizeTab];
    __shared__ uint32_t tcnt[kSizeTab];
    const uint32_t V = ctr->n_occ;
    const int lane = threadIdx.x & (kWave - 1);
    for (uint32_t base = blockIdx.x * kSizeSpan; base < V; base += gridDim.x * kSizeSpan) {
        for (int i = threadIdx.x; i < kSizeTab; i += kBlock) {
            tkey[i] = kEmpty;
            tcnt[i] = 0;
        }
        __syncthreads();
        for (int it = 0; it < kSizeItems; ++it) {
            const uint32_t r = base + it * kBlock + threadIdx.x;
            const bool in = r < V;
            const bool alone = in && linked[r] == 0u;
            if (alone) csize[r] = 1u;
            const bool valid = in && !alone;
            const uint32_t root = valid ? parent[r] : 0xFFFFFFFFu;
            const uint32_t prev = __shfl_up(root, 1, kWave);
            const uint64_t vmask = __ballot(valid);
            const bool prev_valid = lane > 0 && ((vmask >> (lane - 1)) & 1ull);
            const bool head = valid && (!prev_valid || prev != root);
            // a run ends before the next head or the next lane that is not valid
            const uint64_t stops = __ballot(head) | ~vmask;
            if (head) {
                const uint64_t after = (lane == 63) ? 0ull : (stops & (~0ull << (lane + 1)));
                const uint32_t len = (after ? (uint32_t)(__ffsll((long long)after) - 1) : 64u) - (uint32_t)lane;
                uint32_t h = (root * 2654435769u) >> (32 - 11);   // kSizeTab = 2^11 slots
                for (;;) {
                    const uint32_t old = atomicCAS(&tkey[h], kEmpty, root);
                    if (old == kEmpty || old == root) {
                        atomicAdd(&tcnt[h], len);
                        break;
                    }
                    h = (h + 1) & (kSizeTab - 1);
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < kSizeTab; i += kBlock)
            if (tkey[i] != kEmpty) atomicAdd(&csize[tkey[i]], tcnt[i]);
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_zero(uint32_t* p, const DevCounters* __restrict__ ctr)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) p[r] = 0;
}

// ---- grouping -------------------------------------------------------------------
// flags for the two scans: kept root -> 1 (cluster id), and its size (offset)
__global__ void __launch_bounds__(kBlock) k_group_flags(const DevCounters* __restrict__ ctr,
                                                        const uint32_t* __restrict__ parent,
                                                        const uint32_t* __restrict__ csize, uint32_t min_cluster,
                                                        uint32_t* __restrict__ is_root, uint32_t* __restrict__ root_size,
                                                        uint32_t* __restrict__ keep)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t root = parent[r];
        const uint32_t sz = csize[root];
        const bool kept = sz >= min_cluster;
        const bool rt = kept && root == r;
        is_root[r] = rt ? 1u : 0u;
        root_size[r] = rt ? sz : 0u;
        keep[r] = kept ? 1u : 0u;
    }
}

__global__ void __launch_bounds__(kBlock) k_group_clusters(DevCounters* __restrict__ ctr,
                                                           const uint32_t* __restrict__ parent,
                                                           const uint32_t* __restrict__ csize, uint32_t min_cluster,
                                                           const uint32_t* __restrict__ occ_key,
                                                           const uint32_t* __restrict__ cid_scan,
                                                           const uint32_t* __restrict__ off_scan,
                                                           uint32_t* __restrict__ cl_off, uint32_t* __restrict__ cl_tag)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        if (parent[r] == r && csize[r] >= min_cluster) {
            const uint32_t c = cid_scan[r];
            cl_off[c] = off_scan[r];
            cl_tag[c] = occ_key[r];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t K = ctr->meta[0];
        cl_off[K] = ctr->meta[1];
        ctr->kmax = K ? K - 1 : 0;
    }
}

// (cluster id, rank) pairs of the kept voxels, in rank order
__global__ void __launch_bounds__(kBlock) k_group_pairs(const DevCounters* __restrict__ ctr,
                                                        const uint32_t* __restrict__ parent,
                                                        const uint32_t* __restrict__ csize, uint32_t min_cluster,
                                                        const uint32_t* __restrict__ cid_scan,
                                                        const uint32_t* __restrict__ pos_scan,
                                                        uint32_t* __restrict__ out_cid, uint32_t* __restrict__ out_rank)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x) {
        const uint32_t root = parent[r];
        if (csize[root] >= min_cluster) {
            const uint32_t p = pos_scan[r];
            out_cid[p] = cid_scan[root];
            out_rank[p] = r;
        }
    }
}

// CSR points: key and Eq. (1) mean of each kept voxel, cluster-major
__global__ void __launch_bounds__(kBlock) k_group_gather(Geom g, Hash h, const DevCounters* __restrict__ ctr,
                                                         const uint32_t* __restrict__ sorted_rank,
                                                         const uint32_t* __restrict__ occ_key,
                                                         uint32_t* __restrict__ cl_key, float* __restrict__ cl_x,
                                                         float* __restrict__ cl_y, float* __restrict__ cl_z)
{
    const uint32_t n = ctr->meta[1];
    const uint32_t nx = (uint32_t)g.dims[0], ny = (uint32_t)g.dims[1];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t k = occ_key[sorted_rank[i]];
        const uint32_t s = hash_find(h, k);
        float mx = 0.0f, my = 0.0f, mz = 0.0f;
        if (s != kEmpty) {
            const Slot sl = h.slot[s];
            mx = voxel_mean_axis(k % nx, sl.sum[0], sl.cnt, g.voxel_size, g.origin[0]);
            my = voxel_mean_axis((k / nx) % ny, sl.sum[1], sl.cnt, g.voxel_size, g.origin[1]);
            mz = voxel_mean_axis(k / (nx * ny), sl.sum[2], sl.cnt, g.voxel_size, g.origin[2]);
        }
        cl_key[i] = k;
        cl_x[i] = mx;
        cl_y[i] = my;
        cl_z[i] = mz;
    }
}

__global__ void __launch_bounds__(kBlock) k_labels(const DevCounters* __restrict__ ctr,
                                                   const uint32_t* __restrict__ parent,
                                                   const uint32_t* __restrict__ occ_key, uint32_t* __restrict__ labels)
{
    const uint32_t V = ctr->n_occ;
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < V; r += gridDim.x * blockDim.x)
        labels[r] = occ_key[parent[r]];
}

Dims dims_of(const Geom& g)
{
    Dims d;
    d.nx = (uint32_t)g.dims[0];
    d.ny = (uint32_t)g.dims[1];
    d.nz = (uint32_t)g.dims[2];
    d.nxy = d.nx * d.ny;
    return d;
}

}  // namespace

hipError_t launch_ccl(const Geom& g, const uint32_t* bits, SegBuffers& b, uint32_t cap, DevCounters* ctr,
                      hipStream_t s)
{
    const Dims d = dims_of(g);
    const int grid = grid_for(cap);
    {
        StageScope t(VM_STAGE_CCL, s);
        k_ccl_init<<<grid, kBlock, 0, s>>>(bits, b.occ_key, ctr, d, b.parent, b.scan_a);
        k_ccl_merge<<<grid, kBlock, 0, s>>>(bits, b.wrank, b.occ_key, ctr, d, b.parent, b.scan_a);
        k_ccl_flatten<<<grid, kBlock, 0, s>>>(ctr, b.parent);
    }
    return hipGetLastError();
}

hipError_t launch_group(const Geom& g, const Hash& h, SegBuffers& b, uint32_t cap, uint32_t min_cluster,
                        uint32_t* d_labels, DevCounters* ctr, hipStream_t s)
{
    StageScope t(VM_STAGE_GROUP, s);
    const int grid = grid_for(cap);
    if (min_cluster < 1) min_cluster = 1;
    k_zero<<<grid, kBlock, 0, s>>>(b.csize, ctr);
    // scan_a: linked flags from the CCL
    k_ccl_sizes<<<grid_for(cap, kSizeSpan, 1024), kBlock, 0, s>>>(ctr, b.parent, b.scan_a, b.csize);
    uint32_t* is_root = b.scan_a;
    uint32_t* root_size = b.scan_b;
    uint32_t* keep = b.sort_k[1];
    k_group_flags<<<grid, kBlock, 0, s>>>(ctr, b.parent, b.csize, min_cluster, is_root, root_size, keep);
    hipError_t e;
    if ((e = scan_exclusive_dev(is_root, is_root, &ctr->n_occ, cap, &ctr->meta[0], b.blk, s)) != hipSuccess) return e;
    if ((e = scan_exclusive_dev(root_size, root_size, &ctr->n_occ, cap, &ctr->meta[1], b.blk, s)) != hipSuccess)
        return e;
    if ((e = scan_exclusive_dev(keep, keep, &ctr->n_occ, cap, nullptr, b.blk, s)) != hipSuccess) return e;
    k_group_clusters<<<grid, kBlock, 0, s>>>(ctr, b.parent, b.csize, min_cluster, b.occ_key, is_root, root_size,
                                             b.cl_off, b.cl_tag);
    k_group_pairs<<<grid, kBlock, 0, s>>>(ctr, b.parent, b.csize, min_cluster, is_root, keep, b.sort_k[0],
                                          b.sort_v[0]);
    // stable sort by cluster id keeps ascending keys inside each cluster
    const uint32_t kbound = cap / min_cluster + 1;
    const int bits_needed = 32 - __builtin_clz(kbound | 1u);
    int res = 0;
    if ((e = radix_sort_pairs_dev(b.sort_k, b.sort_v, &ctr->meta[1], cap, bits_needed, &ctr->kmax, b.hist, b.blk,
                                  &res, s)) != hipSuccess)
        return e;
    k_group_gather<<<grid, kBlock, 0, s>>>(g, h, ctr, b.sort_v[res], b.occ_key, b.cl_key, b.cl_x, b.cl_y, b.cl_z);
    if (d_labels) k_labels<<<grid, kBlock, 0, s>>>(ctr, b.parent, b.occ_key, d_labels);
    return hipGetLastError();
}

}  // namespace vm

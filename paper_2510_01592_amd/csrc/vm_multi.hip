// vm_multi.hip -- several cluster sets (e.g. one frame of each of several
// robots' maps) through one sequence of launches: the sets are merged into
// one cluster list, (a)-(c) of Sec. III-C "Multi-plane estimation" and the
// boundary polygons run once over the merged list with the tiled two-pass
// kernels (a floor of millions of points spreads over the whole chip), and
// each set's results are copied out exactly as that set alone would get
// them.  Every cluster keeps its own set's RNG frame word, so its planes do
// not depend on the company it is merged with.
#include "vm_common.h"

#include <algorithm>

namespace vm {
namespace {

constexpr uint32_t kMultiMax = 16;   // sets per call (the table travels as a kernel argument)
constexpr int kMBlock = 256;

struct MultiSet {
    const uint32_t* meta;
    const uint32_t* off;
    const float* x;
    const float* y;
    const float* z;
    const uint32_t* tag;
    uint32_t k_in;        // clusters this set may contribute: min(set, planes, hulls k_cap)
    uint32_t out_k_cap;   // min(planes, hulls k_cap)
    uint32_t n_cap;       // the set's point bound
    uint32_t frame;       // RNG counter word of its clusters
    float4* plane;
    int32_t* best;
    int32_t* nin;
    uint32_t* in_off;
    uint32_t* in_idx;
    int32_t* counts;
    float4* hyp;
    uint32_t* pstatus;
    uint32_t in_cap;
    uint32_t v_cap;
    uint32_t* v_off;
    uint32_t* v_idx;
    float* v_xyz;
    double* area;
    uint32_t* hstatus;
};

struct MultiTab {
    MultiSet s[kMultiMax];
    uint32_t n;
};

// The merged list and the merged pass's outputs, then the two-pass workspace.
struct MultiWork {
    uint32_t* meta;     // [2] merged K, N
    uint32_t* off;      // [k_cap + 1]
    uint32_t* tag;      // [k_cap]
    uint32_t* cframe;   // [k_cap]
    float* x;           // [n_cap]
    float* y;
    float* z;
    uint32_t* status;   // [2] the merged pass's own flags (each set's are set per set)
    float4* plane;      // [k_cap]
    int32_t* best;
    int32_t* nin;
    double* area;
    int32_t* counts;    // [k_cap][H]
    float4* hyp;        // [k_cap][H]
    uint32_t* in_off;   // [k_cap + 1] merged inlier offsets
    uint32_t* in_idx;   // [n_cap]
    uint32_t* v_off;    // [k_cap + 1] merged vertex offsets
    uint32_t* v_idx;    // [n_cap]
    float* v_xyz;       // [n_cap][3]
    uint32_t* sv;       // [k_cap + 1] vertex offsets after each set's own capacity rule
    uint32_t* mset;     // [kMultiMax][4]: K, N, first merged cluster, first merged point
    WorkLayout w;
    size_t bytes;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

MultiWork multi_layout(void* base, uint32_t k_cap, uint32_t n_cap, uint32_t H)
{
    MultiWork m{};
    char* p = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* r = p ? p + o : nullptr;
        o += align256(bytes);
        return r;
    };
    const size_t kc1 = (size_t)k_cap + 1, nc1 = (size_t)n_cap + 1;
    m.meta = (uint32_t*)take(64);
    m.off = (uint32_t*)take(kc1 * 4);
    m.tag = (uint32_t*)take(kc1 * 4);
    m.cframe = (uint32_t*)take(kc1 * 4);
    m.x = (float*)take(nc1 * 4);
    m.y = (float*)take(nc1 * 4);
    m.z = (float*)take(nc1 * 4);
    m.status = (uint32_t*)take(64);
    m.plane = (float4*)take(kc1 * 16);
    m.best = (int32_t*)take(kc1 * 4);
    m.nin = (int32_t*)take(kc1 * 4);
    m.area = (double*)take(kc1 * 8);
    m.counts = (int32_t*)take((size_t)k_cap * H * 4);
    m.hyp = (float4*)take((size_t)k_cap * H * 16);
    m.in_off = (uint32_t*)take(kc1 * 4);
    m.in_idx = (uint32_t*)take(nc1 * 4);
    m.v_off = (uint32_t*)take(kc1 * 4);
    m.v_idx = (uint32_t*)take(nc1 * 4);
    m.v_xyz = (float*)take(nc1 * 12);
    m.sv = (uint32_t*)take(kc1 * 4);
    m.mset = (uint32_t*)take(kMultiMax * 4 * 4);
    char* wbase = p ? p + o : nullptr;
    m.w = work_layout(wbase, k_cap, n_cap, H);
    m.bytes = o + m.w.bytes;
    return m;
}

// the set holding merged cluster (field 2) or point (field 3) k: the largest
// i whose first one is at or before k
__device__ __forceinline__ uint32_t set_of(const uint32_t* mset, uint32_t n, uint32_t k, int field)
{
    uint32_t i = 0;
    for (uint32_t q = 1; q < n; ++q)
        if (mset[4 * q + field] <= k) i = q;
    return i;
}

// validate every set, place it in the merged list (sets that no longer fit
// contribute nothing and are flagged), write the merged counts
__global__ void __launch_bounds__(kOneBlockThreads) k_multi_prep(MultiTab tab, MultiWork m, uint32_t k_cap,
                                                                 uint32_t n_cap)
{
    __shared__ int bad;
    __shared__ uint32_t sk[kMultiMax], sn[kMultiMax];
    for (uint32_t i = 0; i < tab.n; ++i) {
        const MultiSet& S = tab.s[i];
        const uint32_t K = validate_clusters(S.meta, S.off, S.k_in, S.n_cap, S.pstatus, &bad);
        if (threadIdx.x == 0) {
            sk[i] = K;
            sn[i] = K ? S.off[K] : 0u;
            if (S.meta[0] > S.out_k_cap) atomicOr(S.pstatus, (uint32_t)VM_FLAG_CLUSTERS_CAP);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        uint32_t kb = 0, pb = 0;
        for (uint32_t i = 0; i < tab.n; ++i) {
            uint32_t K = sk[i], N = sn[i];
            if (kb + K > k_cap || pb + N > n_cap) {   // no room left: the set is skipped
                atomicOr(tab.s[i].pstatus, (uint32_t)VM_FLAG_CLUSTERS_CAP);
                atomicOr(tab.s[i].hstatus, (uint32_t)VM_FLAG_CLUSTERS_CAP);
                K = 0;
                N = 0;
            }
            m.mset[4 * i + 0] = K;
            m.mset[4 * i + 1] = N;
            m.mset[4 * i + 2] = kb;
            m.mset[4 * i + 3] = pb;
            kb += K;
            pb += N;
        }
        m.meta[0] = kb;
        m.meta[1] = pb;
        m.off[kb] = pb;
        m.status[0] = 0;
        m.status[1] = 0;
    }
}

// the merged list: offsets, tags, frame words and points of every set
__global__ void __launch_bounds__(kMBlock) k_multi_gather(MultiTab tab, MultiWork m)
{
    const uint32_t Kt = m.meta[0], Nt = m.meta[1];
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < Kt; k += stride) {
        const uint32_t i = set_of(m.mset, tab.n, k, 2);
        const uint32_t kl = k - m.mset[4 * i + 2];
        m.off[k] = m.mset[4 * i + 3] + tab.s[i].off[kl];
        m.tag[k] = tab.s[i].tag[kl];
        m.cframe[k] = tab.s[i].frame;
    }
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < Nt; q += stride) {
        const uint32_t i = set_of(m.mset, tab.n, q, 3);
        const uint32_t ql = q - m.mset[4 * i + 3];
        m.x[q] = tab.s[i].x[ql];
        m.y[q] = tab.s[i].y[ql];
        m.z[q] = tab.s[i].z[ql];
    }
}

// A cluster gets a polygon in its set iff its inlier list ends within the
// set's own in_cap (the rule of vm_hulls on the set alone).
__device__ __forceinline__ bool fits_set(const MultiTab& tab, const MultiWork& m, uint32_t k, uint32_t* set)
{
    const uint32_t i = set_of(m.mset, tab.n, k, 2);
    *set = i;
    return m.in_off[k + 1] - m.in_off[m.mset[4 * i + 2]] <= tab.s[i].in_cap;
}

// Per-cluster results and each set's offsets (one workgroup): the vertex
// counts after each set's capacity rule are scanned into sv; the sets'
// totals and overflow flags.
__global__ void __launch_bounds__(kOneBlockThreads) k_multi_scan(MultiTab tab, MultiWork m)
{
    const uint32_t Kt = m.meta[0];
    uint32_t vt[1];
    one_block_scan<kOneBlockThreads, 4, 1>(
        Kt,
        [&](uint32_t k, uint32_t(&v)[1]) {
            uint32_t i;
            v[0] = fits_set(tab, m, k, &i) ? m.v_off[k + 1] - m.v_off[k] : 0u;
        },
        [&](uint32_t k, const uint32_t(&e)[1]) { m.sv[k] = e[0]; }, vt);
    if (threadIdx.x == 0) m.sv[Kt] = vt[0];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < tab.n; i += blockDim.x) {
        const MultiSet& S = tab.s[i];
        const uint32_t K = m.mset[4 * i], k0 = m.mset[4 * i + 2];
        const uint32_t ti = m.in_off[k0 + K] - m.in_off[k0], tv = m.sv[k0 + K] - m.sv[k0];
        S.in_off[K] = ti;
        S.v_off[K] = tv;
        if (ti > S.in_cap) {
            atomicOr(S.pstatus, (uint32_t)VM_FLAG_INLIERS_CAP);
            atomicOr(S.hstatus, (uint32_t)VM_FLAG_INLIERS_CAP);
        }
        if (tv > S.v_cap) atomicOr(S.hstatus, (uint32_t)VM_FLAG_HULL_CAP);
    }
}

// Each set's outputs, every array by output position (a huge inlier list is
// copied by many workgroups): per-cluster scalars and offsets, all
// hypotheses' counts and planes when asked for, inlier indices, vertices.
__global__ void __launch_bounds__(kMBlock) k_multi_copy(MultiTab tab, MultiWork m, uint32_t H, int with_all)
{
    const uint32_t Kt = m.meta[0];
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t t0 = blockIdx.x * blockDim.x + threadIdx.x;
    for (uint32_t k = t0; k < Kt; k += stride) {
        uint32_t i;
        const bool fits = fits_set(tab, m, k, &i);
        const MultiSet& S = tab.s[i];
        const uint32_t k0 = m.mset[4 * i + 2], kl = k - k0;
        S.plane[kl] = m.plane[k];
        S.best[kl] = m.best[k];
        S.nin[kl] = m.nin[k];
        S.in_off[kl] = m.in_off[k] - m.in_off[k0];
        S.v_off[kl] = m.sv[k] - m.sv[k0];
        S.area[kl] = fits ? m.area[k] : 0.0;
    }
    if (with_all) {
        const uint64_t kh = (uint64_t)Kt * H;
        for (uint64_t q = t0; q < kh; q += stride) {
            const uint32_t k = (uint32_t)(q / H), h = (uint32_t)(q % H);
            const uint32_t i = set_of(m.mset, tab.n, k, 2);
            const MultiSet& S = tab.s[i];
            const size_t dst = (size_t)(k - m.mset[4 * i + 2]) * H + h;
            if (S.counts) S.counts[dst] = m.counts[q];
            if (S.hyp) S.hyp[dst] = m.hyp[q];
        }
    }
    // inlier indices (cluster-local, the same in the merged list): set i's
    // entries are one contiguous range of the merged list
    const uint32_t ni = m.in_off[Kt];
    for (uint32_t g = t0; g < ni; g += stride) {
        uint32_t i = 0;
        for (uint32_t q = 1; q < tab.n; ++q)
            if (m.in_off[m.mset[4 * q + 2]] <= g) i = q;
        const uint32_t j = g - m.in_off[m.mset[4 * i + 2]];
        if (j < tab.s[i].in_cap) tab.s[i].in_idx[j] = m.in_idx[g];
    }
    // vertices of the clusters that keep their polygon
    const uint32_t nv = m.v_off[Kt];
    for (uint32_t g = t0; g < nv; g += stride) {
        uint32_t lo = 0, hi = Kt;   // the cluster: largest k with v_off[k] <= g
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (m.v_off[mid] <= g) lo = mid;
            else hi = mid;
        }
        uint32_t i;
        if (!fits_set(tab, m, lo, &i)) continue;
        const MultiSet& S = tab.s[i];
        const uint32_t pos = m.sv[lo] - m.sv[m.mset[4 * i + 2]] + (g - m.v_off[lo]);
        if (pos >= S.v_cap) continue;   // flagged by the scan
        S.v_idx[pos] = m.v_idx[g];
        S.v_xyz[3 * (size_t)pos + 0] = m.v_xyz[3 * (size_t)g + 0];
        S.v_xyz[3 * (size_t)pos + 1] = m.v_xyz[3 * (size_t)g + 1];
        S.v_xyz[3 * (size_t)pos + 2] = m.v_xyz[3 * (size_t)g + 2];
    }
}

}  // namespace

size_t multi_workspace_bytes(uint32_t k_cap, uint32_t n_cap, uint32_t H)
{
    return multi_layout(nullptr, k_cap, n_cap, H).bytes;
}

vm_status planes_hulls_multi(uint32_t n, const vm_clusters* sets, const uint32_t* frames, const vm_ransac_params& p,
                             const vm_planes* planes, const vm_hulls_out* hulls, uint32_t k_cap, uint32_t n_cap,
                             void* d_work, size_t work_bytes, hipStream_t s)
{
    if (n < 1 || n > kMultiMax || k_cap > kOneBlockMax) return VM_E_CAPACITY;
    const uint32_t H = p.n_hyp;
    const MultiWork m = multi_layout(d_work, k_cap, n_cap, H);
    if (m.bytes > work_bytes) return VM_E_CAPACITY;
    MultiTab tab{};
    tab.n = n;
    bool with_all = false;
    for (uint32_t i = 0; i < n; ++i) {
        MultiSet& S = tab.s[i];
        const vm_clusters& c = sets[i];
        S.meta = c.d_meta;
        S.off = c.d_off;
        S.x = c.d_x;
        S.y = c.d_y;
        S.z = c.d_z;
        S.tag = c.d_tag;
        S.out_k_cap = std::min(planes[i].k_cap, hulls[i].k_cap);
        S.k_in = std::min(c.k_cap, S.out_k_cap);
        S.n_cap = c.n_cap;
        S.frame = frames[i];
        S.plane = (float4*)planes[i].d_plane;
        S.best = planes[i].d_best_h;
        S.nin = planes[i].d_n_inliers;
        S.in_off = planes[i].d_in_off;
        S.in_idx = planes[i].d_in_idx;
        S.counts = planes[i].d_counts;
        S.hyp = (float4*)planes[i].d_hyp;
        S.pstatus = planes[i].d_status;
        S.in_cap = planes[i].in_cap;
        S.v_cap = hulls[i].v_cap;
        S.v_off = hulls[i].d_v_off;
        S.v_idx = hulls[i].d_v_idx;
        S.v_xyz = hulls[i].d_v_xyz;
        S.area = hulls[i].d_area;
        S.hstatus = hulls[i].d_status;
        with_all = with_all || S.counts || S.hyp;
    }
    {
        StageScope t(VM_STAGE_GROUP, s);
        k_multi_prep<<<1, kOneBlockThreads, 0, s>>>(tab, m, k_cap, n_cap);
        k_multi_gather<<<1024, kMBlock, 0, s>>>(tab, m);
        VM_HIP(hipGetLastError());
    }
    vm_clusters mc;
    mc.k_cap = k_cap;
    mc.n_cap = n_cap;
    mc.d_meta = m.meta;
    mc.d_off = m.off;
    mc.d_x = m.x;
    mc.d_y = m.y;
    mc.d_z = m.z;
    mc.d_key = nullptr;
    mc.d_tag = m.tag;
    // the merged outputs hold every inlier and vertex (each at most one per point)
    vm_planes mp{};
    mp.k_cap = k_cap;
    mp.in_cap = n_cap;
    mp.d_plane = (float*)m.plane;
    mp.d_best_h = m.best;
    mp.d_n_inliers = m.nin;
    mp.d_in_off = m.in_off;
    mp.d_in_idx = m.in_idx;
    mp.d_counts = with_all ? m.counts : nullptr;
    mp.d_hyp = with_all ? (float*)m.hyp : nullptr;
    mp.d_status = m.status;
    vm_hulls_out mh{};
    mh.k_cap = k_cap;
    mh.v_cap = n_cap;
    mh.d_v_off = m.v_off;
    mh.d_v_idx = m.v_idx;
    mh.d_v_xyz = m.v_xyz;
    mh.d_area = m.area;
    mh.d_status = m.status + 1;
    vm_status st = ransac_planes(mc, p, mp, m.w, s, m.cframe);
    if (st != VM_OK) return st;
    st = vm::hulls(mc, mp, mh, m.w, s);
    if (st != VM_OK) return st;
    StageScope t(VM_STAGE_HULL, s);
    k_multi_scan<<<1, kOneBlockThreads, 0, s>>>(tab, m);
    k_multi_copy<<<2048, kMBlock, 0, s>>>(tab, m, H, with_all ? 1 : 0);
    VM_HIP(hipGetLastError());
    return VM_OK;
}

}  // namespace vm

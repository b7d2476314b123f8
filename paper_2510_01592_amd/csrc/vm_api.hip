// vm_api.hip -- the C ABI (include/vm.h): argument checks, map ownership,
// per-stage timing, and the order in which the stages are enqueued.
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "vm_common.h"
#include "vm_tilescan.h"

using namespace vm;

struct vm_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

struct vm_map_s {
    int device = 0;
    Geom g{};
    Hash h{};
    uint32_t cap = 0;
    uint32_t* bits = nullptr;
    DevCounters* ctr = nullptr;
    SegBuffers b{};
    InsertScratch ins{};
    std::vector<void*> allocs;
    // workspace for the map's own RANSAC/hull pass (grown on demand)
    void* work = nullptr;
    size_t work_bytes = 0;
    uint32_t work_k = 0, work_hyp = 0;
    bool have_clusters = false;
    uint32_t last_min_cluster = 1;
    // classification buffers (allocated on the first steppable call)
    StepBuffers sb{};
    void* step_mem = nullptr;
    // ray and keep bitmaps of the clearing pass (allocated on the first call)
    uint32_t* clr_mem = nullptr;
    // per-sweep change flags of label propagation (device) and their host copy
    uint32_t* lp_flags = nullptr;
    uint32_t* lp_host = nullptr;
};

namespace vm {

// ---- stage timing ---------------------------------------------------------------
namespace {
struct TimingState {
    std::mutex mu;
    bool enabled = false;
    std::vector<hipEvent_t> pool;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
};
TimingState& timing()
{
    static TimingState* t = new TimingState();
    return *t;
}
hipEvent_t take_event(TimingState& t)
{
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

// Both events of a scope are taken from the pool before the first one is
// recorded, so nothing slow (an event creation) sits between a stage's
// kernels and its closing event.
StageScope::StageScope(int stage, hipStream_t s) : stage_(stage), s_(s), ev0_(nullptr), ev1_(nullptr)
{
    TimingState& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.enabled) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    hipEvent_t a = take_event(t), b = take_event(t);
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
        if (a) t.pool.push_back(a);
        if (b) t.pool.push_back(b);
        return;
    }
    ev0_ = a;
    ev1_ = b;
}

StageScope::~StageScope()
{
    if (!ev0_) return;
    hipEvent_t b = (hipEvent_t)ev1_;
    const bool ok = hipEventRecord(b, s_) == hipSuccess;
    TimingState& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    if (ok) t.recs.push_back({stage_, (hipEvent_t)ev0_, b});
    else {
        t.pool.push_back((hipEvent_t)ev0_);
        t.pool.push_back(b);
    }
}

}  // namespace vm

namespace {

bool bad_ptr(const void* p) { return p == nullptr; }

bool capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st == hipStreamCaptureStatusActive;
}

vm_status map_alloc(vm_map m, void** p, size_t bytes)
{
    if (hipMalloc(p, bytes ? bytes : 4) != hipSuccess) {
        (void)hipGetLastError();
        return VM_E_OOM;
    }
    m->allocs.push_back(*p);
    return VM_OK;
}

void map_free_all(vm_map m)
{
    for (void* p : m->allocs) (void)hipFree(p);
    m->allocs.clear();
    if (m->work) (void)hipFree(m->work);
    m->work = nullptr;
    if (m->step_mem) (void)hipFree(m->step_mem);
    m->step_mem = nullptr;
    if (m->clr_mem) (void)hipFree(m->clr_mem);
    m->clr_mem = nullptr;
    if (m->lp_flags) (void)hipFree(m->lp_flags);
    m->lp_flags = nullptr;
    if (m->lp_host) (void)hipHostFree(m->lp_host);
    m->lp_host = nullptr;
}

bool step_params_ok(const vm_step_params* sp)
{
    return sp && sp->radius >= 1 && sp->radius <= 2 && sp->cos_th >= -1.0 && sp->cos_th <= 1.0 && sp->d_th > 0.0 &&
           sp->d_th < 1e30;
}

Pose pose_of(const vm_pose* p)
{
    Pose q{};
    if (!p) {
        q.R[0] = q.R[4] = q.R[8] = 1.0;
        return q;
    }
    for (int i = 0; i < 9; ++i) q.R[i] = p->R[i];
    for (int i = 0; i < 3; ++i) q.t[i] = p->t[i];
    return q;
}

bool finite_pose(const vm_pose* p)
{
    if (!p) return true;
    for (int i = 0; i < 9; ++i)
        if (!(p->R[i] == p->R[i]) || p->R[i] > 1e300 || p->R[i] < -1e300) return false;
    for (int i = 0; i < 3; ++i)
        if (!(p->t[i] == p->t[i]) || p->t[i] > 1e300 || p->t[i] < -1e300) return false;
    return true;
}

uint32_t map_k_bound(vm_map m, uint32_t min_cluster)
{
    if (min_cluster < 1) min_cluster = 1;
    return m->cap / min_cluster + 1;
}

void fill_cluster_view(vm_map m, uint32_t min_cluster, vm_clusters* out)
{
    out->k_cap = map_k_bound(m, min_cluster);
    out->n_cap = m->cap;
    out->d_meta = m->ctr->meta;
    out->d_off = m->b.cl_off;
    out->d_x = m->b.cl_x;
    out->d_y = m->b.cl_y;
    out->d_z = m->b.cl_z;
    out->d_key = m->b.cl_key;
    out->d_tag = m->b.cl_tag;
}

vm_status check_planes(const vm_planes* p, uint32_t n_hyp)
{
    if (!p || bad_ptr(p->d_plane) || bad_ptr(p->d_best_h) || bad_ptr(p->d_n_inliers) || bad_ptr(p->d_in_off) ||
        bad_ptr(p->d_status) || (p->in_cap > 0 && bad_ptr(p->d_in_idx)))
        return VM_E_ARG;
    (void)n_hyp;
    return VM_OK;
}

vm_status check_hulls(const vm_hulls_out* o)
{
    if (!o || bad_ptr(o->d_v_off) || bad_ptr(o->d_area) || bad_ptr(o->d_status) ||
        (o->v_cap > 0 && (bad_ptr(o->d_v_idx) || bad_ptr(o->d_v_xyz))))
        return VM_E_ARG;
    return VM_OK;
}

vm_status check_params(const vm_ransac_params* p)
{
    if (!p || p->n_hyp < 1 || p->n_hyp > 65536 || !(p->eps > 0.0f) || p->reserved != 0) return VM_E_ARG;
    return VM_OK;
}

vm_status check_clusters(const vm_clusters* c)
{
    if (!c || bad_ptr(c->d_meta) || bad_ptr(c->d_off) || bad_ptr(c->d_x) || bad_ptr(c->d_y) || bad_ptr(c->d_z) ||
        bad_ptr(c->d_tag))
        return VM_E_ARG;
    return VM_OK;
}

}  // namespace

extern "C" {

const char* vm_status_string(vm_status s)
{
    switch (s) {
        case VM_OK: return "ok";
        case VM_E_ARG: return "invalid argument";
        case VM_E_OOM: return "device allocation failed";
        case VM_E_CAPACITY: return "capacity exceeded";
        case VM_E_DEVICE: return "HIP runtime error";
        case VM_E_STATE: return "call out of order";
        default: return "unknown status";
    }
}

int32_t vm_version(void) { return 100; }

vm_status vm_map_create(const vm_map_desc* d, vm_map* out)
{
    if (!d || !out) return VM_E_ARG;
    *out = nullptr;
    if (!(d->voxel_size > 0.0) || d->voxel_size > 1e6) return VM_E_ARG;
    for (int a = 0; a < 3; ++a) {
        if (d->dims[a] < 1) return VM_E_ARG;
        if (!(d->origin[a] == d->origin[a]) || d->origin[a] > 1e12 || d->origin[a] < -1e12) return VM_E_ARG;
    }
    const uint64_t ncell = (uint64_t)d->dims[0] * (uint64_t)d->dims[1] * (uint64_t)d->dims[2];
    if (ncell >= (1ull << 32) || ncell == 0) return VM_E_ARG;
    if (d->hash_capacity_log2 < 10 || d->hash_capacity_log2 > 30) return VM_E_ARG;
    if (d->reserved != 0 || (d->insert_batch_log2 != 0 && (d->insert_batch_log2 < 16 || d->insert_batch_log2 > 26)))
        return VM_E_ARG;

    vm_map m = new (std::nothrow) vm_map_s();
    if (!m) return VM_E_OOM;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return VM_E_DEVICE;
    }
    m->cap = 1u << d->hash_capacity_log2;
    for (int a = 0; a < 3; ++a) {
        m->g.origin[a] = d->origin[a];
        m->g.dims[a] = d->dims[a];
    }
    m->g.voxel_size = d->voxel_size;
    m->g.inv_q = 1048576.0 / d->voxel_size;
    m->g.nwords = (uint32_t)((ncell + 31) / 32);

    const size_t cap = m->cap;
    vm_status st = VM_OK;
    auto A = [&](void** p, size_t bytes) {
        if (st == VM_OK) st = map_alloc(m, p, bytes);
    };
    A((void**)&m->h.slot, cap * sizeof(Slot));
    m->h.log2cap = d->hash_capacity_log2;
    m->h.mask = m->cap - 1;
    A((void**)&m->bits, (size_t)m->g.nwords * 4);
    A((void**)&m->ctr, sizeof(DevCounters));
    SegBuffers& b = m->b;
    A((void**)&b.occ_key, cap * 4);
    A((void**)&b.parent, cap * 4);
    A((void**)&b.csize, cap * 4);
    A((void**)&b.scan_a, cap * 4);
    A((void**)&b.scan_b, cap * 4);
    for (int i = 0; i < 2; ++i) {
        A((void**)&b.sort_k[i], cap * 4);
        A((void**)&b.sort_v[i], cap * 4);
    }
    A((void**)&b.cl_off, (cap + 2) * 4);
    A((void**)&b.cl_tag, cap * 4);
    A((void**)&b.cl_key, cap * 4);
    A((void**)&b.cl_x, cap * 4);
    A((void**)&b.cl_y, cap * 4);
    A((void**)&b.cl_z, cap * 4);
    A((void**)&b.wrank, ((size_t)m->g.nwords + 1) * 4);
    const uint32_t batch = 1u << (d->insert_batch_log2 ? d->insert_batch_log2 : 22);
    const uint64_t scan_n = std::max<uint64_t>(std::max<uint64_t>(cap, m->g.nwords),
                                               std::max<uint64_t>(radix_hist_words(cap), bucket_hist_words(batch)));
    // scan partials; also the fused scans' per-tile totals (3 words per 1024 items)
    A((void**)&b.blk, std::max<size_t>(scan_blk_words(scan_n), 3 * (size_t)ts_tiles(scan_n)) * 4);
    A((void**)&b.hist, radix_hist_words(cap) * 4);
    A((void**)&b.pairs, ccl_tiles(m->g) * kCclTilePairs * 8);
    A((void**)&b.npair, ccl_tiles(m->g) * 4);
    InsertScratch& ins = m->ins;
    ins.cap = batch;
    A((void**)&ins.key, (size_t)batch * 4);
    A((void**)&ins.rec, (size_t)batch * 16);
    A((void**)&ins.packed, (size_t)batch * 8);
    A((void**)&ins.hist, bucket_hist_words(batch) * 4);
    ins.blk = b.blk;
    if (st != VM_OK) {
        map_free_all(m);
        delete m;
        return st;
    }
    if (launch_clear(m->g, m->h, m->bits, m->ctr, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        map_free_all(m);
        delete m;
        return VM_E_DEVICE;
    }
    *out = m;
    return VM_OK;
}

vm_status vm_map_destroy(vm_map m)
{
    if (!m) return VM_E_ARG;
    (void)hipDeviceSynchronize();
    map_free_all(m);
    delete m;
    return VM_OK;
}

vm_status vm_map_clear(vm_map m, void* stream)
{
    if (!m) return VM_E_ARG;
    if (capturing((hipStream_t)stream)) return VM_E_STATE;   // clears with memset nodes
    VM_HIP(launch_clear(m->g, m->h, m->bits, m->ctr, (hipStream_t)stream));
    m->have_clusters = false;
    return VM_OK;
}

vm_status vm_map_stats(vm_map m, void* stream, vm_map_stats_t* out)
{
    if (!m || !out) return VM_E_ARG;
    if (capturing((hipStream_t)stream)) return VM_E_STATE;
    VM_HIP(hipStreamSynchronize((hipStream_t)stream));
    DevCounters c;
    VM_HIP(hipMemcpy(&c, m->ctr, sizeof c, hipMemcpyDeviceToHost));
    out->occupied = c.occupied;
    out->points_in = c.points_in;
    out->points_dropped = c.points_dropped;
    out->points_lost = c.points_lost;
    out->status_flags = c.flags;
    out->hash_capacity_log2 = m->h.log2cap;
    out->last_touched = c.touched;
    out->voxels_cleared = c.cleared;
    out->voxels_shifted_out = c.shifted_out;
    return VM_OK;
}

vm_status vm_map_stats_async(vm_map m, vm_map_stats_t* d_out, void* stream)
{
    if (!m || !d_out) return VM_E_ARG;
    VM_HIP(launch_stats(m->ctr, m->h.log2cap, d_out, (hipStream_t)stream));
    return VM_OK;
}

vm_status vm_insert(vm_map m, const float* d_xyz, int64_t n, const vm_pose* pose, void* stream)
{
    if (!m || n < 0 || (n > 0 && !d_xyz) || !finite_pose(pose)) return VM_E_ARG;
    if (n == 0) return VM_OK;
    StageScope t(VM_STAGE_INSERT, (hipStream_t)stream);
    VM_HIP(launch_insert(d_xyz, n, pose_of(pose), m->g, m->h, m->bits, m->ctr, m->ins, (hipStream_t)stream));
    return VM_OK;
}

vm_status vm_map_shift(vm_map m, int32_t dx, int32_t dy, int32_t dz, void* stream)
{
    if (!m) return VM_E_ARG;
    const int32_t lim = 1 << 30;
    if (dx <= -lim || dx >= lim || dy <= -lim || dy >= lim || dz <= -lim || dz >= lim) return VM_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return VM_E_STATE;
    if (dx == 0 && dy == 0 && dz == 0) return VM_OK;
    VM_HIP(launch_rank(m->g, m->bits, m->b, m->cap, m->ctr, s));
    VM_HIP(launch_scroll(m->g, m->h, m->bits, m->b, m->cap, dx, dy, dz, m->ctr, s));
    const int32_t d[3] = {dx, dy, dz};
    for (int k = 0; k < 3; ++k) m->g.origin[k] = m->g.origin[k] + (double)d[k] * m->g.voxel_size;
    m->have_clusters = false;
    return VM_OK;
}

vm_status vm_map_recenter(vm_map m, const double center[3], int32_t shift_out[3], void* stream)
{
    if (!m || !center) return VM_E_ARG;
    int32_t d[3];
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(center[k])) return VM_E_ARG;
        const double c = floor((center[k] - m->g.origin[k]) / m->g.voxel_size) - (double)(m->g.dims[k] / 2);
        if (!(c > -1073741824.0 && c < 1073741824.0)) return VM_E_ARG;
        d[k] = (int32_t)c;
    }
    if (shift_out)
        for (int k = 0; k < 3; ++k) shift_out[k] = d[k];
    return vm_map_shift(m, d[0], d[1], d[2], stream);
}

vm_status vm_map_origin(vm_map m, double origin_out[3])
{
    if (!m || !origin_out) return VM_E_ARG;
    for (int k = 0; k < 3; ++k) origin_out[k] = m->g.origin[k];
    return VM_OK;
}

vm_status vm_clear_rays(vm_map m, const float* d_xyz, int64_t n, const vm_pose* pose, void* stream)
{
    if (!m || n < 0 || (n > 0 && !d_xyz) || !finite_pose(pose)) return VM_E_ARG;
    // the sensor's voxel, found as a point's voxel is: the floor of the
    // fixed-point coordinate, then its floor division by 2^20
    const Pose q = pose_of(pose);
    int32_t sv[3];
    for (int k = 0; k < 3; ++k) {
        const double f = floor((q.t[k] - m->g.origin[k]) * m->g.inv_q);
        if (!(f >= 0.0 && f < (double)m->g.dims[k] * 1048576.0)) return VM_E_ARG;   // outside the grid
        sv[k] = (int32_t)((int64_t)f >> 20);
    }
    hipStream_t s = (hipStream_t)stream;
    if (!m->clr_mem) {
        if (capturing(s)) return VM_E_STATE;   // no allocation inside a capture
        const size_t bytes = (size_t)m->g.nwords * 4 * 2;
        if (hipMalloc((void**)&m->clr_mem, bytes) != hipSuccess) {
            (void)hipGetLastError();
            m->clr_mem = nullptr;
            return VM_E_OOM;
        }
        if (hipMemset(m->clr_mem, 0, bytes) != hipSuccess) {
            (void)hipFree(m->clr_mem);
            m->clr_mem = nullptr;
            return VM_E_DEVICE;
        }
    }
    StageScope t(VM_STAGE_CLEAR, s);
    VM_HIP(launch_clear_rays(d_xyz, n, q, m->g, sv, m->h, m->bits, m->clr_mem, m->clr_mem + m->g.nwords, m->ctr, s));
    return VM_OK;
}

vm_status vm_map_export(vm_map m, uint32_t* d_key, uint32_t* d_count, uint64_t* d_sum, float* d_mean, uint64_t cap,
                        uint64_t* n_out, void* stream)
{
    if (!m || !n_out) return VM_E_ARG;
    if (capturing((hipStream_t)stream)) return VM_E_STATE;
    hipStream_t s = (hipStream_t)stream;
    VM_HIP(launch_rank(m->g, m->bits, m->b, m->cap, m->ctr, s));
    VM_HIP(launch_export(m->g, m->h, m->b, m->ctr, d_key, d_count, (unsigned long long*)d_sum, d_mean, cap, s));
    VM_HIP(hipStreamSynchronize(s));
    DevCounters c;
    VM_HIP(hipMemcpy(&c, m->ctr, sizeof c, hipMemcpyDeviceToHost));
    *n_out = c.n_occ;
    return c.n_occ > cap ? VM_E_CAPACITY : VM_OK;
}

vm_status vm_map_import(vm_map m, const uint32_t* d_key, const uint32_t* d_count, const uint64_t* d_sum, uint64_t n,
                        void* stream)
{
    if (!m || (n > 0 && (!d_key || !d_count || !d_sum))) return VM_E_ARG;
    if (capturing((hipStream_t)stream)) return VM_E_STATE;
    if (n > m->cap / 2 + m->cap / 4) return VM_E_CAPACITY;
    VM_HIP(launch_import(m->g, m->h, m->bits, m->ctr, d_key, d_count, (const unsigned long long*)d_sum, n,
                         (hipStream_t)stream));
    m->have_clusters = false;
    return VM_OK;
}

vm_status vm_ccl(vm_map m, uint32_t min_cluster, uint32_t* d_labels, vm_clusters* out, void* stream)
{
    if (!m) return VM_E_ARG;
    if (min_cluster < 1) min_cluster = 1;
    hipStream_t s = (hipStream_t)stream;
    {
        StageScope t(VM_STAGE_RANK, s);
        VM_HIP(launch_rank(m->g, m->bits, m->b, m->cap, m->ctr, s));
    }
    VM_HIP(launch_ccl(m->g, m->bits, m->b, m->cap, m->ctr, s));
    VM_HIP(launch_group(m->g, m->h, m->b, m->cap, min_cluster, d_labels, m->ctr, s));
    m->have_clusters = true;
    m->last_min_cluster = min_cluster;
    if (out) fill_cluster_view(m, min_cluster, out);
    return VM_OK;
}

vm_status vm_ccl_propagate(vm_map m, uint32_t min_cluster, uint32_t* d_labels, vm_clusters* out, uint32_t* sweeps,
                           void* stream)
{
    if (!m) return VM_E_ARG;
    if (min_cluster < 1) min_cluster = 1;
    hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return VM_E_STATE;   // the host decides when to stop
    if (!m->lp_flags) {
        if (hipMalloc((void**)&m->lp_flags, kLpBatchMax * 4) != hipSuccess) {
            (void)hipGetLastError();
            m->lp_flags = nullptr;
            return VM_E_OOM;
        }
        if (hipHostMalloc((void**)&m->lp_host, kLpBatchMax * 4, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            m->lp_host = nullptr;
            (void)hipFree(m->lp_flags);
            m->lp_flags = nullptr;
            return VM_E_OOM;
        }
    }
    {
        StageScope t(VM_STAGE_RANK, s);
        VM_HIP(launch_rank(m->g, m->bits, m->b, m->cap, m->ctr, s));
    }
    uint32_t* label = m->b.sort_v[1];   // free until the grouping step
    uint32_t total = 0;
    {
        StageScope t(VM_STAGE_CCL, s);
        VM_HIP(launch_lp_init(m->b, m->cap, label, m->ctr, s));
        // batches of 1, 2, 4, ... sweeps; the first sweep that changes nothing
        // ends the loop (the sweeps after it in its batch change nothing either)
        uint32_t batch = 1;
        for (;;) {
            VM_HIP(launch_lp_sweeps(m->g, m->bits, m->b, m->cap, label, m->lp_flags, batch, m->ctr, s));
            VM_HIP(hipMemcpyAsync(m->lp_host, m->lp_flags, batch * 4, hipMemcpyDeviceToHost, s));
            VM_HIP(hipStreamSynchronize(s));
            uint32_t i = 0;
            while (i < batch && m->lp_host[i]) ++i;
            total += i < batch ? i + 1 : batch;
            if (i < batch) break;
            if (total > (1u << 24)) return VM_E_STATE;   // cannot happen: labels only decrease
            batch = batch * 2 < kLpBatchMax ? batch * 2 : kLpBatchMax;
        }
    }
    {
        StageScope t(VM_STAGE_CCL_LINK, s);
        VM_HIP(launch_lp_finish(m->bits, m->b, m->cap, label, m->ctr, s));
    }
    VM_HIP(launch_group(m->g, m->h, m->b, m->cap, min_cluster, d_labels, m->ctr, s));
    m->have_clusters = true;
    m->last_min_cluster = min_cluster;
    if (sweeps) *sweeps = total;
    if (out) fill_cluster_view(m, min_cluster, out);
    return VM_OK;
}

vm_status vm_ccl_steppable(vm_map m, const vm_step_params* sp, uint32_t min_cluster, float* d_normal,
                           uint8_t* d_steppable, uint32_t* d_labels, vm_clusters* out, void* stream)
{
    if (!m || !step_params_ok(sp)) return VM_E_ARG;
    if (min_cluster < 1) min_cluster = 1;
    hipStream_t s = (hipStream_t)stream;
    if (!m->step_mem) {
        if (capturing(s)) return VM_E_STATE;   // no allocation inside a capture
        const size_t cap = m->cap;
        if (hipMalloc(&m->step_mem, cap * 16 * 2 + cap + 256) != hipSuccess) {
            (void)hipGetLastError();
            m->step_mem = nullptr;
            return VM_E_OOM;
        }
        char* p = (char*)m->step_mem;
        m->sb.mean = (float4*)p;
        m->sb.normal = (float4*)(p + cap * 16);
        m->sb.step = (uint8_t*)(p + cap * 32);
    }
    {
        StageScope t(VM_STAGE_RANK, s);
        VM_HIP(launch_rank(m->g, m->bits, m->b, m->cap, m->ctr, s));
    }
    {
        StageScope t(VM_STAGE_CCL, s);
        VM_HIP(launch_steppable(m->g, m->h, m->bits, m->b, m->cap, m->sb, sp->radius, sp->n_th, sp->cos_th, sp->d_th,
                                d_normal, d_steppable, m->ctr, s));
    }
    VM_HIP(launch_group(m->g, m->h, m->b, m->cap, min_cluster, nullptr, m->ctr, s));
    if (d_labels) VM_HIP(launch_step_labels(m->b, m->sb, m->cap, m->ctr, d_labels, s));
    m->have_clusters = true;
    m->last_min_cluster = min_cluster;
    if (out) fill_cluster_view(m, min_cluster, out);
    return VM_OK;
}

size_t vm_workspace_bytes(uint32_t k_cap, uint32_t n_cap, uint32_t n_hyp)
{
    // one buffer serves both the multi-launch passes and the persistent one
    return std::max(work_layout(nullptr, k_cap, n_cap, n_hyp).bytes, fused_workspace_bytes(k_cap, n_cap, n_hyp));
}

vm_status vm_ransac_planes(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* out, void* d_work,
                           size_t work_bytes, void* stream)
{
    if (check_clusters(cl) != VM_OK || check_params(params) != VM_OK || check_planes(out, params ? params->n_hyp : 0) != VM_OK ||
        !d_work)
        return VM_E_ARG;
    const uint32_t kc = std::min(cl->k_cap, out->k_cap);
    const WorkLayout w = work_layout(d_work, kc, cl->n_cap, params->n_hyp);
    if (work_bytes < w.bytes) return VM_E_CAPACITY;
    return ransac_planes(*cl, *params, *out, w, (hipStream_t)stream);
}

// ---- the allocation-free form of vm_ransac_planes -------------------------------
// Its workspace is this file-scope device array: every GPU the library runs
// on holds one copy, at its own address, until the process ends.  In host code
// the array's name is only a stand-in, so the device address is looked up
// once per device (with that device current) and only that address is used.
namespace {
constexpr size_t kNoAllocWorkBytes = VM_NOALLOC_WORK_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocWorkBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the current device's copy of `scratch` (nullptr on failure)
void* scratch_of_current_device()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}   // namespace

vm_status vm_ransac_planes_noalloc(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* out,
                                   void* stream)
{
    if (check_clusters(cl) != VM_OK || check_params(params) != VM_OK || check_planes(out, params ? params->n_hyp : 0) != VM_OK)
        return VM_E_ARG;
    const uint32_t kc = std::min(cl->k_cap, out->k_cap);
    if (work_layout(nullptr, kc, cl->n_cap, params->n_hyp).bytes > kNoAllocWorkBytes) return VM_E_CAPACITY;
    void* base = scratch_of_current_device();
    if (!base) return VM_E_DEVICE;
    const WorkLayout w = work_layout(base, kc, cl->n_cap, params->n_hyp);
    return ransac_planes(*cl, *params, *out, w, (hipStream_t)stream);
}

vm_status vm_set_count_config(const vm_count_config* cfg)
{
    const vm_count_config c = cfg ? *cfg : count_config_default();
    if (!count_config_valid(c)) return VM_E_ARG;
    count_config_set(c);
    return VM_OK;
}

vm_status vm_get_count_config(vm_count_config* out)
{
    if (!out) return VM_E_ARG;
    *out = count_config_get();
    return VM_OK;
}

namespace {
// one field of the counting decomposition and the values tried for it
struct TuneAxis {
    uint32_t vm_count_config::*field;
    uint32_t values[6];
    int n;
};
}   // namespace

vm_status vm_autotune_count(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* out, void* d_work,
                            size_t work_bytes, void* stream, uint32_t reps, vm_count_config* best)
{
    if (reps < 1 || reps > 16) return VM_E_ARG;
    const hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return VM_E_STATE;
    const vm_count_config start = count_config_get();
    // validates the arguments and warms up under the current setting
    vm_status st = vm_ransac_planes(cl, params, out, d_work, work_bytes, stream);
    if (st != VM_OK) return st;
    hipEvent_t e0, e1;
    VM_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return VM_E_DEVICE;
    }
    // average milliseconds of `reps` calls under c (after one untimed call)
    auto time_of = [&](const vm_count_config& c, float* ms) -> vm_status {
        count_config_set(c);
        vm_status r = vm_ransac_planes(cl, params, out, d_work, work_bytes, stream);
        if (r != VM_OK) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return VM_E_DEVICE;
        for (uint32_t i = 0; i < reps && r == VM_OK; ++i) r = vm_ransac_planes(cl, params, out, d_work, work_bytes, stream);
        if (r != VM_OK) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return VM_E_DEVICE;
        *ms /= (float)reps;
        return VM_OK;
    };
    const TuneAxis axes[] = {
        {&vm_count_config::wave_max_points, {0, 256, 512, 768, 1024}, 5},
        {&vm_count_config::plane_max_points, {0, 64, 128, 192, 256}, 5},
        {&vm_count_config::count_grid, {1024, 2048, 4096, 8192, 16384}, 5},
        {&vm_count_config::chunk_mult, {1, 2, 4, 8}, 4},
    };
    vm_count_config cur = start;
    float cur_ms = 0.f;
    st = time_of(cur, &cur_ms);
    for (const TuneAxis& a : axes) {
        for (int i = 0; i < a.n && st == VM_OK; ++i) {
            vm_count_config c = cur;
            c.*a.field = a.values[i];
            if (c.*a.field == cur.*a.field) continue;
            // a smaller wave bound caps the plane bound
            if (c.plane_max_points > c.wave_max_points) c.plane_max_points = c.wave_max_points;
            if (!count_config_valid(c)) continue;
            float ms = 0.f;
            st = time_of(c, &ms);
            if (st == VM_OK && ms < cur_ms) {
                cur = c;
                cur_ms = ms;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VM_OK) {
        count_config_set(start);
        return st;
    }
    count_config_set(cur);
    if (best) *best = cur;
    return VM_OK;
}

vm_status vm_planes_hulls(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* planes,
                          vm_hulls_out* hulls, void* d_work, size_t work_bytes, void* stream)
{
    if (check_clusters(cl) != VM_OK || check_params(params) != VM_OK || check_planes(planes, 1) != VM_OK ||
        check_hulls(hulls) != VM_OK || !d_work)
        return VM_E_ARG;
    const uint32_t kc = std::min(cl->k_cap, std::min(planes->k_cap, hulls->k_cap));
    if (kc > kOneBlockMax) return VM_E_CAPACITY;
    if (work_bytes < vm_workspace_bytes(kc, cl->n_cap, params->n_hyp)) return VM_E_CAPACITY;
    vm_fused_config cfg;
    if (!fused_cache_get(kc, cl->n_cap, params->n_hyp, &cfg)) cfg = fused_config_get();
    return planes_and_hulls(*cl, *params, nullptr, *planes, *hulls, d_work, work_bytes, cfg, (hipStream_t)stream);
}

size_t vm_multi_workspace_bytes(uint32_t k_cap, uint32_t n_cap, uint32_t n_hyp)
{
    return multi_workspace_bytes(k_cap, n_cap, n_hyp);
}

vm_status vm_planes_hulls_multi(uint32_t n, const vm_clusters* sets, const uint32_t* frames,
                                const vm_ransac_params* params, vm_planes* planes, vm_hulls_out* hulls, uint32_t k_cap,
                                uint32_t n_cap, void* d_work, size_t work_bytes, void* stream)
{
    if (n < 1 || n > 16 || !sets || !frames || !planes || !hulls || !d_work || check_params(params) != VM_OK ||
        k_cap < 1 || k_cap > kOneBlockMax)
        return VM_E_ARG;
    for (uint32_t i = 0; i < n; ++i)
        if (check_clusters(&sets[i]) != VM_OK || check_planes(&planes[i], 1) != VM_OK ||
            check_hulls(&hulls[i]) != VM_OK)
            return VM_E_ARG;
    if (work_bytes < multi_workspace_bytes(k_cap, n_cap, params->n_hyp)) return VM_E_CAPACITY;
    return planes_hulls_multi(n, sets, frames, *params, planes, hulls, k_cap, n_cap, d_work, work_bytes,
                              (hipStream_t)stream);
}

vm_status vm_set_fused_config(const vm_fused_config* cfg)
{
    const vm_fused_config c = cfg ? *cfg : fused_config_default();
    if (!fused_config_valid(c)) return VM_E_ARG;
    fused_config_set(c);
    if (!cfg) fused_cache_clear();
    return VM_OK;
}

vm_status vm_get_fused_config(vm_fused_config* out)
{
    if (!out) return VM_E_ARG;
    *out = fused_config_get();
    return VM_OK;
}

vm_status vm_autotune_fused(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* planes,
                            vm_hulls_out* hulls, void* d_work, size_t work_bytes, void* stream, uint32_t reps,
                            vm_fused_config* best)
{
    if (reps < 1 || reps > 16) return VM_E_ARG;
    const hipStream_t s = (hipStream_t)stream;
    if (capturing(s)) return VM_E_STATE;
    // validates the arguments and warms up
    vm_status st = vm_planes_hulls(cl, params, planes, hulls, d_work, work_bytes, stream);
    if (st != VM_OK) return st;
    const uint32_t kc = std::min(cl->k_cap, std::min(planes->k_cap, hulls->k_cap));
    hipEvent_t e0, e1;
    VM_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return VM_E_DEVICE;
    }
    auto time_of = [&](const vm_fused_config& c, float* ms) -> vm_status {
        vm_status r = planes_and_hulls(*cl, *params, nullptr, *planes, *hulls, d_work, work_bytes, c, s);
        if (r != VM_OK) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return VM_E_DEVICE;
        for (uint32_t i = 0; i < reps && r == VM_OK; ++i)
            r = planes_and_hulls(*cl, *params, nullptr, *planes, *hulls, d_work, work_bytes, c, s);
        if (r != VM_OK) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(ms, e0, e1) != hipSuccess)
            return VM_E_DEVICE;
        *ms /= (float)reps;
        return VM_OK;
    };
    struct Axis {
        uint32_t vm_fused_config::*field;
        uint32_t values[6];
        int n;
    };
    const Axis axes[] = {
        {&vm_fused_config::groups_per_cu, {2, 3, 4, 5, 6, 8}, 6},
        {&vm_fused_config::hyp_chunk, {128, 256, 384, 512}, 4},
        {&vm_fused_config::small_max, {0, 64, 128, 256}, 4},
    };
    vm_fused_config cur;
    if (!fused_cache_get(kc, cl->n_cap, params->n_hyp, &cur)) cur = fused_config_get();
    float cur_ms = 0.f;
    st = time_of(cur, &cur_ms);
    for (const Axis& a : axes) {
        for (int i = 0; i < a.n && st == VM_OK; ++i) {
            vm_fused_config c = cur;
            c.*a.field = a.values[i];
            if (c.*a.field == cur.*a.field || !fused_config_valid(c)) continue;
            float ms = 0.f;
            st = time_of(c, &ms);
            if (st == VM_OK && ms < cur_ms) {
                cur = c;
                cur_ms = ms;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VM_OK) return st;
    fused_cache_put(kc, cl->n_cap, params->n_hyp, cur);
    if (best) *best = cur;
    return VM_OK;
}

vm_status vm_hulls(const vm_clusters* cl, const vm_planes* planes, vm_hulls_out* out, void* d_work, size_t work_bytes,
                   void* stream)
{
    if (check_clusters(cl) != VM_OK || check_planes(planes, 1) != VM_OK || check_hulls(out) != VM_OK || !d_work)
        return VM_E_ARG;
    // the hull pass needs no per-hypothesis storage
    const uint32_t kc = std::min(std::min(cl->k_cap, planes->k_cap), out->k_cap);
    const WorkLayout w = work_layout(d_work, kc, cl->n_cap, 1);
    if (work_bytes < w.bytes) return VM_E_CAPACITY;
    return hulls(*cl, *planes, *out, w, (hipStream_t)stream);
}

namespace {
vm_status segment_frame_impl(vm_map m, const float* d_xyz, int64_t n, const vm_pose* pose, const vm_seg_params* params,
                             const vm_step_params* sp, vm_planes* planes, vm_hulls_out* hulls_out, uint32_t* d_labels,
                             vm_clusters* clusters_out, void* stream);
}

vm_status vm_segment_frame(vm_map m, const float* d_xyz, int64_t n, const vm_pose* pose, const vm_seg_params* params,
                           vm_planes* planes, vm_hulls_out* hulls_out, uint32_t* d_labels, vm_clusters* clusters_out,
                           void* stream)
{
    return segment_frame_impl(m, d_xyz, n, pose, params, nullptr, planes, hulls_out, d_labels, clusters_out, stream);
}

vm_status vm_segment_frame_steppable(vm_map m, const float* d_xyz, int64_t n, const vm_pose* pose,
                                     const vm_seg_params* params, const vm_step_params* sp, vm_planes* planes,
                                     vm_hulls_out* hulls_out, uint32_t* d_labels, vm_clusters* clusters_out,
                                     void* stream)
{
    if (!step_params_ok(sp)) return VM_E_ARG;
    return segment_frame_impl(m, d_xyz, n, pose, params, sp, planes, hulls_out, d_labels, clusters_out, stream);
}

}  // extern "C"

namespace {
vm_status segment_frame_impl(vm_map m, const float* d_xyz, int64_t n, const vm_pose* pose, const vm_seg_params* params,
                             const vm_step_params* sp, vm_planes* planes, vm_hulls_out* hulls_out, uint32_t* d_labels,
                             vm_clusters* clusters_out, void* stream)
{
    if (!m || !params || (params->flags & ~VM_SEG_CLEAR_RAYS) != 0 || check_params(&params->ransac) != VM_OK)
        return VM_E_ARG;
    if (check_planes(planes, params->ransac.n_hyp) != VM_OK || check_hulls(hulls_out) != VM_OK) return VM_E_ARG;
    if (n < 0 || (n > 0 && !d_xyz) || !finite_pose(pose)) return VM_E_ARG;
    const uint32_t minc = params->min_cluster < 1 ? 1 : params->min_cluster;
    const uint32_t kb = std::min(map_k_bound(m, minc), planes->k_cap);
    // the map's own workspace: allocated once per (cluster bound, hypotheses)
    if (!m->work || m->work_k < kb || m->work_hyp < params->ransac.n_hyp) {
        if (capturing((hipStream_t)stream)) return VM_E_STATE;   // no allocation inside a capture
        const uint32_t k = std::max(kb, m->work_k);
        const uint32_t hh = std::max(params->ransac.n_hyp, m->work_hyp);
        const size_t bytes = vm_workspace_bytes(k, m->cap, hh);
        VM_HIP(hipStreamSynchronize((hipStream_t)stream));
        if (m->work) (void)hipFree(m->work);
        m->work = nullptr;
        if (hipMalloc(&m->work, bytes) != hipSuccess) {
            (void)hipGetLastError();
            m->work_bytes = 0;
            return VM_E_OOM;
        }
        m->work_bytes = bytes;
        m->work_k = k;
        m->work_hyp = hh;
    }
    vm_status st = VM_OK;
    if (params->flags & VM_SEG_CLEAR_RAYS) {
        st = vm_clear_rays(m, d_xyz, n, pose, stream);
        if (st != VM_OK) return st;
    }
    st = vm_insert(m, d_xyz, n, pose, stream);
    if (st != VM_OK) return st;
    vm_clusters cl;
    st = sp ? vm_ccl_steppable(m, sp, minc, nullptr, nullptr, d_labels, &cl, stream)
            : vm_ccl(m, minc, d_labels, &cl, stream);
    if (st != VM_OK) return st;
    if (clusters_out) *clusters_out = cl;
    const WorkLayout w = work_layout(m->work, kb, cl.n_cap, params->ransac.n_hyp);
    if (w.bytes > m->work_bytes) return VM_E_STATE;
    st = ransac_planes(cl, params->ransac, *planes, w, (hipStream_t)stream);
    if (st != VM_OK) return st;
    return hulls(cl, *planes, *hulls_out, w, (hipStream_t)stream);
}
}  // namespace

extern "C" {

vm_status vm_capture_begin(void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (!s) return VM_E_ARG;   // the null stream cannot be captured
    if (capturing(s)) return VM_E_STATE;
    VM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    return VM_OK;
}

vm_status vm_capture_end(void* stream, vm_graph* out)
{
    hipStream_t s = (hipStream_t)stream;
    if (!s || !out) return VM_E_ARG;
    *out = nullptr;
    if (!capturing(s)) return VM_E_STATE;
    hipGraph_t g = nullptr;
    VM_HIP(hipStreamEndCapture(s, &g));
    hipGraphExec_t e = nullptr;
    if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return VM_E_DEVICE;
    }
    // the executable graph's resources go to the device now, not on its first launch
    if (hipGraphUpload(e, s) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(e);
        (void)hipGraphDestroy(g);
        return VM_E_DEVICE;
    }
    vm_graph r = new (std::nothrow) vm_graph_s{g, e};
    if (!r) {
        (void)hipGraphExecDestroy(e);
        (void)hipGraphDestroy(g);
        return VM_E_OOM;
    }
    *out = r;
    return VM_OK;
}

vm_status vm_graph_launch(vm_graph g, void* stream)
{
    if (!g) return VM_E_ARG;
    VM_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return VM_OK;
}

vm_status vm_graph_destroy(vm_graph g)
{
    if (!g) return VM_E_ARG;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return VM_OK;
}

vm_status vm_set_stage_timing(int32_t enable)
{
    TimingState& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    t.enabled = enable != 0;
    // events are created here, outside any timed span
    while (t.enabled && t.pool.size() < 1024) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return VM_E_DEVICE;
        t.pool.push_back(e);
    }
    return VM_OK;
}

vm_status vm_stage_times(double* ms_out, uint64_t* launches_out, int32_t n)
{
    if (n < 0 || (n > 0 && (!ms_out || !launches_out))) return VM_E_ARG;
    TimingState& t = timing();
    std::lock_guard<std::mutex> lk(t.mu);
    for (int i = 0; i < n; ++i) {
        ms_out[i] = 0.0;
        launches_out[i] = 0;
    }
    vm_status st = VM_OK;
    for (auto& r : t.recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) st = VM_E_DEVICE;
        if (r.stage >= 0 && r.stage < n) {
            ms_out[r.stage] += ms;
            launches_out[r.stage] += 1;
        }
        t.pool.push_back(r.a);
        t.pool.push_back(r.b);
    }
    t.recs.clear();
    return st;
}

}  // extern "C"

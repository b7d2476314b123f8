/*
 * vm.h -- C ABI of the MI355X (gfx950) voxel-map plane-segmentation library.
 *
 * The library implements the data-parallel path of Niijima et al., "Real-time
 * Multi-Plane Segmentation Based on GPU Accelerated High-Resolution 3D Voxel
 * Mapping for Legged Robot Locomotion" (arXiv 2510.01592):
 *   vm_insert        Sec. III-B, Eq. (1)    points + pose -> sparse voxel map
 *   vm_clear_rays    Sec. III-B, Eq. (2)    free the voxels the frame's rays cross
 *   vm_ccl           Sec. III-C, Alg. 1     occupied voxels -> component labels,
 *                                           clusters (grouping)
 *   vm_ransac_planes Sec. III-C (a)-(c)     one plane + inlier set per cluster
 *   vm_hulls         Sec. III-C, boundary   one convex polygon per plane
 *   vm_segment_frame Sec. III-A overview    all of the above for one frame
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named d_* are device (HBM) pointers on the current HIP device;
 *   everything else is host memory read during the call only.
 * - `stream` is a hipStream_t (passed as void*; NULL = the null stream).  All
 *   device work is enqueued on it and the call returns without waiting,
 *   except where a call says it synchronises.  Device buffers handed to a
 *   call must stay alive until the stream has passed that call.
 * - Argument errors are detected on the host before anything is enqueued and
 *   return VM_E_ARG; nothing is written then.  Conditions only the device can
 *   see (hash table full, output capacity exceeded) never write out of
 *   bounds: the overflowing items are dropped and a VM_FLAG_* bit is OR-ed
 *   into a device status word (the map's, readable with vm_map_stats, or the
 *   caller's d_status).  No C++ exception crosses this ABI.
 * - Calls on one map, and calls sharing one workspace, must be serialised by
 *   the caller (one stream at a time); different maps and workspaces are
 *   independent.
 * - Numeric conventions: IEEE binary32/binary64, round-to-nearest-even, no
 *   contraction; every fused multiply-add is an explicit fma.  The results
 *   are deterministic: they do not depend on launch shapes, scheduling or
 *   stream interleaving.
 */
#ifndef VM_H
#define VM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes (return values) ------------------------------------- */
typedef int32_t vm_status;
#define VM_OK            0
#define VM_E_ARG        -1   /* invalid argument (null pointer, bad size, bad geometry) */
#define VM_E_OOM        -2   /* device allocation failed */
#define VM_E_CAPACITY   -3   /* a host-known size exceeds a capacity */
#define VM_E_DEVICE     -4   /* a HIP runtime call failed */
#define VM_E_STATE      -5   /* call out of order (e.g. no clusters computed yet) */

/* ---- device status flags (OR-ed into a device uint32 word) ------------ */
#define VM_FLAG_HASH_FULL      0x1u  /* a new voxel found no free hash slot; its points were dropped */
#define VM_FLAG_CLUSTERS_CAP   0x2u  /* more clusters than the output's k_cap; the rest were skipped */
#define VM_FLAG_INLIERS_CAP    0x4u  /* inlier index output full; later inliers not listed */
#define VM_FLAG_HULL_CAP       0x8u  /* hull vertex output full; later polygons truncated */
#define VM_FLAG_BAD_CLUSTERS   0x10u /* cluster offsets not ascending from 0 or beyond n_cap; nothing processed */

/* Human-readable text for a status code (static storage). */
const char* vm_status_string(vm_status s);

/* Library version, major*10000 + minor*100 + patch. */
int32_t vm_version(void);

/* ---- the voxel map (Sec. III-B) ---------------------------------------- */
typedef struct vm_map_s* vm_map;

/* Grid geometry and storage of a map.  Voxel (x, y, z) covers
 * [origin + s*(x,y,z), origin + s*(x+1,y+1,z+1)) (half-open cells) and has
 * key x + NX*(y + NY*z); NX*NY*NZ must be below 2^32.  Occupied voxels live in
 * an open-addressing hash of 2^hash_capacity_log2 slots (at most half of them
 * should be used); the map also holds a 1-bit-per-cell occupancy index
 * (NX*NY*NZ/8 bytes) and the per-frame segmentation buffers, all allocated
 * once by vm_map_create. */
typedef struct {
    double   origin[3];           /* metres, map frame */
    double   voxel_size;          /* s, metres, > 0 */
    int32_t  dims[3];             /* NX, NY, NZ, each >= 1 */
    uint32_t hash_capacity_log2;  /* 10..30 */
    uint32_t insert_batch_log2;   /* largest point batch one grouped insert pass takes
                                     (0: 2^22); larger calls are split. 16..26 */
    uint32_t reserved;            /* must be 0 */
} vm_map_desc;

/* Rigid transform map_from_sensor: p_map = R p_sensor + t (R row-major). */
typedef struct {
    double R[9];
    double t[3];
} vm_pose;

typedef struct {
    uint64_t occupied;        /* occupied voxels */
    uint64_t points_in;       /* points accumulated since create/clear */
    uint64_t points_dropped;  /* non-finite or outside the grid */
    uint64_t points_lost;     /* inside the grid but dropped because the hash was full */
    uint32_t status_flags;    /* VM_FLAG_* seen since create/clear */
    uint32_t hash_capacity_log2;
    uint64_t last_touched;    /* voxel slot updates of the last vm_insert call on its
                                 grouped path: one per distinct voxel of each batch
                                 (a voxel with more than 1024 points in one batch may
                                 take more; 0 for calls small enough for per-point
                                 atomics) */
    uint64_t voxels_cleared;  /* voxels cleared by vm_clear_rays since create/clear */
    uint64_t voxels_shifted_out; /* voxels dropped by vm_map_shift since create/clear */
} vm_map_stats_t;

/* Allocate a map on the current device (hipMalloc; the map owns the memory
 * until vm_map_destroy) and clear it (synchronously).  VM_E_ARG for bad
 * geometry, VM_E_OOM if the device allocation fails. */
vm_status vm_map_create(const vm_map_desc* desc, vm_map* out);
vm_status vm_map_destroy(vm_map map);
/* Empty the map (asynchronous on `stream`). */
vm_status vm_map_clear(vm_map map, void* stream);
/* Synchronises `stream`, then reports the map's counters. */
vm_status vm_map_stats(vm_map map, void* stream, vm_map_stats_t* out);

/* Enqueue a copy of the map's counters (as vm_map_stats would report them
 * once `stream` reaches this point) into caller-owned device memory d_out;
 * nothing waits for the host. */
vm_status vm_map_stats_async(vm_map map, vm_map_stats_t* d_out, void* stream);

/* Sec. III-B "Voxel information update", Eq. (1).  Transforms the n float32
 * xyz points at d_xyz (AoS, 12 bytes each, caller-owned device memory) by
 * `pose` in fp64 (x' = fma(R02, z, fma(R01, y, fma(R00, x, t0))), likewise for
 * y', z'), voxelises them, and accumulates each into its voxel: count += 1 and
 * the 2^-20-voxel fixed-point offset added to the voxel's integer sums, so
 * the stored mean is the arithmetic mean that Eq. (1)'s recurrence computes,
 * independent of arrival order.  Non-finite points and points outside the
 * grid are counted and dropped.  Large calls group the points by voxel first
 * (hash buckets, then per-bucket sums) and update each touched voxel once;
 * small ones update per point with integer atomics; both give the same map.  n = 0 is a no-op; n < 0 is
 * VM_E_ARG. */
vm_status vm_insert(vm_map map, const float* d_xyz, int64_t n, const vm_pose* pose, void* stream);

/* Sec. III-B "Voxel information clearing", Eq. (2): free space along the
 * frame's rays.  The sensor sits at the pose's translation t; each of the n
 * points (sensor frame, transformed as in vm_insert) casts a ray on voxel
 * indices from the sensor's voxel to its own voxel: the 3D Bresenham line
 * (the axis of largest extent drives, x before y before z on ties, a minor
 * axis steps when its error term reaches zero), the sensor's voxel included,
 * the point's voxel excluded, cut where the line leaves the grid.  Every
 * occupied voxel on some ray that holds none of the frame's points becomes
 * free: its count and sums return to zero and it leaves the occupancy index
 * (its hash slot keeps the key, so a later vm_insert that lands there simply
 * occupies it again).  The removal set is deduplicated in two bitmaps (cells
 * on a ray, cells holding a point) before any slot is touched, so the result
 * does not depend on point order or scheduling.  Non-finite points and
 * points more than 10^15 quanta (s*2^-20) from the origin cast no ray.  Call
 * it before vm_insert of the same frame.  VM_E_ARG if the sensor lies outside
 * the grid or n < 0; the two bitmaps (2 * NX*NY*NZ/8 bytes) are allocated on
 * the first call (VM_E_STATE if that first call is being captured, VM_E_OOM
 * if the allocation fails). */
vm_status vm_clear_rays(vm_map map, const float* d_xyz, int64_t n, const vm_pose* pose, void* stream);

/* Export the occupied voxels in ascending key order (e.g. for checkpoints
 * and checks).  Synchronises `stream`.  Writes min(occupied, cap) entries:
 * d_key[i], d_count[i], d_sum[3i..3i+2] (integer offset sums, units of
 * s*2^-20), d_mean[3i..3i+2] (float32 voxel mean; may be NULL).  *n_out
 * receives the occupied count; VM_E_CAPACITY if cap is too small (the first
 * cap entries are still written). */
vm_status vm_map_export(vm_map map, uint32_t* d_key, uint32_t* d_count, uint64_t* d_sum,
                        float* d_mean, uint64_t cap, uint64_t* n_out, void* stream);

/* Replace the map's content with n voxels (keys strictly ascending and
 * inside the grid, counts >= 1); the inverse of vm_map_export.
 * Asynchronous. */
vm_status vm_map_import(vm_map map, const uint32_t* d_key, const uint32_t* d_count,
                        const uint64_t* d_sum, uint64_t n, void* stream);

/* Sec. III-B: the local map is robot-centric, its grid follows the robot.
 * Moves the grid by (dx, dy, dz) whole voxels: the origin becomes
 * origin + s*(dx, dy, dz) (fp64), voxel (x, y, z) becomes (x-dx, y-dy, z-dz)
 * with its count and integer sums unchanged (so its mean stays where it was,
 * exactly), and voxels leaving the grid are dropped (counted in
 * voxels_shifted_out).  The hash is rebuilt, which also frees the slots that
 * cleared voxels kept.  The segmentation buffers serve as staging: cluster
 * views of earlier vm_ccl calls become invalid.  Host state changes (the
 * origin), so it cannot be captured (VM_E_STATE).  A zero shift is a no-op;
 * a shift of 2^30 voxels or more on an axis is VM_E_ARG. */
vm_status vm_map_shift(vm_map map, int32_t dx, int32_t dy, int32_t dz, void* stream);

/* The shift that puts the voxel containing `center` (map frame) at the grid's
 * middle voxel (dims/2, integer division), applied with vm_map_shift; the
 * shift goes to shift_out (optional).  VM_E_ARG for a non-finite centre. */
vm_status vm_map_recenter(vm_map map, const double center[3], int32_t shift_out[3], void* stream);

/* The grid's current origin (host memory, immediate). */
vm_status vm_map_origin(vm_map map, double origin_out[3]);

/* ---- clusters (Sec. III-C, Alg. 1 and grouping) ----------------------- */

/* A set of point clusters in CSR form.  Cluster k owns points
 * [d_off[k], d_off[k+1]) of the structure-of-arrays d_x/d_y/d_z; its RANSAC
 * stream is selected by d_tag[k].  The number of clusters and of points can
 * live on the device (d_meta[0] = K, d_meta[1] = total points), so a
 * pipeline never has to wait for the host; k_cap and n_cap bound them and size
 * every grid.  Views returned by vm_ccl point into the map and stay valid
 * until the next vm_ccl / vm_segment_frame / vm_map_destroy on that map. */
typedef struct {
    uint32_t        k_cap;   /* host: upper bound on K (d_off has k_cap+1 entries, d_tag k_cap) */
    uint32_t        n_cap;   /* host: upper bound on the total point count */
    const uint32_t* d_meta;  /* device: [0] = K, [1] = total points */
    const uint32_t* d_off;
    const float*    d_x;
    const float*    d_y;
    const float*    d_z;
    const uint32_t* d_key;   /* device, optional (NULL): voxel key of each point */
    const uint32_t* d_tag;   /* device: per-cluster RNG tag (for map clusters: the label) */
} vm_clusters;

/* Alg. 1's fixed point over all occupied voxels of `map`: every voxel gets
 * the smallest key of its 26-connected component (exact integer result).
 * Then the grouping step: components of at least min_cluster voxels become
 * clusters, ordered by label, with their voxels in ascending key order and
 * each point the voxel's Eq. (1) mean; tag = label.
 * d_labels (optional, NULL to skip): receives one label per occupied voxel
 * in ascending key order (the caller sizes it by vm_map_stats().occupied).
 * `out` receives a device-resident view (see vm_clusters).  Asynchronous. */
vm_status vm_ccl(vm_map map, uint32_t min_cluster, uint32_t* d_labels, vm_clusters* out,
                 void* stream);

/* Alg. 1 run as the paper runs it, as a comparison baseline for vm_ccl:
 * every occupied voxel starts with its own key as label, and sweeps over the
 * 26-adjacency (each edge once) let both ends of an edge take the smaller
 * label with atomic minima, until a sweep changes no label.  The labels, the
 * clusters and every output are those of vm_ccl (the same fixed point); the
 * number of sweeps run, the last one changing nothing, goes to *sweeps
 * (optional).  Synchronises `stream` between batches of sweeps (the host
 * decides when to stop), so it cannot be captured (VM_E_STATE); a small flag
 * buffer is allocated on the first call (VM_E_OOM if that fails). */
vm_status vm_ccl_propagate(vm_map map, uint32_t min_cluster, uint32_t* d_labels, vm_clusters* out,
                           uint32_t* sweeps, void* stream);

/* ---- steppable points (Sec. III-C "Steppable point classification" and
 *      "Clustering of steppable points") --------------------------------- */
typedef struct {
    uint32_t radius;   /* neighbourhood of Eq. (3): occupied voxels at most this many cells away on
                          every axis (the voxel itself included); 1..2 */
    uint32_t n_th;     /* Eq. (4)'s N_th: least neighbour points of a steppable voxel (3) */
    double   cos_th;   /* cos of theta_th (15 deg): Eq. (4) needs n_z >= cos_th; Alg. 1's angle gate
                          needs n_i . n_j > cos_th; in [-1, 1] */
    double   d_th;     /* Alg. 1's distance gate |mu_i - mu_j| < d_th, metres (0.05), > 0 */
} vm_step_params;

/* Eq. (3)-(4) for every occupied voxel of `map`: the normal is the unit
 * eigenvector of the smallest eigenvalue (cyclic Jacobi, fp64) of the scatter
 * matrix of the neighbour voxels' means about their mean (gathered in
 * ascending key order), oriented to +z (ties +y, +x), rounded to float32; a
 * voxel is steppable when it has at least n_th neighbour points and
 * n_z >= cos_th.  Then Alg. 1 over the steppable voxels with both gates, to
 * its fixed point: every steppable voxel gets the smallest key of its gated
 * component; voxels that are not steppable belong to no cluster.  Then the
 * grouping of vm_ccl (components of at least min_cluster voxels, ordered by
 * label).  Optional outputs, ascending key order, sized by the occupied
 * count: d_normal (float32 x 3), d_steppable (uint8), d_labels (0xFFFFFFFF
 * where not steppable).  The map allocates its classification buffers on the
 * first call (VM_E_STATE if that first call is captured).  Asynchronous. */
vm_status vm_ccl_steppable(vm_map map, const vm_step_params* sp, uint32_t min_cluster, float* d_normal,
                           uint8_t* d_steppable, uint32_t* d_labels, vm_clusters* out, void* stream);

/* ---- planes (Sec. III-C "Multi-plane estimation") --------------------- */
typedef struct {
    uint32_t n_hyp;      /* hypotheses per cluster, 1..65536 */
    float    eps;        /* inlier threshold, metres (the paper uses 0.01) */
    uint64_t seed;       /* Philox4x64-10 key word 0 */
    uint32_t frame;      /* counter word 2 (per-map frame number) */
    uint32_t reserved;   /* must be 0 */
    const uint32_t* d_frame;  /* optional device word: when non-NULL the frame number is
                                 read from it when the work executes (graph replays
                                 advance it between launches); `frame` is then unused */
} vm_ransac_params;

/* Per-cluster RANSAC outputs (caller-owned device buffers).  For cluster k:
 * hypothesis h draws three distinct point indices from Philox4x64-10 with key
 * (seed, 0) and counter (h, tag[k], frame, 0), fits the plane through them in
 * fp64 (unit normal oriented to +z, ties to +y then +x; rounded to float32),
 * and counts the points with |fmaf(nz,z,fmaf(ny,y,fmaf(nx,x,d)))| < eps.  The
 * first hypothesis with the largest count wins (degenerate triples count
 * -1).  Clusters with no valid hypothesis get best_h = -1, n_inliers = 0 and
 * a zero plane. */
typedef struct {
    uint32_t  k_cap;       /* capacity of the per-cluster arrays */
    uint32_t  in_cap;      /* capacity of d_in_idx */
    float*    d_plane;     /* [k_cap][4] nx, ny, nz, d of the winner */
    int32_t*  d_best_h;    /* [k_cap] */
    int32_t*  d_n_inliers; /* [k_cap] */
    uint32_t* d_in_off;    /* [k_cap+1] inlier CSR: cluster k's inliers at [in_off[k], in_off[k+1]) */
    uint32_t* d_in_idx;    /* [in_cap] cluster-local point indices, ascending */
    int32_t*  d_counts;    /* optional [k_cap][n_hyp]: every hypothesis' count (NULL to skip) */
    float*    d_hyp;       /* optional [k_cap][n_hyp][4]: every hypothesis' plane (NULL to skip) */
    uint32_t* d_status;    /* [1] device word, VM_FLAG_* OR-ed in (never cleared by the library) */
} vm_planes;

/* Device scratch for vm_ransac_planes / vm_hulls / vm_planes_hulls, in bytes: k_cap is the
 * number of clusters a call may process, min(clusters.k_cap, outputs'
 * k_cap); n_cap the clusters' point bound; n_hyp the hypotheses per cluster
 * (1 for a buffer that only serves vm_hulls). */
size_t vm_workspace_bytes(uint32_t k_cap, uint32_t n_cap, uint32_t n_hyp);

/* Sec. III-C (a)-(c) on every cluster of `cl`, all clusters in one pass.
 * d_work: caller-owned device scratch of at least
 * vm_workspace_bytes(cl->k_cap, cl->n_cap, params->n_hyp) bytes.
 * Asynchronous. */
vm_status vm_ransac_planes(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* out,
                           void* d_work, size_t work_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): vm_ransac_planes
 * with the library's own fixed workspace instead of d_work.  The workspace is
 * one device array of VM_NOALLOC_WORK_BYTES per GPU, held from the first call
 * on that GPU until the process ends; this call allocates nothing.  Calls with
 * vm_workspace_bytes(min(cl->k_cap, out->k_cap), cl->n_cap, params->n_hyp) >
 * VM_NOALLOC_WORK_BYTES return VM_E_CAPACITY before anything is enqueued.
 * Every call on one GPU shares that GPU's array: calls that may overlap on
 * one GPU (different streams, or host threads) race and must be serialised by
 * the caller.  Results are identical to vm_ransac_planes'.  VM_E_DEVICE if the
 * array's device address cannot be obtained. */
#define VM_NOALLOC_WORK_BYTES (64u << 20)
vm_status vm_ransac_planes_noalloc(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* out,
                                   void* stream);

/* Work decomposition of the inlier counting of Sec. III-C (b).  Counts are
 * integer sums of the same tests, so every valid setting gives identical
 * results; only the speed differs.  The setting is process-wide and read
 * when a call is enqueued (a captured graph keeps the one it was captured
 * with). */
typedef struct {
    uint32_t count_grid;        /* workgroups of the tiled counting kernel: a multiple of 8
                                   (one per XCD), 8..65536; default 16384 */
    uint32_t chunk_mult;        /* the hypotheses of a point tile (of a wave-counted cluster) are
                                   split into chunks so that there are about chunk_mult work items
                                   per workgroup (per wave), 1..16; default 2 */
    uint32_t wave_max_points;   /* clusters of at most this many points are counted by one wave
                                   each, 0..1024 (0: all tiled); default 256 */
    uint32_t plane_max_points;  /* of those, clusters of at most this many points put the lanes
                                   over hypotheses instead of points, 0..min(256, wave_max_points);
                                   default 256 */
} vm_count_config;

/* Set the counting decomposition (NULL: the defaults).  VM_E_ARG if a field
 * is out of range (nothing changes then). */
vm_status vm_set_count_config(const vm_count_config* cfg);
vm_status vm_get_count_config(vm_count_config* out);

/* Time vm_ransac_planes on this workload under candidate decompositions
 * (one field at a time, starting from the current setting; `reps` calls
 * each, 1..16) and keep the fastest, which is set and returned in *best.
 * Synchronises `stream`; the outputs hold the last call's (identical)
 * results.  Arguments as for vm_ransac_planes; VM_E_STATE while capturing. */
vm_status vm_autotune_count(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* out, void* d_work,
                            size_t work_bytes, void* stream, uint32_t reps, vm_count_config* best);

/* ---- polygons (Sec. III-C "Boundary polygon generation") -------------- */

/* For cluster k with a plane: the 2D convex hull of its inliers in the
 * plane.  In-plane basis (fp64): u = normalize(a x n) with a = e_x if
 * |nx| < 0.9 else e_y, v = n x u; origin = the first inlier.  Vertices are
 * listed counter-clockwise from the lexicographically smallest (u, v),
 * without collinear or repeated points.  d_v_idx holds cluster-local point
 * indices, d_v_xyz the vertices projected onto the plane (fp64 -> float32),
 * d_area the shoelace area in fp64 (0 if fewer than 3 vertices or no plane). */
typedef struct {
    uint32_t  k_cap;
    uint32_t  v_cap;     /* capacity of d_v_idx / d_v_xyz */
    uint32_t* d_v_off;   /* [k_cap+1] */
    uint32_t* d_v_idx;   /* [v_cap] */
    float*    d_v_xyz;   /* [v_cap][3] */
    double*   d_area;    /* [k_cap] */
    uint32_t* d_status;  /* [1] device word, VM_FLAG_* OR-ed in */
} vm_hulls_out;

/* Asynchronous; d_work as for vm_ransac_planes (the same buffer may be
 * reused: the calls are ordered on the stream). */
vm_status vm_hulls(const vm_clusters* cl, const vm_planes* planes, vm_hulls_out* out,
                   void* d_work, size_t work_bytes, void* stream);

/* ---- planes and polygons in one persistent launch ---------------------- */
/* Sec. III-C (a)-(c) and "Boundary polygon generation" for every cluster of
 * `cl`, run cluster-parallel as one persistent launch over a device work
 * queue (the batched form for thousands of clusters of very uneven size):
 * clusters sorted by size, largest first, are cut into (point tile,
 * hypothesis chunk) items; each item's integer counts go to their own slot;
 * the workgroup that completes a cluster's last item selects its best
 * hypothesis, lists its inliers and builds its polygon.  The outputs --
 * planes (including the optional d_counts / d_hyp), inlier CSR, polygons,
 * areas, status flags -- are bit-identical to vm_ransac_planes followed by
 * vm_hulls, for every work split (vm_fused_config).  d_work: at least
 * vm_workspace_bytes(min(cl->k_cap, planes->k_cap, hulls->k_cap), cl->n_cap,
 * params->n_hyp) bytes.  That cluster bound must be at most 65536
 * (VM_E_CAPACITY otherwise).  Asynchronous. */
vm_status vm_planes_hulls(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* planes,
                          vm_hulls_out* hulls, void* d_work, size_t work_bytes, void* stream);

/* Work split of vm_planes_hulls.  Every valid setting gives identical
 * results; only the speed differs. */
typedef struct {
    uint32_t hyp_chunk;      /* hypotheses per work item: a multiple of 64, 64..512; default 512 */
    uint32_t small_max;      /* clusters of at most this many points are counted with the lanes over the
                                hypotheses (one item per chunk), larger ones in 4096-point tiles; 0..256,
                                default 0 (every cluster in tiles) */
    uint32_t groups_per_cu;  /* persistent workgroups per compute unit, 1..8; default 5 */
    uint32_t reserved;       /* must be 0 */
} vm_fused_config;

/* The process-wide split (NULL: the defaults), used by vm_planes_hulls
 * calls whose shape has no autotuned entry; VM_E_ARG if a field is out of
 * range (nothing changes then). */
vm_status vm_set_fused_config(const vm_fused_config* cfg);
vm_status vm_get_fused_config(vm_fused_config* out);

/* Time vm_planes_hulls on this workload under candidate splits (one field
 * at a time from the current setting, `reps` calls each, 1..16), keep the
 * fastest for this call's shape bucket (log2 of the cluster bound, of n_cap
 * and of n_hyp; later calls in the bucket use it) and return it in *best.
 * Synchronises `stream`; the outputs hold the last call's (identical)
 * results.  VM_E_STATE while capturing.  vm_set_fused_config(NULL) also
 * clears the per-shape entries. */
vm_status vm_autotune_fused(const vm_clusters* cl, const vm_ransac_params* params, vm_planes* planes,
                            vm_hulls_out* hulls, void* d_work, size_t work_bytes, void* stream, uint32_t reps,
                            vm_fused_config* best);

/* Several cluster sets -- e.g. the clusters of several robots' maps, one
 * frame each -- in one sequence of launches (the served form's continuous
 * batching): the sets are merged into one cluster list in d_work (at most
 * k_cap clusters, 1..65536, and n_cap points in all), the two-pass kernels
 * of vm_ransac_planes and vm_hulls run once over the merged list (their
 * tiled passes spread a very large cluster over the chip), set i's clusters use
 * RNG counter word frames[i] (params->frame and params->d_frame are not
 * used), and set i's results go to planes[i] / hulls[i] exactly as
 * vm_planes_hulls on that set alone with params->frame = frames[i] would
 * write them (same capacity rules per set).  A set that no longer fits the
 * merged bounds (in set order) contributes no clusters and gets
 * VM_FLAG_CLUSTERS_CAP in both its status words.  n: 1..16 sets, whose
 * outputs must not overlap.  d_work: vm_multi_workspace_bytes(k_cap, n_cap,
 * params->n_hyp) bytes.  Asynchronous. */
vm_status vm_planes_hulls_multi(uint32_t n, const vm_clusters* sets, const uint32_t* frames,
                                const vm_ransac_params* params, vm_planes* planes, vm_hulls_out* hulls, uint32_t k_cap,
                                uint32_t n_cap, void* d_work, size_t work_bytes, void* stream);
size_t vm_multi_workspace_bytes(uint32_t k_cap, uint32_t n_cap, uint32_t n_hyp);

/* ---- one frame (Sec. III-A overview) ------------------------------------ */
typedef struct {
    uint32_t         min_cluster;   /* clusters below this many voxels are dropped (30) */
    uint32_t         flags;         /* VM_SEG_* bits; others must be 0 */
    vm_ransac_params ransac;
} vm_seg_params;

#define VM_SEG_CLEAR_RAYS 0x1u   /* vm_clear_rays of the frame before its vm_insert */

/* vm_insert of the frame (after vm_clear_rays of it when params->flags has
 * VM_SEG_CLEAR_RAYS), then vm_ccl, vm_ransac_planes and vm_hulls over the
 * whole accumulated map, using the map's own workspace.  Outputs as for the
 * individual calls; d_labels and clusters_out may be NULL.  Asynchronous:
 * nothing waits for the host. */
vm_status vm_segment_frame(vm_map map, const float* d_xyz, int64_t n, const vm_pose* pose,
                           const vm_seg_params* params, vm_planes* planes, vm_hulls_out* hulls,
                           uint32_t* d_labels, vm_clusters* clusters_out, void* stream);

/* vm_segment_frame with vm_ccl_steppable in place of vm_ccl: the paper's
 * full Sec. III-C path (classification, gated clustering, planes, polygons). */
vm_status vm_segment_frame_steppable(vm_map map, const float* d_xyz, int64_t n, const vm_pose* pose,
                                     const vm_seg_params* params, const vm_step_params* sp, vm_planes* planes,
                                     vm_hulls_out* hulls, uint32_t* d_labels, vm_clusters* clusters_out,
                                     void* stream);

/* ---- graph capture and replay ------------------------------------------- */
/* Record the library calls enqueued on `stream` between vm_capture_begin and
 * vm_capture_end into an executable HIP graph instead of running them
 * (hipStreamBeginCapture / hipGraphInstantiate).  Every argument of the
 * captured calls is frozen (pointers, sizes, poses, parameters); only the
 * contents of device buffers may change between replays (new points in the
 * same buffer, a device frame counter via vm_ransac_params.d_frame).  Calls
 * that would have to allocate or synchronise (a first vm_segment_frame on a
 * map, vm_map_stats, vm_map_export) return VM_E_STATE while capturing; stage
 * timing is skipped inside captures.  vm_graph_launch enqueues one replay on
 * `stream`; replays of one graph must not overlap. */
typedef struct vm_graph_s* vm_graph;
vm_status vm_capture_begin(void* stream);
vm_status vm_capture_end(void* stream, vm_graph* out);
vm_status vm_graph_launch(vm_graph graph, void* stream);
vm_status vm_graph_destroy(vm_graph graph);

/* ---- per-stage timing ---------------------------------------------------- */
/* When enabled, every stage kernel of the library is bracketed by HIP events
 * recorded on the stream it runs on; vm_stage_times synchronises each
 * recorded event and returns accumulated milliseconds and launch counts per
 * stage (index = VM_STAGE_*), then resets them.  Costs an event pair per
 * launch, so leave it off outside measurements. */
#define VM_STAGE_INSERT      0   /* voxelise + sort + slot updates (or per-point atomics) */
#define VM_STAGE_RANK        1   /* occupancy ranks and the sorted occupied keys */
#define VM_STAGE_CCL         2   /* in-tile labelling (one kernel) */
#define VM_STAGE_CCL_LINK    3   /* cross-tile hooks + flatten */
#define VM_STAGE_GROUP       4   /* sizes, cluster ids, sort, CSR gather */
#define VM_STAGE_HYPOTHESES  5   /* validation, tile list, hypotheses */
#define VM_STAGE_COUNT       6   /* inlier counting (one kernel) */
#define VM_STAGE_SELECT      7   /* best hypothesis, inlier CSR */
#define VM_STAGE_HULL        8   /* polygons */
#define VM_STAGE_CLEAR       9   /* ray casting and voxel clearing */
#define VM_STAGE_N           10
vm_status vm_set_stage_timing(int32_t enable);
vm_status vm_stage_times(double* ms_out, uint64_t* launches_out, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* VM_H */

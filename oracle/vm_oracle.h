/*
 * vm_oracle.h -- slow, plain CPU reference of the voxel-map plane-segmentation
 * path.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * benchmark's CPU-baseline leg call it; the product path never does.
 *
 * It shares no code, header, table or constant generator with the HIP
 * library.  Every function computes the plain definition of its step
 * (arithmetic mean, connected components, argmax of inlier counts, convex
 * hull) or, for the randomised RANSAC step, the algorithm's own steps in the
 * paper's order.  Numeric conventions: IEEE binary32/binary64 with
 * round-to-nearest-even, no contraction (built with -ffp-contract=off), every
 * fused multiply-add written out as fma()/fmaf().
 */
#ifndef VM_ORACLE_H
#define VM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VO_NO_KEY 0xFFFFFFFFu

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): one block. */
void vo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Sec. III-C (a): the three distinct point indices in [0, n) that hypothesis
 * h of cluster `tag` in frame `frame` samples (n >= 3). */
void vo_draw3(uint64_t seed, uint64_t tag, uint64_t frame, uint64_t h, uint64_t n, uint64_t out[3]);

/* Sec. III-B "Voxel information update", first step: transform each sensor
 * point by map_from_sensor (R row-major, t) and voxelise it.  Per point i:
 *   key[i]  = x + NX*(y + NY*z) of the voxel, or VO_NO_KEY if the point is
 *             non-finite or outside the grid;
 *   frac[3i..3i+2] = offset inside the voxel in units of s/2^20.
 * Returns the number of kept points. */
int64_t vo_voxelize(const float* xyz, int64_t n, const double R[9], const double t[3],
                    const double origin[3], double voxel_size, const int32_t dims[3],
                    uint32_t* key, uint64_t* frac);

/* Eq. (1): accumulate voxelised points into a map held as arrays sorted by
 * key (count and integer offset sums per voxel).  The input map arrays
 * (n_in entries) and the output arrays (capacity out_cap) must not alias.
 * Returns the new number of occupied voxels, or -1 if out_cap is too small. */
int64_t vo_map_accumulate(const uint32_t* in_key, const uint32_t* in_cnt, const uint64_t* in_sum,
                          int64_t n_in, const uint32_t* pt_key, const uint64_t* pt_frac,
                          int64_t n_pts, uint32_t* out_key, uint32_t* out_cnt, uint64_t* out_sum,
                          int64_t out_cap);

/* Eq. (1) closed form: the voxel's mean position, one float32 xyz per voxel. */
void vo_voxel_mean(const uint32_t* key, const uint32_t* cnt, const uint64_t* sum, int64_t n,
                   const double origin[3], double voxel_size, const int32_t dims[3], float* mu);

/* Alg. 1 fixed point: label[i] = smallest key in the 26-connected component of
 * occupied voxel i.  keys must be strictly ascending.  Breadth-first search
 * from each unvisited voxel in ascending key order.  Returns the number of
 * components, or -1 on allocation failure. */
int64_t vo_ccl26(const uint32_t* keys, int64_t n, const int32_t dims[3], uint32_t* label);

/* Sec. III-C "Multi-plane estimation" (a)-(c) for one cluster of n points in
 * canonical order.  counts[h] = inliers of hypothesis h (-1: degenerate),
 * hyp[4h..4h+3] = its float32 plane (nx,ny,nz,d).  best = [nx,ny,nz,d] of the
 * winning hypothesis; inlier_idx lists its inliers (ascending local indices).
 * Returns the best hypothesis index, or -1 if every hypothesis is degenerate
 * (or n < 3). *n_inliers receives the inlier count (0 if none). */
int32_t vo_ransac(const float* x, const float* y, const float* z, int64_t n,
                  uint32_t n_hyp, float eps, uint64_t seed, uint64_t tag, uint64_t frame,
                  int32_t* counts, float* hyp, float best[4], uint32_t* inlier_idx,
                  int64_t* n_inliers);

/* Sec. III-C "Boundary polygon generation": 2D convex hull of m points lying
 * near the plane (nx,ny,nz,d).  hull_idx receives indices into the m points,
 * counter-clockwise from the lexicographically smallest (u,v); hull_xyz the
 * vertices projected onto the plane; *area the polygon area (m^2, 0 when the
 * hull has fewer than 3 vertices).  Returns the vertex count, or -1 on
 * allocation failure.  Buffers must hold m entries. */
int64_t vo_hull(const float* x, const float* y, const float* z, int64_t m, const float plane[4],
                uint32_t* hull_idx, float* hull_xyz, double* area);

/* The in-plane 2D coordinates used by vo_hull (exposed for tests). */
void vo_hull_project(const float* x, const float* y, const float* z, int64_t m,
                     const float plane[4], double* u_out, double* v_out);

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (fp64): A is
 * diagonalised in place, V receives the eigenvectors as columns. */
void vo_jacobi3(double A[3][3], double V[3][3]);

/* Sec. III-C "Steppable point classification", Eq. (3)-(4).  For each of the
 * n occupied voxels (keys strictly ascending, means mu float32 xyz): the
 * neighbour points are the means of the occupied voxels at most `radius`
 * cells away on every axis (itself included, visited in ascending key
 * order), N their number (n_nb, optional); the normal is the unit eigenvector
 * of the smallest eigenvalue of their scatter matrix about their mean (fp64,
 * vo_jacobi3), oriented to +z (ties +y, +x), rounded to float32;
 * steppable = N >= n_th and n_z >= cos_th.  radius 1..2. */
void vo_classify(const uint32_t* keys, const float* mu, int64_t n, const int32_t dims[3], int32_t radius,
                 uint32_t n_th, double cos_th, float* normal, uint8_t* steppable, uint32_t* n_nb);

/* Alg. 1 with its distance and normal-angle gates, to its fixed point:
 * steppable 26-neighbours i, j are adjacent when |mu_i - mu_j|^2 < d_th^2 and
 * n_i . n_j > cos_th (float32 normals, fp64 arithmetic); label = smallest key
 * of the component, VO_NO_KEY for voxels that are not steppable.  Returns the
 * number of components, -1 on allocation failure. */
int64_t vo_ccl_gated(const uint32_t* keys, const float* mu, const float* normal, const uint8_t* steppable,
                     int64_t n, const int32_t dims[3], double d_th, double cos_th, uint32_t* label);

/* Sec. III-B "Voxel information clearing": the voxels of the ray from voxel a
 * to voxel b on the 3D Bresenham line (largest extent drives, ties x, y, z),
 * a included, b excluded, cut where it leaves the grid; up to cap xyz
 * triples in out; returns their number. */
int64_t vo_ray_voxels(const int64_t a[3], const int64_t b[3], const int32_t dims[3], int64_t* out, int64_t cap);

/* Eq. (2) for one frame (pose R, t; the sensor at t, inside the grid):
 * occupied voxels on the ray of any of the frame's points and holding none
 * of them are removed from the map arrays (filtered in place, keys stay
 * ascending).  Returns the new voxel count, -1 on allocation failure or a
 * sensor outside the grid. */
int64_t vo_clear_rays(uint32_t* key, uint32_t* cnt, uint64_t* sum, int64_t n, const float* xyz, int64_t npts,
                      const double R[9], const double t[3], const double origin[3], double voxel_size,
                      const int32_t dims[3]);

#ifdef __cplusplus
}
#endif
#endif

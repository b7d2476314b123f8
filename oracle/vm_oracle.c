/*
 * vm_oracle.c -- plain CPU reference for the voxel-map plane-segmentation path
 * (Niijima et al., "Real-time Multi-Plane Segmentation Based on GPU
 * Accelerated High-Resolution 3D Voxel Mapping for Legged Robot Locomotion").
 *
 * TEST INFRASTRUCTURE ONLY.  Used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; the library never links or calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math, no FTZ).
 * Every fused multiply-add below is written as fma()/fmaf(); every other
 * operation is a single correctly rounded IEEE operation, evaluated in the
 * order written.
 */
#include "vm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Counter-based RNG.  The paper gives every RANSAC thread its own random    */
/* state (Sec. III-C (a)); a counter-based generator gives each (hypothesis, */
/* cluster, frame) its own stream without any state.  Philox4x64-10 as       */
/* published by Salmon et al. (SC'11): 10 rounds of two 64x64->128 products  */
/* with a Weyl-sequence key schedule.                                        */
/* ------------------------------------------------------------------------ */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void vo_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, &hi0, &lo0);
        mulhilo64(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-B, voxel information update: transform + voxelise.              */
/* Fixed point: the position inside the grid is floor((p - o) * 2^20 / s);   */
/* its top bits are the voxel index, the low 20 bits the in-voxel offset.    */
/* ------------------------------------------------------------------------ */
int64_t vo_voxelize(const float* xyz, int64_t n, const double R[9], const double t[3],
                    const double origin[3], double voxel_size, const int32_t dims[3],
                    uint32_t* key, uint64_t* frac)
{
    const double inv = 1048576.0 / voxel_size;
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double px = (double)xyz[3 * i + 0];
        const double py = (double)xyz[3 * i + 1];
        const double pz = (double)xyz[3 * i + 2];
        double w[3];
        for (int a = 0; a < 3; ++a)
            w[a] = fma(R[3 * a + 2], pz, fma(R[3 * a + 1], py, fma(R[3 * a + 0], px, t[a])));
        int64_t q[3];
        int ok = 1;
        for (int a = 0; a < 3; ++a) {
            const double f = floor((w[a] - origin[a]) * inv);
            /* also rejects NaN: every comparison with NaN is false */
            if (!(f >= 0.0 && f < (double)dims[a] * 1048576.0)) { ok = 0; break; }
            q[a] = (int64_t)f;
        }
        if (!ok) {
            key[i] = VO_NO_KEY;
            frac[3 * i] = frac[3 * i + 1] = frac[3 * i + 2] = 0;
            continue;
        }
        const uint64_t ix = (uint64_t)(q[0] >> 20), iy = (uint64_t)(q[1] >> 20), iz = (uint64_t)(q[2] >> 20);
        key[i] = (uint32_t)(ix + (uint64_t)dims[0] * (iy + (uint64_t)dims[1] * iz));
        for (int a = 0; a < 3; ++a) frac[3 * i + a] = (uint64_t)(q[a] & 0xFFFFF);
        ++kept;
    }
    return kept;
}

typedef struct { uint32_t key; int64_t idx; } vo_kidx;

static int cmp_kidx(const void* pa, const void* pb)
{
    const vo_kidx* a = (const vo_kidx*)pa;
    const vo_kidx* b = (const vo_kidx*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

/* Eq. (1): c <- c + 1 and mu <- (c mu + p)/(c + 1).  Unrolled, mu is the
 * arithmetic mean of the voxel's points; it is kept exactly as the integer
 * sum of the fixed-point offsets, so the result does not depend on the order
 * in which points arrive. */
int64_t vo_map_accumulate(const uint32_t* in_key, const uint32_t* in_cnt, const uint64_t* in_sum,
                          int64_t n_in, const uint32_t* pt_key, const uint64_t* pt_frac,
                          int64_t n_pts, uint32_t* out_key, uint32_t* out_cnt, uint64_t* out_sum,
                          int64_t out_cap)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n_pts; ++i) m += pt_key[i] != VO_NO_KEY;
    vo_kidx* s = (vo_kidx*)malloc((size_t)(m > 0 ? m : 1) * sizeof(vo_kidx));
    if (!s) return -1;
    m = 0;
    for (int64_t i = 0; i < n_pts; ++i)
        if (pt_key[i] != VO_NO_KEY) { s[m].key = pt_key[i]; s[m].idx = i; ++m; }
    qsort(s, (size_t)m, sizeof(vo_kidx), cmp_kidx);

    int64_t a = 0, b = 0, o = 0;
    while (a < n_in || b < m) {
        uint32_t k;
        if (b >= m || (a < n_in && in_key[a] <= s[b].key)) k = in_key[a];
        else k = s[b].key;
        if (o >= out_cap) { free(s); return -1; }
        uint32_t c = 0;
        uint64_t sx = 0, sy = 0, sz = 0;
        if (a < n_in && in_key[a] == k) {
            c = in_cnt[a];
            sx = in_sum[3 * a]; sy = in_sum[3 * a + 1]; sz = in_sum[3 * a + 2];
            ++a;
        }
        while (b < m && s[b].key == k) {
            const int64_t i = s[b].idx;
            c += 1;
            sx += pt_frac[3 * i]; sy += pt_frac[3 * i + 1]; sz += pt_frac[3 * i + 2];
            ++b;
        }
        out_key[o] = k; out_cnt[o] = c;
        out_sum[3 * o] = sx; out_sum[3 * o + 1] = sy; out_sum[3 * o + 2] = sz;
        ++o;
    }
    free(s);
    return o;
}

void vo_voxel_mean(const uint32_t* key, const uint32_t* cnt, const uint64_t* sum, int64_t n,
                   const double origin[3], double voxel_size, const int32_t dims[3], float* mu)
{
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t k = key[i];
        const uint64_t idx[3] = { k % (uint64_t)dims[0], (k / (uint64_t)dims[0]) % (uint64_t)dims[1],
                                  k / ((uint64_t)dims[0] * (uint64_t)dims[1]) };
        for (int a = 0; a < 3; ++a) {
            const uint64_t mq = sum[3 * i + a] / (uint64_t)cnt[i];   /* mean offset, truncated */
            const double cell = (double)idx[a] + (double)mq * 0x1p-20;
            mu[3 * i + a] = (float)fma(cell, voxel_size, origin[a]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Alg. 1: min-label propagation over the adjacency graph converges to the    */
/* smallest initial label of each connected component.  With initial label = */
/* voxel key and 26-neighbour adjacency, that fixed point is computed here   */
/* directly by breadth-first search.                                          */
/* ------------------------------------------------------------------------ */
int64_t vo_ccl26(const uint32_t* keys, int64_t n, const int32_t dims[3], uint32_t* label)
{
    const int64_t NX = dims[0], NY = dims[1], NZ = dims[2];
    const int64_t ncell = NX * NY * NZ;
    int32_t* where = (int32_t*)malloc((size_t)ncell * sizeof(int32_t));
    int64_t* queue = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!where || !queue) { free(where); free(queue); return -1; }
    memset(where, 0xFF, (size_t)ncell * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i) { where[keys[i]] = (int32_t)i; label[i] = VO_NO_KEY; }
    int64_t ncomp = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (label[s] != VO_NO_KEY) continue;
        /* every voxel with a smaller key is already labelled, so keys[s] is the
         * smallest key of its component */
        const uint32_t lab = keys[s];
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = lab;
        while (head < tail) {
            const int64_t v = queue[head++];
            const int64_t k = keys[v];
            const int64_t x = k % NX, y = (k / NX) % NY, z = k / (NX * NY);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy && !dz) continue;
                        const int64_t xx = x + dx, yy = y + dy, zz = z + dz;
                        if (xx < 0 || yy < 0 || zz < 0 || xx >= NX || yy >= NY || zz >= NZ) continue;
                        const int32_t u = where[xx + NX * (yy + NY * zz)];
                        if (u < 0 || label[u] != VO_NO_KEY) continue;
                        label[u] = lab;
                        queue[tail++] = u;
                    }
        }
        ++ncomp;
    }
    free(where);
    free(queue);
    return ncomp;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-C, cluster-parallel RANSAC, run one cluster at a time.           */
/* ------------------------------------------------------------------------ */

/* Three distinct indices in [0, n) from one Philox block: a uniform, then b
 * uniform over the n-1 others, then c uniform over the n-2 others. */
static void draw3(const uint64_t r[4], uint64_t n, uint64_t* a, uint64_t* b, uint64_t* c)
{
    const uint64_t u0 = r[0] >> 32, u1 = r[1] >> 32, u2 = r[2] >> 32;
    uint64_t ia = (u0 * n) >> 32;
    uint64_t ib = (u1 * (n - 1)) >> 32;
    if (ib >= ia) ib += 1;
    uint64_t ic = (u2 * (n - 2)) >> 32;
    const uint64_t lo = ia < ib ? ia : ib, hi = ia < ib ? ib : ia;
    if (ic >= lo) ic += 1;
    if (ic >= hi) ic += 1;
    *a = ia; *b = ib; *c = ic;
}

void vo_draw3(uint64_t seed, uint64_t tag, uint64_t frame, uint64_t h, uint64_t n, uint64_t out[3])
{
    const uint64_t key[2] = { seed, 0 };
    const uint64_t ctr[4] = { h, tag, frame, 0 };
    uint64_t r[4];
    vo_philox4x64_10(ctr, key, r);
    draw3(r, n, &out[0], &out[1], &out[2]);
}

/* (a) plane through three points; returns 0 for a degenerate triple. */
static int plane3(const float* x, const float* y, const float* z, uint64_t a, uint64_t b, uint64_t c,
                  float out[4])
{
    const double ax = x[a], ay = y[a], az = z[a];
    const double e1x = (double)x[b] - ax, e1y = (double)y[b] - ay, e1z = (double)z[b] - az;
    const double e2x = (double)x[c] - ax, e2y = (double)y[c] - ay, e2z = (double)z[c] - az;
    double nx = e1y * e2z - e1z * e2y;
    double ny = e1z * e2x - e1x * e2z;
    double nz = e1x * e2y - e1y * e2x;
    const double nn = nx * nx + ny * ny + nz * nz;
    if (!(nn >= 1e-24)) return 0;
    const double inv = 1.0 / sqrt(nn);
    nx = nx * inv; ny = ny * inv; nz = nz * inv;
    /* one orientation per plane: z-component positive, ties broken by y then x */
    if (nz < 0.0 || (nz == 0.0 && (ny < 0.0 || (ny == 0.0 && nx < 0.0)))) {
        nx = -nx; ny = -ny; nz = -nz;
    }
    const double d = -(nx * ax + ny * ay + nz * az);
    out[0] = (float)nx; out[1] = (float)ny; out[2] = (float)nz; out[3] = (float)d;
    return 1;
}

/* (b) point-to-plane distance below the threshold, in float32. */
static int is_inlier(const float p[4], float px, float py, float pz, float eps)
{
    return fabsf(fmaf(p[2], pz, fmaf(p[1], py, fmaf(p[0], px, p[3])))) < eps;
}

int32_t vo_ransac(const float* x, const float* y, const float* z, int64_t n,
                  uint32_t n_hyp, float eps, uint64_t seed, uint64_t tag, uint64_t frame,
                  int32_t* counts, float* hyp, float best[4], uint32_t* inlier_idx,
                  int64_t* n_inliers)
{
    const uint64_t key[2] = { seed, 0 };
    int32_t hbest = -1;
    int64_t cbest = -1;
    best[0] = best[1] = best[2] = best[3] = 0.0f;
    *n_inliers = 0;
    for (uint32_t h = 0; h < n_hyp; ++h) {
        float pl[4] = { 0.0f, 0.0f, 0.0f, 0.0f };
        int64_t cnt = -1;
        if (n >= 3) {
            const uint64_t ctr[4] = { h, tag, frame, 0 };
            uint64_t r[4], a, b, c;
            vo_philox4x64_10(ctr, key, r);
            draw3(r, (uint64_t)n, &a, &b, &c);
            if (plane3(x, y, z, a, b, c, pl)) {
                cnt = 0;
                for (int64_t j = 0; j < n; ++j) cnt += is_inlier(pl, x[j], y[j], z[j], eps);
            }
        }
        if (counts) counts[h] = (int32_t)cnt;
        if (hyp) memcpy(hyp + 4 * (size_t)h, pl, sizeof pl);
        /* (c) the maximum count wins; the first hypothesis wins a tie */
        if (cnt > cbest) { cbest = cnt; hbest = (int32_t)h; memcpy(best, pl, sizeof pl); }
    }
    if (hbest < 0) return -1;
    int64_t m = 0;
    for (int64_t j = 0; j < n; ++j)
        if (is_inlier(best, x[j], y[j], z[j], eps)) {
            if (inlier_idx) inlier_idx[m] = (uint32_t)j;
            ++m;
        }
    *n_inliers = m;
    return hbest;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-C, boundary polygon: convex hull of the inliers in the plane.    */
/* ------------------------------------------------------------------------ */
static void plane_basis(const float plane[4], double u[3], double v[3], double nrm[3])
{
    nrm[0] = plane[0]; nrm[1] = plane[1]; nrm[2] = plane[2];
    double a[3] = { 0.0, 0.0, 0.0 };
    if (fabs(nrm[0]) < 0.9) a[0] = 1.0; else a[1] = 1.0;
    double c[3] = { a[1] * nrm[2] - a[2] * nrm[1], a[2] * nrm[0] - a[0] * nrm[2], a[0] * nrm[1] - a[1] * nrm[0] };
    const double inv = 1.0 / sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    u[0] = c[0] * inv; u[1] = c[1] * inv; u[2] = c[2] * inv;
    v[0] = nrm[1] * u[2] - nrm[2] * u[1];
    v[1] = nrm[2] * u[0] - nrm[0] * u[2];
    v[2] = nrm[0] * u[1] - nrm[1] * u[0];
}

void vo_hull_project(const float* x, const float* y, const float* z, int64_t m,
                     const float plane[4], double* u_out, double* v_out)
{
    double u[3], v[3], nrm[3];
    plane_basis(plane, u, v, nrm);
    if (m <= 0) return;
    const double ox = x[0], oy = y[0], oz = z[0];
    for (int64_t i = 0; i < m; ++i) {
        const double dx = (double)x[i] - ox, dy = (double)y[i] - oy, dz = (double)z[i] - oz;
        u_out[i] = u[0] * dx + u[1] * dy + u[2] * dz;
        v_out[i] = v[0] * dx + v[1] * dy + v[2] * dz;
    }
}

typedef struct { double u, v; int64_t i; } vo_p2;

static int cmp_p2(const void* pa, const void* pb)
{
    const vo_p2* a = (const vo_p2*)pa;
    const vo_p2* b = (const vo_p2*)pb;
    if (a->u != b->u) return a->u < b->u ? -1 : 1;
    if (a->v != b->v) return a->v < b->v ? -1 : 1;
    return (a->i > b->i) - (a->i < b->i);
}

static double cross3(const vo_p2* o, const vo_p2* a, const vo_p2* b)
{
    return (a->u - o->u) * (b->v - o->v) - (a->v - o->v) * (b->u - o->u);
}

/* Andrew's monotone chain: lower chain left to right, upper chain right to
 * left, dropping every point that does not make a strict left turn. */
int64_t vo_hull(const float* x, const float* y, const float* z, int64_t m, const float plane[4],
                uint32_t* hull_idx, float* hull_xyz, double* area)
{
    *area = 0.0;
    if (m <= 0) return 0;
    double* uu = (double*)malloc((size_t)m * sizeof(double));
    double* vv = (double*)malloc((size_t)m * sizeof(double));
    vo_p2* p = (vo_p2*)malloc((size_t)m * sizeof(vo_p2));
    int64_t* st = (int64_t*)malloc((size_t)(2 * m + 1) * sizeof(int64_t));
    if (!uu || !vv || !p || !st) { free(uu); free(vv); free(p); free(st); return -1; }
    vo_hull_project(x, y, z, m, plane, uu, vv);
    for (int64_t i = 0; i < m; ++i) { p[i].u = uu[i]; p[i].v = vv[i]; p[i].i = i; }
    qsort(p, (size_t)m, sizeof(vo_p2), cmp_p2);

    int64_t h = 0;
    if (m == 1) {
        st[h++] = 0;
    } else {
        for (int64_t i = 0; i < m; ++i) {                      /* lower chain */
            while (h >= 2 && cross3(&p[st[h - 2]], &p[st[h - 1]], &p[i]) <= 0.0) --h;
            st[h++] = i;
        }
        const int64_t lower = h + 1;
        for (int64_t i = m - 2; i >= 0; --i) {                 /* upper chain */
            while (h >= lower && cross3(&p[st[h - 2]], &p[st[h - 1]], &p[i]) <= 0.0) --h;
            st[h++] = i;
        }
        --h;                                                  /* last point repeats the first */
    }
    for (int64_t k = 0; k < h; ++k) hull_idx[k] = (uint32_t)p[st[k]].i;
    if (h >= 3) {
        double s = 0.0;
        for (int64_t k = 0; k < h; ++k) {
            const vo_p2* a = &p[st[k]];
            const vo_p2* b = &p[st[(k + 1) % h]];
            s = s + (a->u * b->v - b->u * a->v);
        }
        *area = 0.5 * s;
    }
    const double nx = plane[0], ny = plane[1], nz = plane[2], d = plane[3];
    for (int64_t k = 0; k < h; ++k) {
        const int64_t i = hull_idx[k];
        const double px = x[i], py = y[i], pz = z[i];
        const double dist = nx * px + ny * py + nz * pz + d;
        hull_xyz[3 * k + 0] = (float)(px - dist * nx);
        hull_xyz[3 * k + 1] = (float)(py - dist * ny);
        hull_xyz[3 * k + 2] = (float)(pz - dist * nz);
    }
    free(uu); free(vv); free(p); free(st);
    return h;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-C "Steppable point classification", Eq. (3) and Eq. (4).       */
/* ------------------------------------------------------------------------ */

/* index of key k among the n ascending keys, or -1 */
static int64_t find_key(const uint32_t* keys, int64_t n, uint32_t k)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && keys[lo] == k) ? lo : -1;
}

/* Cyclic Jacobi method for a symmetric 3x3 matrix (Golub & Van Loan): rotations
 * in the planes (0,1), (0,2), (1,2) in turn, each annihilating one
 * off-diagonal entry with the symmetric Schur rotation, sweeps repeated until
 * the off-diagonal part is negligible against the diagonal (at most 16).  On
 * return A is (nearly) diagonal and the columns of V are the eigenvectors. */
void vo_jacobi3(double A[3][3], double V[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    static const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 16; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-30 * dia) break;
        for (int r = 0; r < 3; ++r) {
            const int p = P[r], q = Q[r];
            const double apq = A[p][q];
            if (apq == 0.0) continue;
            /* the rotation angle: cot(2 theta) = tau, t = tan(theta), the smaller root */
            const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t);
            const double s = t * c;
            /* A <- J^T A J and V <- V J, J the identity but for
             * J[p][p] = c, J[p][q] = s, J[q][p] = -s, J[q][q] = c */
            for (int k = 0; k < 3; ++k) {
                const double akp = A[k][p], akq = A[k][q];
                A[k][p] = c * akp - s * akq;
                A[k][q] = s * akp + c * akq;
            }
            for (int k = 0; k < 3; ++k) {
                const double apk = A[p][k], aqk = A[q][k];
                A[p][k] = c * apk - s * aqk;
                A[q][k] = s * apk + c * aqk;
            }
            for (int k = 0; k < 3; ++k) {
                const double vkp = V[k][p], vkq = V[k][q];
                V[k][p] = c * vkp - s * vkq;
                V[k][q] = s * vkp + c * vkq;
            }
        }
    }
}

void vo_classify(const uint32_t* keys, const float* mu, int64_t n, const int32_t dims[3], int32_t radius,
                 uint32_t n_th, double cos_th, float* normal, uint8_t* steppable, uint32_t* n_nb)
{
    const int64_t NX = dims[0], NY = dims[1], NZ = dims[2];
    for (int64_t i = 0; i < n; ++i) {
        const int64_t k = keys[i];
        const int64_t x = k % NX, y = (k / NX) % NY, z = k / (NX * NY);
        /* the neighbour points, in ascending key order (i itself included) */
        double px[125], py[125], pz[125];
        uint32_t cnt = 0;
        for (int dz = -radius; dz <= radius; ++dz)
            for (int dy = -radius; dy <= radius; ++dy)
                for (int dx = -radius; dx <= radius; ++dx) {
                    const int64_t xx = x + dx, yy = y + dy, zz = z + dz;
                    if (xx < 0 || yy < 0 || zz < 0 || xx >= NX || yy >= NY || zz >= NZ) continue;
                    const int64_t j = find_key(keys, n, (uint32_t)(xx + NX * (yy + NY * zz)));
                    if (j < 0) continue;
                    px[cnt] = mu[3 * j + 0];
                    py[cnt] = mu[3 * j + 1];
                    pz[cnt] = mu[3 * j + 2];
                    ++cnt;
                }
        /* their scatter matrix about their mean (the covariance up to a factor) */
        double mx = 0.0, my = 0.0, mz = 0.0;
        for (uint32_t a = 0; a < cnt; ++a) {
            mx += px[a];
            my += py[a];
            mz += pz[a];
        }
        mx /= (double)cnt;
        my /= (double)cnt;
        mz /= (double)cnt;
        double A[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        for (uint32_t a = 0; a < cnt; ++a) {
            const double ex = px[a] - mx, ey = py[a] - my, ez = pz[a] - mz;
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
        double V[3][3];
        vo_jacobi3(A, V);
        /* Eq. (3): the eigenvector of the smallest eigenvalue (first on ties),
         * unit length, oriented to +z (then +y, then +x) */
        int m = 0;
        for (int e = 1; e < 3; ++e)
            if (A[e][e] < A[m][m]) m = e;
        double nx = V[0][m], ny = V[1][m], nz = V[2][m];
        const double len = sqrt(nx * nx + ny * ny + nz * nz);
        nx /= len;
        ny /= len;
        nz /= len;
        if (nz < 0.0 || (nz == 0.0 && (ny < 0.0 || (ny == 0.0 && nx < 0.0)))) {
            nx = -nx;
            ny = -ny;
            nz = -nz;
        }
        normal[3 * i + 0] = (float)nx;
        normal[3 * i + 1] = (float)ny;
        normal[3 * i + 2] = (float)nz;
        /* Eq. (4): enough neighbours and a normal within theta_th of the vertical */
        steppable[i] = (cnt >= n_th && nz >= cos_th) ? 1 : 0;
        if (n_nb) n_nb[i] = cnt;
    }
}

/* Alg. 1 with its gates, to its fixed point: among steppable voxels, i and j
 * (26-neighbours) are adjacent when |mu_i - mu_j| < d_th and the angle
 * between their normals is below theta_th (n_i . n_j > cos_th); label[i] is
 * the smallest key of i's component, VO_NO_KEY for voxels that are not
 * steppable.  Breadth-first search from each unlabelled steppable voxel in
 * ascending key order.  Returns the number of components (-1: no memory). */
int64_t vo_ccl_gated(const uint32_t* keys, const float* mu, const float* normal, const uint8_t* steppable,
                     int64_t n, const int32_t dims[3], double d_th, double cos_th, uint32_t* label)
{
    const int64_t NX = dims[0], NY = dims[1], NZ = dims[2];
    int64_t* queue = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!queue) return -1;
    for (int64_t i = 0; i < n; ++i) label[i] = VO_NO_KEY;
    const double d2_th = d_th * d_th;
    int64_t ncomp = 0;
    for (int64_t s = 0; s < n; ++s) {
        if (!steppable[s] || label[s] != VO_NO_KEY) continue;
        const uint32_t lab = keys[s];
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = lab;
        while (head < tail) {
            const int64_t v = queue[head++];
            const int64_t k = keys[v];
            const int64_t x = k % NX, y = (k / NX) % NY, z = k / (NX * NY);
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy && !dz) continue;
                        const int64_t xx = x + dx, yy = y + dy, zz = z + dz;
                        if (xx < 0 || yy < 0 || zz < 0 || xx >= NX || yy >= NY || zz >= NZ) continue;
                        const int64_t u = find_key(keys, n, (uint32_t)(xx + NX * (yy + NY * zz)));
                        if (u < 0 || !steppable[u] || label[u] != VO_NO_KEY) continue;
                        const double ddx = (double)mu[3 * v] - (double)mu[3 * u];
                        const double ddy = (double)mu[3 * v + 1] - (double)mu[3 * u + 1];
                        const double ddz = (double)mu[3 * v + 2] - (double)mu[3 * u + 2];
                        if (!(ddx * ddx + ddy * ddy + ddz * ddz < d2_th)) continue;
                        const double dot = (double)normal[3 * v] * (double)normal[3 * u] +
                                           (double)normal[3 * v + 1] * (double)normal[3 * u + 1] +
                                           (double)normal[3 * v + 2] * (double)normal[3 * u + 2];
                        if (!(dot > cos_th)) continue;
                        label[u] = lab;
                        queue[tail++] = u;
                    }
        }
        ++ncomp;
    }
    free(queue);
    return ncomp;
}

/* ------------------------------------------------------------------------ */
/* Sec. III-B "Voxel information clearing", Eq. (2).                         */
/* ------------------------------------------------------------------------ */

/* floor(q / 2^20) of an integral fp64 value q */
static int64_t voxel_index(double q)
{
    const int64_t v = (int64_t)q;
    return v >= 0 ? v / 1048576 : -((-v + 1048575) / 1048576);
}

/* The voxels of a ray from voxel a to voxel b: the 3D Bresenham line (the
 * axis with the largest extent drives, x before y before z on ties; each
 * minor axis steps when its error term reaches zero), a included, b
 * excluded, cut where it leaves the grid.  Writes at most cap voxel
 * coordinates (xyz triples) and returns their number. */
int64_t vo_ray_voxels(const int64_t a[3], const int64_t b[3], const int32_t dims[3], int64_t* out, int64_t cap)
{
    int64_t p[3] = {a[0], a[1], a[2]};
    int64_t d[3], sgn[3];
    for (int k = 0; k < 3; ++k) {
        const int64_t v = b[k] - a[k];
        d[k] = v < 0 ? -v : v;
        sgn[k] = v < 0 ? -1 : 1;
    }
    int m = 0;                                   /* driving axis */
    if (d[1] > d[m]) m = 1;
    if (d[2] > d[m]) m = 2;
    const int u = (m + 1) % 3, w = (m + 2) % 3;  /* the minor axes */
    int64_t eu = 2 * d[u] - d[m], ew = 2 * d[w] - d[m];
    int64_t cnt = 0;
    for (int64_t step = 0; step < d[m]; ++step) {
        if (p[0] < 0 || p[1] < 0 || p[2] < 0 || p[0] >= dims[0] || p[1] >= dims[1] || p[2] >= dims[2]) break;
        if (cnt < cap) {
            out[3 * cnt + 0] = p[0];
            out[3 * cnt + 1] = p[1];
            out[3 * cnt + 2] = p[2];
        }
        ++cnt;
        if (eu >= 0) {
            p[u] += sgn[u];
            eu -= 2 * d[m];
        }
        if (ew >= 0) {
            p[w] += sgn[w];
            ew -= 2 * d[m];
        }
        eu += 2 * d[u];
        ew += 2 * d[w];
        p[m] += sgn[m];
    }
    return cnt;
}

/* Eq. (2) for one frame: every occupied voxel that a ray from the sensor
 * (the pose's translation t) to one of the frame's points passes through is
 * cleared, unless it holds one of the frame's points itself.  Rays run on
 * voxel indices, from the sensor's voxel to the point's voxel (the floor of
 * the fp64 transformed coordinates, as in vo_voxelize); points that are not
 * finite cast no ray.  The map arrays (keys ascending) are filtered in place;
 * returns the new occupied count, or -1 (no memory, or the sensor outside
 * the grid). */
int64_t vo_clear_rays(uint32_t* key, uint32_t* cnt, uint64_t* sum, int64_t n, const float* xyz, int64_t npts,
                      const double R[9], const double t[3], const double origin[3], double voxel_size,
                      const int32_t dims[3])
{
    const int64_t NX = dims[0], NY = dims[1], NZ = dims[2];
    const int64_t ncell = NX * NY * NZ;
    uint8_t* mark = (uint8_t*)calloc((size_t)ncell, 1);   /* 1: on a ray, 2: a point's own voxel */
    int64_t* path = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)(NX + NY + NZ + 3));
    if (!mark || !path) { free(mark); free(path); return -1; }
    /* voxel indices exactly as vo_voxelize finds them: the 2^-20-voxel
     * fixed-point coordinate, then its integer part (floor division) */
    const double inv_q = 1048576.0 / voxel_size;
    int64_t s[3];
    for (int k = 0; k < 3; ++k) s[k] = voxel_index(floor((t[k] - origin[k]) * inv_q));
    if (s[0] < 0 || s[1] < 0 || s[2] < 0 || s[0] >= NX || s[1] >= NY || s[2] >= NZ) {
        free(mark);
        free(path);
        return -1;
    }
    for (int64_t i = 0; i < npts; ++i) {
        const double px = xyz[3 * i], py = xyz[3 * i + 1], pz = xyz[3 * i + 2];
        const double w[3] = {fma(R[2], pz, fma(R[1], py, fma(R[0], px, t[0]))),
                             fma(R[5], pz, fma(R[4], py, fma(R[3], px, t[1]))),
                             fma(R[8], pz, fma(R[7], py, fma(R[6], px, t[2])))};
        if (!isfinite(w[0]) || !isfinite(w[1]) || !isfinite(w[2])) continue;
        int64_t e[3];
        int inside = 1;
        for (int k = 0; k < 3; ++k) {
            const double f = floor((w[k] - origin[k]) * inv_q);
            if (f < -1e15 || f > 1e15) { inside = -1; break; }   /* no ray to a point this far */
            e[k] = voxel_index(f);
            if (e[k] < 0 || e[k] >= dims[k]) inside = 0;
        }
        if (inside < 0) continue;
        if (inside) mark[e[0] + NX * (e[1] + NY * e[2])] = 2;
        const int64_t np = vo_ray_voxels(s, e, dims, path, NX + NY + NZ + 3);
        for (int64_t q = 0; q < np; ++q) {
            const int64_t c = path[3 * q] + NX * (path[3 * q + 1] + NY * path[3 * q + 2]);
            if (mark[c] == 0) mark[c] = 1;
        }
    }
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (mark[key[i]] == 1) continue;         /* cleared: on a ray, holding none of the frame's points */
        key[m] = key[i];
        cnt[m] = cnt[i];
        sum[3 * m + 0] = sum[3 * i + 0];
        sum[3 * m + 1] = sum[3 * i + 1];
        sum[3 * m + 2] = sum[3 * i + 2];
        ++m;
    }
    free(mark);
    free(path);
    return m;
}

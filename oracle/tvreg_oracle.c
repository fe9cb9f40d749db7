/*
 * FP64 CPU oracle for TV-regularised CT reconstruction -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It is written for obviousness, not speed: every
 * quantity follows its defining formula in the paper (section / equation /
 * algorithm cited at each function), in double precision, built with
 * -O2 -ffp-contract=off.  Where the paper is silent the reading taken is
 * stated at the function.  No code is shared with the HIP library.
 *
 * Geometry reading (the paper only says "system matrix", Sec. II-A, and
 * "forward mapping of the discretized image", Sec. IV-A):
 *   - unit voxels, volume centred at the origin; voxel (i,j,k) is the box
 *     [i - nx/2, i+1 - nx/2] x [j - ny/2, ...] x [k - nz/2, ...], stored at
 *     i + nx*(j + ny*k);
 *   - one ray per detector pixel centre; a_ij is the exact length of ray i
 *     inside voxel j (Siddon 1985), zero-length pieces dropped, cells
 *     half-open so a ray lying in a voxel face belongs to the higher index;
 *   - view angle theta, e_s = (cos, sin, 0), e_u = (-sin, cos, 0), e_v = z;
 *     pixel centre u = (col - (cols-1)/2) pitch_u, w = (row - (rows-1)/2) pitch_v;
 *     parallel beam: the line through u e_u + w e_v with direction e_s;
 *     cone beam: source R e_s, pixel at -(SDD - R) e_s + u e_u + w e_v;
 *   - parallel beam along given directions d (the paper's 3D parallel beam,
 *     Sec. IV-A): the line through u e_u + w e_v along d, with
 *     e_u = (e_z x d)/|e_z x d| (e_x if d is along z) and e_v = d x e_u.
 */
#include "tvreg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int32_t og_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Rays                                                                      */
/* ------------------------------------------------------------------------ */

void og_ray_endpoints(const og_geom *g, int32_t v, int32_t row, int32_t col,
                      double p0[3], double p1[3])
{
    double u = ((double)col - 0.5 * (double)(g->cols - 1)) * g->pitch_u;
    double w = ((double)row - 0.5 * (double)(g->rows - 1)) * g->pitch_v;
    if (g->cone == 2) {
        /* parallel rays along the view direction d (normalised); the
           detector plane passes through the origin with axes
           e_u = (e_z x d) / |e_z x d| (e_x when d runs along z) and
           e_v = d x e_u, which for d = (cos, sin, 0) are the axes of the
           parallel beam about z below */
        const double *q = g->dirs + 3 * (size_t)v;
        double nd = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
        double d[3] = {q[0] / nd, q[1] / nd, q[2] / nd};
        double eu[3], ev[3];
        double a = sqrt(d[0] * d[0] + d[1] * d[1]);
        if (a > 0.0) {
            eu[0] = -d[1] / a;
            eu[1] = d[0] / a;
            eu[2] = 0.0;
        } else {
            eu[0] = 1.0;
            eu[1] = 0.0;
            eu[2] = 0.0;
        }
        ev[0] = d[1] * eu[2] - d[2] * eu[1];
        ev[1] = d[2] * eu[0] - d[0] * eu[2];
        ev[2] = d[0] * eu[1] - d[1] * eu[0];
        double h = (double)(g->nx + g->ny + g->nz);
        for (int k = 0; k < 3; ++k) {
            double o = u * eu[k] + w * ev[k];
            p0[k] = o - h * d[k];
            p1[k] = o + h * d[k];
        }
        return;
    }
    double th = g->angles[v];
    double c = cos(th), s = sin(th);
    if (g->cone) {
        double R = g->src_to_centre, D = g->src_to_det;
        p0[0] = R * c;
        p0[1] = R * s;
        p0[2] = 0.0;
        p1[0] = -(D - R) * c - u * s;
        p1[1] = -(D - R) * s + u * c;
        p1[2] = w;
    } else {
        /* a segment long enough to contain the whole line's passage through
           the volume: the volume lies within radius |(nx,ny,nz)|/2 of the
           origin and the line's closest point to the origin is u e_u + w e_v */
        double h = (double)(g->nx + g->ny + g->nz);
        double ox = -u * s, oy = u * c, oz = w;
        p0[0] = ox - h * c;
        p0[1] = oy - h * s;
        p0[2] = oz;
        p1[0] = ox + h * c;
        p1[1] = oy + h * s;
        p1[2] = oz;
    }
}

/* ------------------------------------------------------------------------ */
/* Siddon's exact radiological path                                          */
/* ------------------------------------------------------------------------ */

/*
 * Segment p(a) = p0 + a (p1 - p0), a in [0, 1].  Computes every parameter
 * value at which the segment crosses a voxel plane inside the volume,
 * merges them (each axis's list is already sorted), and gives each
 * consecutive pair the length (a_{q+1} - a_q) |p1 - p0| in the voxel
 * containing the pair's midpoint.  Writes at most nx+ny+nz+2 entries;
 * `work` must hold 2*(nx+ny+nz+3) doubles.  Returns the entry count.
 */
int32_t og_siddon(const og_geom *g, const double p0[3], const double p1[3],
                  int32_t *idx, double *len, double *work)
{
    const int32_t n[3] = {g->nx, g->ny, g->nz};
    double lo[3], d[3];
    double amin = 0.0, amax = 1.0;
    for (int a = 0; a < 3; ++a) {
        lo[a] = -0.5 * (double)n[a];
        d[a] = p1[a] - p0[a];
    }
    for (int a = 0; a < 3; ++a) {
        double hi = lo[a] + (double)n[a];
        if (d[a] != 0.0) {
            double t0 = (lo[a] - p0[a]) / d[a];
            double t1 = (hi - p0[a]) / d[a];
            amin = fmax(amin, fmin(t0, t1));
            amax = fmin(amax, fmax(t0, t1));
        } else if (!(p0[a] >= lo[a] && p0[a] < hi)) {
            return 0;
        }
    }
    if (!(amax > amin))
        return 0;

    /* per-axis ascending crossing lists, then a three-way merge */
    int32_t total = g->nx + g->ny + g->nz + 3;
    double *lists[3];
    int32_t cnt[3] = {0, 0, 0};
    lists[0] = work;
    lists[1] = work + (g->nx + 1);
    lists[2] = lists[1] + (g->ny + 1);
    double *merged = work + total;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0)
            continue;
        for (int32_t q = 0; q <= n[a]; ++q) {
            int32_t i = d[a] > 0.0 ? q : n[a] - q; /* ascending in a */
            double al = (lo[a] + (double)i - p0[a]) / d[a];
            if (al > amin && al < amax)
                lists[a][cnt[a]++] = al;
        }
    }
    int32_t nm = 0, pos[3] = {0, 0, 0};
    merged[nm++] = amin;
    for (;;) {
        int best = -1;
        double bv = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (pos[a] < cnt[a] && (best < 0 || lists[a][pos[a]] < bv)) {
                best = a;
                bv = lists[a][pos[a]];
            }
        }
        if (best < 0)
            break;
        merged[nm++] = bv;
        pos[best]++;
    }
    merged[nm++] = amax;

    double raylen = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    int32_t k = 0;
    for (int32_t q = 0; q + 1 < nm; ++q) {
        double da = merged[q + 1] - merged[q];
        if (!(da > 0.0))
            continue; /* coincident crossings give no segment */
        double am = 0.5 * (merged[q] + merged[q + 1]);
        int32_t ii[3];
        int ok = 1;
        for (int a = 0; a < 3; ++a) {
            ii[a] = (int32_t)floor(p0[a] + am * d[a] - lo[a]);
            if (ii[a] < 0 || ii[a] >= n[a])
                ok = 0;
        }
        if (!ok)
            continue; /* cannot happen for a midpoint strictly inside */
        idx[k] = ii[0] + g->nx * (ii[1] + g->ny * ii[2]);
        len[k] = da * raylen;
        ++k;
    }
    return k;
}

/* Length of the segment p0->p1 inside the box [lo, hi) (slab method). */
double og_slab_length(const double p0[3], const double p1[3], const double lo[3],
                      const double hi[3])
{
    double amin = 0.0, amax = 1.0, d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double d = p1[a] - p0[a];
        d2 += d * d;
        if (d != 0.0) {
            double t0 = (lo[a] - p0[a]) / d;
            double t1 = (hi[a] - p0[a]) / d;
            amin = fmax(amin, fmin(t0, t1));
            amax = fmin(amax, fmax(t0, t1));
        } else if (!(p0[a] >= lo[a] && p0[a] < hi[a])) {
            return 0.0;
        }
    }
    return amax > amin ? (amax - amin) * sqrt(d2) : 0.0;
}

static int64_t n_rays(const og_geom *g)
{
    return (int64_t)g->n_views * g->rows * g->cols;
}

static void ray_of(const og_geom *g, int64_t i, int32_t *v, int32_t *row, int32_t *col)
{
    *col = (int32_t)(i % g->cols);
    *row = (int32_t)((i / g->cols) % g->rows);
    *v = (int32_t)(i / ((int64_t)g->cols * g->rows));
}

/* y = A x: ray sums along Siddon paths (Sec. II-A, eq. 1). */
void og_project(const og_geom *g, const double *x, double *y)
{
    int32_t cap = g->nx + g->ny + g->nz + 3;
    int64_t m = n_rays(g);
#pragma omp parallel
    {
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
        double *work = (double *)malloc(sizeof(double) * 2 * cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            int32_t v, row, col;
            double p0[3], p1[3];
            ray_of(g, i, &v, &row, &col);
            og_ray_endpoints(g, v, row, col, p0, p1);
            int32_t k = og_siddon(g, p0, p1, idx, len, work);
            double s = 0.0;
            for (int32_t q = 0; q < k; ++q)
                s += len[q] * x[idx[q]];
            y[i] = s;
        }
        free(idx);
        free(len);
        free(work);
    }
}

double og_ray_sum(const og_geom *g, int32_t v, int32_t row, int32_t col, const double *x)
{
    int32_t cap = g->nx + g->ny + g->nz + 3;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * cap);
    double *len = (double *)malloc(sizeof(double) * cap);
    double *work = (double *)malloc(sizeof(double) * 2 * cap);
    double p0[3], p1[3];
    og_ray_endpoints(g, v, row, col, p0, p1);
    int32_t k = og_siddon(g, p0, p1, idx, len, work);
    double s = 0.0;
    for (int32_t q = 0; q < k; ++q)
        s += len[q] * x[idx[q]];
    free(idx);
    free(len);
    free(work);
    return s;
}

int64_t og_nnz(const og_geom *g)
{
    int32_t cap = g->nx + g->ny + g->nz + 3;
    int64_t m = n_rays(g), total = 0;
#pragma omp parallel reduction(+ : total)
    {
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
        double *work = (double *)malloc(sizeof(double) * 2 * cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            int32_t v, row, col;
            double p0[3], p1[3];
            ray_of(g, i, &v, &row, &col);
            og_ray_endpoints(g, v, row, col, p0, p1);
            total += og_siddon(g, p0, p1, idx, len, work);
        }
        free(idx);
        free(len);
        free(work);
    }
    return total;
}

/*
 * x = A^T r: the transpose of og_project, ray by ray.  Each thread scatters
 * into its own full-size buffer over a fixed (static) range of rays; the
 * buffers are then summed in thread order.
 */
void og_backproject(const og_geom *g, const double *r, double *x)
{
    int32_t cap = g->nx + g->ny + g->nz + 3;
    int64_t m = n_rays(g);
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
    int nt = og_num_threads();
    double *buf = (double *)calloc((size_t)nt * (size_t)N, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double *mine = buf + (size_t)t * (size_t)N;
        int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * cap);
        double *len = (double *)malloc(sizeof(double) * cap);
        double *work = (double *)malloc(sizeof(double) * 2 * cap);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            int32_t v, row, col;
            double p0[3], p1[3];
            ray_of(g, i, &v, &row, &col);
            og_ray_endpoints(g, v, row, col, p0, p1);
            int32_t k = og_siddon(g, p0, p1, idx, len, work);
            for (int32_t q = 0; q < k; ++q)
                mine[idx[q]] += len[q] * r[i];
        }
        free(idx);
        free(len);
        free(work);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t)
            s += buf[(size_t)t * (size_t)N + (size_t)j];
        x[j] = s;
    }
    free(buf);
}

/* y_i = sum_j |ray_i inside voxel_j| x_j with every (ray, voxel) pair
   tested by the slab formula: O(m N), tiny volumes only. */
void og_project_bruteforce(const og_geom *g, const double *x, double *y)
{
    int64_t m = n_rays(g);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        int32_t v, row, col;
        double p0[3], p1[3], lo[3], hi[3];
        ray_of(g, i, &v, &row, &col);
        og_ray_endpoints(g, v, row, col, p0, p1);
        double s = 0.0;
        for (int32_t k = 0; k < g->nz; ++k)
            for (int32_t jj = 0; jj < g->ny; ++jj)
                for (int32_t ii = 0; ii < g->nx; ++ii) {
                    lo[0] = ii - 0.5 * g->nx;
                    lo[1] = jj - 0.5 * g->ny;
                    lo[2] = k - 0.5 * g->nz;
                    hi[0] = lo[0] + 1.0;
                    hi[1] = lo[1] + 1.0;
                    hi[2] = lo[2] + 1.0;
                    double l = og_slab_length(p0, p1, lo, hi);
                    if (l > 0.0)
                        s += l * x[ii + g->nx * (jj + (int64_t)g->ny * k)];
                }
        y[i] = s;
    }
}

/* Dense A (m x N, row-major) from the brute-force slab lengths. */
void og_matrix_dense(const og_geom *g, double *A)
{
    int64_t m = n_rays(g);
    int64_t N = (int64_t)g->nx * g->ny * g->nz;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        int32_t v, row, col;
        double p0[3], p1[3], lo[3], hi[3];
        ray_of(g, i, &v, &row, &col);
        og_ray_endpoints(g, v, row, col, p0, p1);
        for (int64_t j = 0; j < N; ++j) {
            int32_t ii = (int32_t)(j % g->nx);
            int32_t jj = (int32_t)((j / g->nx) % g->ny);
            int32_t k = (int32_t)(j / ((int64_t)g->nx * g->ny));
            lo[0] = ii - 0.5 * g->nx;
            lo[1] = jj - 0.5 * g->ny;
            lo[2] = k - 0.5 * g->nz;
            hi[0] = lo[0] + 1.0;
            hi[1] = lo[1] + 1.0;
            hi[2] = lo[2] + 1.0;
            A[i * N + j] = og_slab_length(p0, p1, lo, hi);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Smoothed total variation                                                  */
/* ------------------------------------------------------------------------ */

/*
 * T_tau(x) = sum_j Phi_tau(D_j x)  (eq. 2 with the Euclidean norm replaced
 * by its Huber smoothing, which gives the Lipschitz gradient the methods of
 * Sec. III assume):
 *   Phi_tau(z) = |z| - tau/2  if |z| >= tau,  |z|^2 / (2 tau) otherwise;
 *   D_j x = forward differences (x_{j+e} - x_j) along x, y, z; a component
 *   whose neighbour lies outside the volume is 0 (reflecting boundary).
 * grad (optional) = sum_j D_j^T (D_j x / max(tau, |D_j x|)), formed by
 * scattering each voxel's term to the voxels its differences touch.
 */
double og_tv(int32_t nx, int32_t ny, int32_t nz, double tau, const double *x, double *grad)
{
    int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    int64_t N = sz * nz;
    if (grad)
        memset(grad, 0, sizeof(double) * (size_t)N);
    double T = 0.0;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                int64_t q = i * sx + j * sy + k * sz;
                double dx = (i + 1 < nx) ? x[q + sx] - x[q] : 0.0;
                double dy = (j + 1 < ny) ? x[q + sy] - x[q] : 0.0;
                double dz = (k + 1 < nz) ? x[q + sz] - x[q] : 0.0;
                double nrm = sqrt(dx * dx + dy * dy + dz * dz);
                T += (nrm >= tau) ? nrm - 0.5 * tau : nrm * nrm / (2.0 * tau);
                if (grad) {
                    double den = fmax(tau, nrm);
                    double qx = dx / den, qy = dy / den, qz = dz / den;
                    grad[q] -= qx + qy + qz;
                    if (i + 1 < nx)
                        grad[q + sx] += qx;
                    if (j + 1 < ny)
                        grad[q + sy] += qy;
                    if (k + 1 < nz)
                        grad[q + sz] += qz;
                }
            }
    return T;
}

/*
 * Bregman distance of the Huber function Phi_tau between a and b,
 *   B(a, b) = Phi(a) - Phi(b) - grad Phi(b)^T (a - b),   d = a - b given,
 * written per regime so that the result is formed from d without
 * subtracting nearly equal quantities (the four expressions follow from
 * |a|^2 = |b|^2 + 2 b.d + |d|^2):
 *   |a|,|b| <  tau:  |d|^2 / (2 tau)
 *   |a|,|b| >= tau:  |a| / 2 * |a/|a| - b/|b||^2
 *   |a| >= tau > |b|: (|d|^2 - (|a| - tau)^2) / (2 tau)
 *   |a| < tau <= |b|: |a - tau b/|b||^2 / (2 tau)
 */
double og_huber_bregman(const double a[3], const double b[3], const double d[3], double tau)
{
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (na < tau && nb < tau)
        return dd / (2.0 * tau);
    if (na >= tau && nb >= tau) {
        /* a/|a| - b/|b| = d/|a| - (b/|b|) ((a + b).d) / (|a| (|a| + |b|)) */
        double s = ((a[0] + b[0]) * d[0] + (a[1] + b[1]) * d[1] + (a[2] + b[2]) * d[2]) /
                   (na * (na + nb));
        double e2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            double e = d[c] / na - (b[c] / nb) * s;
            e2 += e * e;
        }
        return 0.5 * na * e2;
    }
    if (na >= tau) {
        double t = na - tau;
        double v = (dd - t * t) / (2.0 * tau);
        return v > 0.0 ? v : 0.0;
    }
    double e2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        double e = a[c] - tau * b[c] / nb;
        e2 += e * e;
    }
    return e2 / (2.0 * tau);
}

/* B_T(x, y) = T(x) - T(y) - grad T(y)^T (x - y) = sum_j B(D_j x, D_j y). */
double og_tv_bregman(int32_t nx, int32_t ny, int32_t nz, double tau, const double *x,
                     const double *y)
{
    int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    double s = 0.0;
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                int64_t q = i * sx + j * sy + k * sz;
                double a[3], bb[3], d[3];
                int64_t st[3] = {sx, sy, sz};
                int in[3] = {i + 1 < nx, j + 1 < ny, k + 1 < nz};
                for (int c = 0; c < 3; ++c) {
                    a[c] = in[c] ? x[q + st[c]] - x[q] : 0.0;
                    bb[c] = in[c] ? y[q + st[c]] - y[q] : 0.0;
                    d[c] = in[c] ? (x[q + st[c]] - y[q + st[c]]) - (x[q] - y[q]) : 0.0;
                }
                s += og_huber_bregman(a, bb, d, tau);
            }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Operators behind the solvers                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t m, N;
    int32_t nx, ny, nz;
    const og_geom *g;   /* geometry operator, or */
    const double *A;    /* dense row-major m x N */
} og_op;

static void op_apply(const og_op *op, const double *x, double *y)
{
    if (op->g) {
        og_project(op->g, x, y);
        return;
    }
    for (int64_t i = 0; i < op->m; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < op->N; ++j)
            s += op->A[i * op->N + j] * x[j];
        y[i] = s;
    }
}

static void op_apply_t(const og_op *op, const double *r, double *x)
{
    if (op->g) {
        og_backproject(op->g, r, x);
        return;
    }
    for (int64_t j = 0; j < op->N; ++j)
        x[j] = 0.0;
    for (int64_t i = 0; i < op->m; ++i)
        for (int64_t j = 0; j < op->N; ++j)
            x[j] += op->A[i * op->N + j] * r[i];
}

/* f(x) = 1/2 |A x - b|^2 + alpha T_tau(x)  (eq. 1, smoothed TV) */
static double op_f(const og_op *op, const double *b, double alpha, double tau,
                   const double *x, double *tmp_m)
{
    op_apply(op, x, tmp_m);
    double s = 0.0;
    for (int64_t i = 0; i < op->m; ++i) {
        double ri = tmp_m[i] - b[i];
        s += ri * ri;
    }
    double T = alpha != 0.0 ? og_tv(op->nx, op->ny, op->nz, tau, x, NULL) : 0.0;
    return 0.5 * s + alpha * T;
}

/* f(x) and grad f(x) = A^T (A x - b) + alpha grad T_tau(x) */
static double op_fg(const og_op *op, const double *b, double alpha, double tau,
                    const double *x, double *grad, double *tmp_m, double *tmp_n)
{
    op_apply(op, x, tmp_m);
    double s = 0.0;
    for (int64_t i = 0; i < op->m; ++i) {
        tmp_m[i] -= b[i];
        s += tmp_m[i] * tmp_m[i];
    }
    op_apply_t(op, tmp_m, grad);
    double T = 0.0;
    if (alpha != 0.0) {
        T = og_tv(op->nx, op->ny, op->nz, tau, x, tmp_n);
        for (int64_t j = 0; j < op->N; ++j)
            grad[j] += alpha * tmp_n[j];
    }
    return 0.5 * s + alpha * T;
}

double og_phi(const og_geom *g, const double *b, double alpha, double tau, const double *x)
{
    og_op op = {n_rays(g), (int64_t)g->nx * g->ny * g->nz, g->nx, g->ny, g->nz, g, NULL};
    double *tm = (double *)malloc(sizeof(double) * (size_t)op.m);
    double f = op_f(&op, b, alpha, tau, x, tm);
    free(tm);
    return f;
}

double og_phi_grad(const og_geom *g, const double *b, double alpha, double tau,
                   const double *x, double *grad)
{
    og_op op = {n_rays(g), (int64_t)g->nx * g->ny * g->nz, g->nx, g->ny, g->nz, g, NULL};
    double *tm = (double *)malloc(sizeof(double) * (size_t)op.m);
    double *tn = (double *)malloc(sizeof(double) * (size_t)op.N);
    double f = op_fg(&op, b, alpha, tau, x, grad, tm, tn);
    free(tm);
    free(tn);
    return f;
}

/* P_Q for Q = nonnegative orthant (Sec. IV-A) */
static double pq(double v) { return v > 0.0 ? v : 0.0; }

/* P_Q for a box Q = [lo, hi]^N (Sec. III: any feasible set with an easy
   projection); equals pq for lo = 0, hi = +inf */
static double pq_box(double v, double lo, double hi) { return v > lo ? (v < hi ? v : hi) : lo; }

/* |G_nu(x)|_2 with G_nu(x) = nu (x - P_Q(x - grad/nu))  (eq. 10) */
double og_gradmap_norm_box(int64_t n, const double *x, const double *grad, double nu, double lo,
                           double hi)
{
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double gj = nu * (x[j] - pq_box(x[j] - grad[j] / nu, lo, hi));
        s += gj * gj;
    }
    return sqrt(s);
}

double og_gradmap_norm(int64_t n, const double *x, const double *grad, double nu)
{
    return og_gradmap_norm_box(n, x, grad, nu, 0.0, INFINITY);
}

static double dist2(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double d = a[j] - b[j];
        s += d * d;
    }
    return s;
}

/* grad(y)^T (x - y) */
static double gdot_diff(int64_t n, const double *g, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j)
        s += g[j] * (x[j] - y[j]);
    return s;
}

static void record(double *h, int32_t len, int32_t k, double v)
{
    if (h && k >= 0 && k < len)
        h[k] = v;
}

/*
 * BT, Alg. 2: starting from L~ = L_start, x = P_Q(y - grad/L~); while
 * f(x) > f(y) + grad^T (x - y) + L~/2 |x - y|^2, multiply L~ by rho_L and
 * recompute x.  Returns 0 on acceptance, -1 when max_trials growths did not
 * satisfy the test (x then holds the last trial).
 */
/*
 * Bregman distance of f at y towards x:
 *   f(x) - f(y) - grad f(y)^T (x - y) = 1/2 |A (x - y)|^2 + alpha B_T(x, y)
 * (exact for the quadratic data term; B_T from og_tv_bregman).  This is the
 * left side of the BT test of Alg. 2 and the numerator of eq. 9 minus the
 * right side's first two terms, rearranged so that no two large objective
 * values are subtracted.  tmp_n and tmp_m are scratch.
 */
static double op_bregman(const og_op *op, const og_params *p, const double *x, const double *y,
                         double *tmp_n, double *tmp_m)
{
    for (int64_t j = 0; j < op->N; ++j)
        tmp_n[j] = x[j] - y[j];
    op_apply(op, tmp_n, tmp_m);
    double s = 0.0;
    for (int64_t i = 0; i < op->m; ++i)
        s += tmp_m[i] * tmp_m[i];
    double bt = p->alpha != 0.0 ? og_tv_bregman(op->nx, op->ny, op->nz, p->tau, x, y) : 0.0;
    return 0.5 * s + p->alpha * bt;
}

/*
 * BT, Alg. 2: starting from L~ = L_start, x = P_Q(y - grad/L~); while
 * f(x) > f(y) + grad^T (x - y) + L~/2 |x - y|^2, multiply L~ by rho_L and
 * recompute x.  Returns 0 on acceptance, -1 when max_trials growths did not
 * satisfy the test (x then holds the last trial).  bt_form = 1 evaluates the
 * same inequality as Bregman_f(x, y) > L~/2 |x - y|^2.  Nesterov's method
 * with a known L (Sec. III-B) takes the step 1/L without the test.
 */
static int op_bt(const og_op *op, const double *b, const og_params *p, const double *y,
                 double fy, const double *gy, double L_start, double *x, double *fx_out,
                 double *L_out, double *tmp_m, double *tmp_n, og_info *info)
{
    double L = L_start;
    for (int32_t trial = 0;; ++trial) {
        for (int64_t j = 0; j < op->N; ++j)
            x[j] = pq_box(y[j] - gy[j] / L, p->lower, p->upper);
        double fx = op_f(op, b, p->alpha, p->tau, x, tmp_m);
        info->func_evals++;
        int reject;
        if (p->method == OG_NESTEROV) {
            reject = 0;
        } else if (p->bt_form == 1) {
            double br = op_bregman(op, p, x, y, tmp_n, tmp_m);
            reject = br > 0.5 * L * dist2(op->N, x, y);
        } else {
            double rhs = fy + gdot_diff(op->N, gy, x, y) + 0.5 * L * dist2(op->N, x, y);
            reject = fx > rhs;
        }
        if (!reject) {
            *fx_out = fx;
            *L_out = L;
            return 0;
        }
        if (trial + 1 >= p->max_trials) {
            *fx_out = fx;
            *L_out = L;
            return -1;
        }
        L *= p->rho_L;
    }
}

static int stop_now(const og_params *p, double gm, double gm0, int64_t N)
{
    if (p->stop_mode == 1)
        return gm / (double)N <= p->eps;
    return gm0 == 0.0 || gm <= p->eps * gm0;
}

/*
 * GP (eq. 6) with step 1/L_k from BT warm-started at L_{k-1}, and UPN
 * (Alg. 3).  GP is UPN with beta_k = 0.  Nesterov's method for given mu and
 * L (Sec. III-B, rate of eq. 8) is UPN with L_k = L_bar (no line-search
 * test) and mu_k = mu_bar (no eq. 9 estimate).  The stop test (Sec. III-D) uses the
 * gradient map at the point whose gradient was just evaluated (x^(k) for GP,
 * y^(k) for UPN) with nu = L_k, which equals L_k (z - x^(k+1)).
 */
static int32_t solve_gp_upn(const og_op *op, const double *b, const og_params *p, double *x,
                            og_info *info, double *hphi, double *hgm, double *hL, double *hmu,
                            double *htheta, int32_t hlen)
{
    int64_t N = op->N, m = op->m;
    int nest = p->method == OG_NESTEROV;
    int upn = p->method == OG_UPN || nest;
    double *xk = (double *)malloc(sizeof(double) * N);   /* x^(k) */
    double *xn = (double *)malloc(sizeof(double) * N);   /* x^(k+1) */
    double *y = (double *)malloc(sizeof(double) * N);    /* y^(k) */
    double *gy = (double *)malloc(sizeof(double) * N);
    double *tm = (double *)malloc(sizeof(double) * m);
    double *tn = (double *)malloc(sizeof(double) * N);
    int32_t status = OG_NOTCONV;
    memcpy(xk, x, sizeof(double) * N);
    memcpy(y, x, sizeof(double) * N);

    /* k = 0: [x^(1), L_0] = BT(x^(0), L_bar) */
    double fy = op_fg(op, b, p->alpha, p->tau, y, gy, tm, tn);
    info->grad_evals++;
    double fx_new, L;
    int bt = op_bt(op, b, p, y, fy, gy, p->L_bar, xn, &fx_new, &L, tm, tn, info);
    double gm0 = L * sqrt(dist2(N, y, xn));
    info->gm0 = gm0;
    info->gm = gm0;
    info->iters = 1;
    info->L = L;
    record(hphi, hlen, 0, fx_new);
    record(hgm, hlen, 0, 1.0);
    record(hL, hlen, 0, L);
    double mu = p->mu_bar > 0.0 ? p->mu_bar : 0.25 * L;
    if (nest)
        mu = p->mu_bar > 0.0 ? p->mu_bar : 0.0;
    if (p->force_mu == 1)
        mu = L;
    else if (p->force_mu == 2)
        mu = L; /* theta_1 = 1, then mu_k = 0: the mu = 0 recurrence from its usual start */
    double theta = sqrt(mu / L);
    record(hmu, hlen, 0, mu);
    record(htheta, hlen, 0, theta);
    double fx_k = 0.0;
    int fx_k_valid = 0;
    if (bt != 0) {
        status = OG_STALL;
        goto done;
    }
    if (stop_now(p, gm0, gm0, N)) {
        status = OG_CONVERGED;
        goto done;
    }
    /* x^(1) accepted; y^(1) = x^(1) */
    memcpy(xk, xn, sizeof(double) * N);
    memcpy(y, xn, sizeof(double) * N);
    fx_k = fx_new;
    fx_k_valid = 1;

    for (int32_t k = 1; k < p->max_iter; ++k) {
        fy = op_fg(op, b, p->alpha, p->tau, y, gy, tm, tn);
        info->grad_evals++;
        bt = op_bt(op, b, p, y, fy, gy, L, xn, &fx_new, &L, tm, tn, info);
        double gm = L * sqrt(dist2(N, y, xn));
        info->iters = k + 1;
        info->gm = gm;
        info->L = L;
        record(hphi, hlen, k, fx_new);
        record(hgm, hlen, k, gm0 > 0 ? gm / gm0 : 0.0);
        record(hL, hlen, k, L);
        if (bt != 0) {
            status = OG_STALL;
            break;
        }
        if (stop_now(p, gm, gm0, N)) {
            status = OG_CONVERGED;
            break;
        }
        double beta = 0.0;
        if (upn) {
            /* eq. 9 between x^(k) and y^(k); skipped where they coincide */
            double nd = dist2(N, xk, y);
            if (nest) {
                /* mu and L are given */
            } else if (p->force_mu == 1) {
                mu = L;
            } else if (p->force_mu == 2) {
                mu = 0.0;
            } else if (nd > 0.0) {
                double num = p->bt_form == 1 ? op_bregman(op, p, xk, y, tn, tm)
                                             : fx_k - fy - gdot_diff(N, gy, xk, y);
                double M = num / (0.5 * nd);
                mu = fmin(mu, M);
                if (mu < 0.0)
                    mu = 0.0;
            }
            /* theta_{k+1}: positive root of t^2 = (1 - t) theta_k^2 + (mu/L) t */
            double q = mu / L, th2 = theta * theta;
            double bq = th2 - q;
            double theta_n = 0.5 * (-bq + sqrt(bq * bq + 4.0 * th2));
            beta = theta * (1.0 - theta) / (th2 + theta_n);
            theta = theta_n;
        }
        record(hmu, hlen, k, mu);
        record(htheta, hlen, k, theta); /* theta_{k+1} (UPN), the unchanged start value otherwise */
        /* y^(k+1) = x^(k+1) + beta_k (x^(k+1) - x^(k)) */
        for (int64_t j = 0; j < N; ++j) {
            y[j] = xn[j] + beta * (xn[j] - xk[j]);
            xk[j] = xn[j];
        }
        fx_k = fx_new;
    }
done:
    if (status == OG_STALL) {
        /* the last accepted point is x^(k) (x^(0) when the first BT stalls) */
        memcpy(x, xk, sizeof(double) * N);
        info->phi = fx_k_valid ? fx_k : fy;
    } else {
        memcpy(x, xn, sizeof(double) * N);
        info->phi = fx_new;
    }
    info->mu = mu;
    info->status = status;
    free(xk);
    free(xn);
    free(y);
    free(gy);
    free(tm);
    free(tn);
    return status;
}

/*
 * GPBB, Alg. 1: Barzilai-Borwein step theta_k = |s|^2 / <s, dg> with
 * s = x^(k) - x^(k-1), dg = grad f(x^(k)) - grad f(x^(k-1)) (theta_0 = 1),
 * then the nonmonotone line search: beta = beta0,
 * xbar = P_Q(x^(k) - beta theta_k grad f(x^(k))), and while
 * f(xbar) >= max{f(x^(k)), ..., f(x^(k-K))} - sigma grad^T (x^(k) - xbar)
 * set beta <- beta^2.  Readings: the max runs over the history available;
 * a non-positive or non-finite <s, dg> keeps theta_{k-1}; the stop test at
 * x^(k) uses nu = 1 / theta_k.
 */
static int32_t solve_gpbb(const og_op *op, const double *b, const og_params *p, double *x,
                          og_info *info, double *hphi, double *hgm, double *hL, int32_t hlen)
{
    int64_t N = op->N, m = op->m;
    double *xk = (double *)malloc(sizeof(double) * N);
    double *xp = (double *)malloc(sizeof(double) * N);
    double *gk = (double *)malloc(sizeof(double) * N);
    double *gp = (double *)malloc(sizeof(double) * N);
    double *xb = (double *)malloc(sizeof(double) * N);
    double *tm = (double *)malloc(sizeof(double) * m);
    double *tn = (double *)malloc(sizeof(double) * N);
    int32_t K = p->gpbb_K;
    double *fh = (double *)malloc(sizeof(double) * (K + 1));
    int32_t nf = 0; /* valid history entries */
    int32_t status = OG_NOTCONV;
    memcpy(xk, x, sizeof(double) * N);
    double theta = 1.0, gm0 = 0.0, fk = 0.0;

    for (int32_t k = 0; k < p->max_iter; ++k) {
        double fval = op_fg(op, b, p->alpha, p->tau, xk, gk, tm, tn);
        info->grad_evals++;
        if (k == 0)
            fk = fval;
        /* history: f(x^(k)), f(x^(k-1)), ..., f(x^(k-K)) */
        for (int32_t q = (nf < K + 1 ? nf : K); q > 0; --q)
            fh[q] = fh[q - 1];
        fh[0] = fk;
        if (nf < K + 1)
            nf++;
        if (k > 0) {
            double ss = 0.0, sy = 0.0;
            for (int64_t j = 0; j < N; ++j) {
                double s = xk[j] - xp[j];
                ss += s * s;
                sy += s * (gk[j] - gp[j]);
            }
            if (sy > 0.0 && isfinite(sy) && isfinite(ss / sy) && ss > 0.0)
                theta = ss / sy;
        }
        double gm = og_gradmap_norm_box(N, xk, gk, 1.0 / theta, p->lower, p->upper);
        if (k == 0) {
            gm0 = gm;
            info->gm0 = gm0;
        }
        info->gm = gm;
        info->iters = k;
        info->L = 1.0 / theta;
        record(hgm, hlen, k, gm0 > 0 ? gm / gm0 : 0.0);
        record(hL, hlen, k, 1.0 / theta);
        record(hphi, hlen, k, fk);
        if (stop_now(p, gm, gm0, N)) {
            status = OG_CONVERGED;
            break;
        }
        double fhat = fh[0];
        for (int32_t q = 1; q < nf; ++q)
            fhat = fmax(fhat, fh[q]);
        double beta = p->gpbb_beta0, fb = 0.0;
        int ok = 0;
        for (int32_t sq = 0; sq <= p->max_squarings; ++sq) {
            for (int64_t j = 0; j < N; ++j)
                xb[j] = pq_box(xk[j] - beta * theta * gk[j], p->lower, p->upper);
            fb = op_f(op, b, p->alpha, p->tau, xb, tm);
            info->func_evals++;
            double gd = 0.0;
            for (int64_t j = 0; j < N; ++j)
                gd += gk[j] * (xk[j] - xb[j]);
            if (!(fb >= fhat - p->gpbb_sigma * gd)) {
                ok = 1;
                break;
            }
            beta = beta * beta;
        }
        if (!ok) {
            status = OG_STALL; /* x^(k) stays the output */
            break;
        }
        /* x^(k+1) = xbar */
        double *t = xp;
        xp = xk;
        xk = xb;
        xb = t;
        t = gp;
        gp = gk;
        gk = t;
        fk = fb;
        info->iters = k + 1;
    }
    memcpy(x, xk, sizeof(double) * N);
    info->phi = fk;
    info->mu = 0.0;
    info->status = status;
    free(xk);
    free(xp);
    free(gk);
    free(gp);
    free(xb);
    free(tm);
    free(tn);
    free(fh);
    return status;
}

static int32_t solve_op(const og_op *op, const double *b, const og_params *p, double *x,
                        og_info *info, double *hphi, double *hgm, double *hL, double *hmu,
                        double *htheta, int32_t hlen)
{
    memset(info, 0, sizeof(*info));
    for (int64_t j = 0; j < op->N; ++j)
        x[j] = pq_box(x[j], p->lower, p->upper); /* start from a feasible point */
    if (p->method == OG_GPBB)
        return solve_gpbb(op, b, p, x, info, hphi, hgm, hL, hlen);
    return solve_gp_upn(op, b, p, x, info, hphi, hgm, hL, hmu, htheta, hlen);
}

int32_t og_solve(const og_geom *g, const double *b, const og_params *p, double *x,
                 og_info *info, double *hist_phi, double *hist_gm, double *hist_L,
                 double *hist_mu, double *hist_theta, int32_t hist_len)
{
    og_op op = {n_rays(g), (int64_t)g->nx * g->ny * g->nz, g->nx, g->ny, g->nz, g, NULL};
    return solve_op(&op, b, p, x, info, hist_phi, hist_gm, hist_L, hist_mu, hist_theta, hist_len);
}

int32_t og_solve_dense(int32_t m, int32_t nx, int32_t ny, int32_t nz, const double *A,
                       const double *b, const og_params *p, double *x, og_info *info,
                       double *hist_phi, double *hist_gm, double *hist_L, double *hist_mu,
                       double *hist_theta, int32_t hist_len)
{
    og_op op = {m, (int64_t)nx * ny * nz, nx, ny, nz, NULL, A};
    return solve_op(&op, b, p, x, info, hist_phi, hist_gm, hist_L, hist_mu, hist_theta, hist_len);
}

/* ------------------------------------------------------------------------ */
/* Differentiated form: K unrolled UPN steps and their reverse-mode adjoint  */
/* (not a passage of the paper; it differentiates the map Alg. 3 applies)    */
/* ------------------------------------------------------------------------ */

/*
 * Hessian of the smoothed TV applied to v:
 *   H(y) v = sum_j D_j^T dq_j,   dq_j = d/dt [D_j(y + t v) / max(tau, |D_j(y + t v)|)]
 * which is D_j v / tau where |D_j y| < tau, and (e - u (u.e)) / |D_j y| with
 * u = D_j y / |D_j y|, e = D_j v where |D_j y| >= tau (the regime split of
 * og_tv; the Hessian jumps across |D_j y| = tau).
 */
void og_tv_hessvec(int32_t nx, int32_t ny, int32_t nz, double tau, const double *y,
                   const double *v, double *out)
{
    int64_t sx = 1, sy = nx, sz = (int64_t)nx * ny;
    int64_t N = sz * nz;
    memset(out, 0, sizeof(double) * (size_t)N);
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                int64_t q = i * sx + j * sy + k * sz;
                int in[3] = {i + 1 < nx, j + 1 < ny, k + 1 < nz};
                int64_t st[3] = {sx, sy, sz};
                double a[3], e[3], dq[3];
                for (int c = 0; c < 3; ++c) {
                    a[c] = in[c] ? y[q + st[c]] - y[q] : 0.0;
                    e[c] = in[c] ? v[q + st[c]] - v[q] : 0.0;
                }
                double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
                if (n >= tau) {
                    double ue = (a[0] * e[0] + a[1] * e[1] + a[2] * e[2]) / n;
                    for (int c = 0; c < 3; ++c)
                        dq[c] = (e[c] - (a[c] / n) * ue) / n;
                } else {
                    for (int c = 0; c < 3; ++c)
                        dq[c] = e[c] / tau;
                }
                out[q] -= dq[0] + dq[1] + dq[2];
                for (int c = 0; c < 3; ++c)
                    if (in[c])
                        out[q + st[c]] += dq[c];
            }
}

/* FNV-style fold of the discrete pattern a step's derivative depends on */
static uint64_t fold(uint64_t h, uint64_t v)
{
    h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
    return h;
}

static uint64_t pattern_signature(uint64_t h, int32_t nx, int32_t ny, int32_t nz, double tau,
                                  const double *y, const double *xn)
{
    int64_t sy = nx, sz = (int64_t)nx * ny, N = sz * nz;
    for (int64_t q = 0; q < N; ++q)
        if (xn[q] > 0.0)
            h = fold(h, (uint64_t)q);
    for (int32_t k = 0; k < nz; ++k)
        for (int32_t j = 0; j < ny; ++j)
            for (int32_t i = 0; i < nx; ++i) {
                int64_t q = i + j * sy + k * sz;
                double dx = (i + 1 < nx) ? y[q + 1] - y[q] : 0.0;
                double dy = (j + 1 < ny) ? y[q + sy] - y[q] : 0.0;
                double dz = (k + 1 < nz) ? y[q + sz] - y[q] : 0.0;
                if (sqrt(dx * dx + dy * dy + dz * dz) >= tau)
                    h = fold(h, (uint64_t)(N + q));
            }
    return h;
}

/*
 * K steps of UPN (Alg. 3) from x^(0) = 0, output x^(K) (the K-th BT output),
 * and, when xK_bar != NULL, the gradient of l(x^(K)) with respect to alpha
 * and b given xK_bar = dl/dx^(K).
 *
 * Forward.  Step j maps y^(j) to x^(j+1) = P_Q(y^(j) - grad f(y^(j)) / L_j).
 * L_j comes from BT (Alg. 2, started at L_bar for j = 0 and at L_{j-1}
 * after) or, with replay != 0, is read from L[j] with no test.  After step 0:
 * mu_0 = mu_bar (or L_0 / 4 when mu_bar <= 0), theta_1 = sqrt(mu_0 / L_0),
 * y^(1) = x^(1).  After step j >= 1: mu_j = max(min(mu_{j-1}, M_j), 0) with
 * M_j = Bregman_f(x^(j), y^(j)) / (|x^(j) - y^(j)|^2 / 2) (eq. 9, evaluated
 * only when x^(j) != y^(j)); theta_{j+1} is the positive root of
 * t^2 = (1 - t) theta_j^2 + (mu_j / L_j) t; beta_j = theta_j (1 - theta_j) /
 * (theta_j^2 + theta_{j+1}); y^(j+1) = x^(j+1) + beta_j (x^(j+1) - x^(j)).
 *
 * Reverse.  The L_j are held fixed (they are decisions, not functions of
 * the inputs); the min in mu_j is differentiated on the branch it took; the
 * projection P_Q contributes the mask [x^(j+1) > 0].  With z = y - grad f(y)/L
 * and grad f(y) = A^T (A y - b) + alpha grad T(y):
 *   dz/dy = I - (A^T A + alpha H(y)) / L,  dz/db = A^T / L,
 *   dz/dalpha = -grad T(y) / L.
 * theta_{j+1} solves F = t^2 + (theta_j^2 - q) t - theta_j^2 = 0, q = mu_j/L_j,
 * so dt/dtheta_j = 2 theta_j (1 - t) / s and dt/dq = t / s with
 * s = dF/dt = 2 t + theta_j^2 - q.  With d = x - y, D = |d|^2 / 2 and
 * M = (|A d|^2 / 2 + alpha B_T(x, y)) / D:
 *   dM/dx = (A^T A d + alpha (grad T(x) - grad T(y)) - M d) / D,
 *   dM/dy = (-A^T A d - alpha H(y) d + M d) / D,   dM/dalpha = B_T / D.
 * Every iterate is kept in memory (no checkpointing).
 *
 * mu_state[j]: 3 for step 0, 0 carried (mu_j = mu_{j-1}), 1 M_j taken,
 * 2 clamped to 0.  *signature folds the projection masks and the Huber
 * regimes met by the forward pass (equal signatures: same smooth piece).
 * Returns 0, or OG_STALL when a BT search hits max_trials (no reverse pass).
 */
int32_t og_unrolled(const og_geom *g, const double *b, const og_params *p, int32_t K,
                    int32_t replay, double *L, double *xK, const double *xK_bar,
                    double *alpha_bar, double *b_bar, double *mu_out, double *beta_out,
                    int32_t *mu_state, uint64_t *signature)
{
    og_op op = {n_rays(g), (int64_t)g->nx * g->ny * g->nz, g->nx, g->ny, g->nz, g, NULL};
    const int64_t N = op.N, m = op.m;
    const double alpha = p->alpha, tau = p->tau;
    double *xs = (double *)calloc((size_t)(K + 1) * N, sizeof(double)); /* x^(0..K) */
    double *ys = (double *)calloc((size_t)K * N, sizeof(double));       /* y^(0..K-1) */
    double *gy = (double *)malloc(sizeof(double) * N);
    double *tm = (double *)malloc(sizeof(double) * m);
    double *tn = (double *)malloc(sizeof(double) * N);
    double *theta = (double *)calloc((size_t)K + 2, sizeof(double));
    double *mu = (double *)calloc((size_t)K, sizeof(double));
    double *beta = (double *)calloc((size_t)K, sizeof(double));
    double *Mv = (double *)calloc((size_t)K, sizeof(double));
    double *Bv = (double *)calloc((size_t)K, sizeof(double));
    double *Dv = (double *)calloc((size_t)K, sizeof(double));
    int32_t *state = (int32_t *)calloc((size_t)K, sizeof(int32_t));
    og_info info;
    memset(&info, 0, sizeof(info));
    int32_t status = 0;
    uint64_t sig = 1469598103934665603ULL;

    /* ---- forward ---- */
    for (int32_t j = 0; j < K; ++j) {
        double *y = ys + (size_t)j * N, *xn = xs + (size_t)(j + 1) * N;
        double *xj = xs + (size_t)j * N;
        double fy = op_fg(&op, b, alpha, tau, y, gy, tm, tn);
        double Lj;
        if (replay) {
            Lj = L[j];
            for (int64_t q = 0; q < N; ++q)
                xn[q] = pq(y[q] - gy[q] / Lj);
        } else {
            double fx;
            double L0 = j == 0 ? p->L_bar : L[j - 1];
            if (op_bt(&op, b, p, y, fy, gy, L0, xn, &fx, &Lj, tm, tn, &info) != 0) {
                status = OG_STALL;
                goto out;
            }
            L[j] = Lj;
        }
        sig = pattern_signature(sig, g->nx, g->ny, g->nz, tau, y, xn);
        if (j == 0) {
            mu[0] = p->mu_bar > 0.0 ? p->mu_bar : 0.25 * Lj;
            state[0] = 3;
            theta[1] = sqrt(mu[0] / Lj);
            beta[0] = 0.0;
            if (K > 1)
                memcpy(ys + (size_t)N, xn, sizeof(double) * N);
            continue;
        }
        double nd = dist2(N, xj, y);
        double mu_j = mu[j - 1];
        state[j] = 0;
        if (nd > 0.0) {
            /* Bregman_f(x, y) = |A (x - y)|^2 / 2 + alpha B_T(x, y) */
            for (int64_t q = 0; q < N; ++q)
                tn[q] = xj[q] - y[q];
            op_apply(&op, tn, tm);
            double a2 = 0.0;
            for (int64_t i = 0; i < m; ++i)
                a2 += tm[i] * tm[i];
            Bv[j] = alpha != 0.0 ? og_tv_bregman(g->nx, g->ny, g->nz, tau, xj, y) : 0.0;
            Dv[j] = 0.5 * nd;
            Mv[j] = (0.5 * a2 + alpha * Bv[j]) / Dv[j];
            if (Mv[j] < mu_j) {
                if (Mv[j] >= 0.0) {
                    mu_j = Mv[j];
                    state[j] = 1;
                } else {
                    mu_j = 0.0;
                    state[j] = 2;
                }
            }
        }
        mu[j] = mu_j;
        double q = mu_j / Lj, th = theta[j], th2 = th * th, bq = th2 - q;
        theta[j + 1] = 0.5 * (-bq + sqrt(bq * bq + 4.0 * th2));
        beta[j] = th * (1.0 - th) / (th2 + theta[j + 1]);
        if (j + 1 < K) {
            double *yn = ys + (size_t)(j + 1) * N;
            for (int64_t r = 0; r < N; ++r)
                yn[r] = xn[r] + beta[j] * (xn[r] - xj[r]);
        }
    }
    memcpy(xK, xs + (size_t)K * N, sizeof(double) * N);

    /* ---- reverse ---- */
    if (xK_bar) {
        double *xb_next = (double *)malloc(sizeof(double) * N); /* adjoint of x^(j+1) */
        double *xb_cur = (double *)calloc((size_t)N, sizeof(double));
        double *yb_next = (double *)calloc((size_t)N, sizeof(double));
        double *yb_cur = (double *)calloc((size_t)N, sizeof(double));
        double *zb = (double *)malloc(sizeof(double) * N);
        double *w = (double *)malloc(sizeof(double) * N);
        double *h = (double *)malloc(sizeof(double) * N);
        double *gT = (double *)malloc(sizeof(double) * N);
        double *gT2 = (double *)malloc(sizeof(double) * N);
        double *pm = (double *)malloc(sizeof(double) * m);
        double *theta_bar = (double *)calloc((size_t)K + 2, sizeof(double));
        double *mu_bar = (double *)calloc((size_t)K, sizeof(double));
        double abar = 0.0;
        memcpy(xb_next, xK_bar, sizeof(double) * N);
        memset(b_bar, 0, sizeof(double) * m);
        for (int32_t j = K - 1; j >= 0; --j) {
            const double *xj = xs + (size_t)j * N, *xn = xs + (size_t)(j + 1) * N;
            const double *y = ys + (size_t)j * N;
            const double Lj = L[j];
            /* extrapolation and scalar schedule of step j (y^(j+1) is used by step j+1) */
            if (j >= 1 && j + 1 < K) {
                double bb = 0.0;
                for (int64_t r = 0; r < N; ++r)
                    bb += yb_next[r] * (xn[r] - xj[r]);
                for (int64_t r = 0; r < N; ++r) {
                    xb_next[r] += (1.0 + beta[j]) * yb_next[r];
                    xb_cur[r] += -beta[j] * yb_next[r];
                }
                double th = theta[j], tn1 = theta[j + 1];
                double num = th * (1.0 - th), den = th * th + tn1;
                theta_bar[j] += bb * ((1.0 - 2.0 * th) / den - num * 2.0 * th / (den * den));
                theta_bar[j + 1] += bb * (-num / (den * den));
                double q = mu[j] / Lj;
                double s = 2.0 * tn1 + th * th - q;
                theta_bar[j] += theta_bar[j + 1] * 2.0 * th * (1.0 - tn1) / s;
                mu_bar[j] += theta_bar[j + 1] * (tn1 / s) / Lj;
                if (state[j] == 0) {
                    mu_bar[j - 1] += mu_bar[j];
                } else if (state[j] == 1) {
                    double c = mu_bar[j] / Dv[j], M = Mv[j];
                    for (int64_t r = 0; r < N; ++r)
                        tn[r] = xj[r] - y[r];                   /* d */
                    op_apply(&op, tn, tm);
                    op_apply_t(&op, tm, w);                    /* A^T A d */
                    og_tv(g->nx, g->ny, g->nz, tau, xj, gT);   /* grad T(x) */
                    og_tv(g->nx, g->ny, g->nz, tau, y, gT2);   /* grad T(y) */
                    og_tv_hessvec(g->nx, g->ny, g->nz, tau, y, tn, h); /* H(y) d */
                    for (int64_t r = 0; r < N; ++r) {
                        xb_cur[r] += c * (w[r] + alpha * (gT[r] - gT2[r]) - M * tn[r]);
                        yb_cur[r] += c * (-w[r] - alpha * h[r] + M * tn[r]);
                    }
                    abar += mu_bar[j] * Bv[j] / Dv[j];
                }
            } else if (j == 0 && K > 1) {
                for (int64_t r = 0; r < N; ++r)
                    xb_next[r] += yb_next[r]; /* y^(1) = x^(1) */
            }
            /* step j: x^(j+1) = P_Q(y^(j) - grad f(y^(j)) / L_j) */
            for (int64_t r = 0; r < N; ++r)
                zb[r] = xn[r] > 0.0 ? xb_next[r] : 0.0;
            op_apply(&op, zb, pm);
            for (int64_t i = 0; i < m; ++i)
                b_bar[i] += pm[i] / Lj;
            op_apply_t(&op, pm, w);
            og_tv(g->nx, g->ny, g->nz, tau, y, gT);
            og_tv_hessvec(g->nx, g->ny, g->nz, tau, y, zb, h);
            double zg = 0.0;
            for (int64_t r = 0; r < N; ++r) {
                yb_cur[r] += zb[r] - (w[r] + alpha * h[r]) / Lj;
                zg += zb[r] * gT[r];
            }
            abar += -zg / Lj;
            /* shift: x^(j) and y^(j) become the next step's outputs */
            double *t = xb_next;
            xb_next = xb_cur;
            xb_cur = t;
            memset(xb_cur, 0, sizeof(double) * N);
            t = yb_next;
            yb_next = yb_cur;
            yb_cur = t;
            memset(yb_cur, 0, sizeof(double) * N);
        }
        *alpha_bar = abar;
        free(xb_next);
        free(xb_cur);
        free(yb_next);
        free(yb_cur);
        free(zb);
        free(w);
        free(h);
        free(gT);
        free(gT2);
        free(pm);
        free(theta_bar);
        free(mu_bar);
    }
out:
    if (mu_out)
        memcpy(mu_out, mu, sizeof(double) * K);
    if (beta_out)
        memcpy(beta_out, beta, sizeof(double) * K);
    if (mu_state)
        memcpy(mu_state, state, sizeof(int32_t) * K);
    if (signature)
        *signature = sig;
    free(xs);
    free(ys);
    free(gy);
    free(tm);
    free(tn);
    free(theta);
    free(mu);
    free(beta);
    free(Mv);
    free(Bv);
    free(Dv);
    free(state);
    return status;
}

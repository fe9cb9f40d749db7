// Internal declarations of the gfx950 TV-reconstruction library: the device
// view of a scan geometry, the reduction-slot layout and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tvr {

// Ray tables.  A ray is p(t) = S + t D; for a cone beam t in [0, 1] runs from
// the source to the pixel, for a parallel beam t is unbounded and D is the
// unit view direction.  The in-plane part (x, y) depends on (view, column),
// the axial part (z) on the detector row only.  Both the projector and the
// gather backprojector evaluate the crossing of the plane at coordinate X as
// t(X) = fma(X, invD, o) with o = -S * invD from these same tables, so A and
// A^T use bitwise identical FP64 crossing parameters.  invD = 0 marks a ray
// parallel to that axis (membership of S in the half-open cell decides).
struct ColEntry {
    double Sx, Sy, Dx, Dy, invDx, invDy, ox, oy;
};
struct RowEntry {
    double Sz, Dz, invDz, oz;
};

__host__ __device__ __forceinline__ double plane_t(double X, double invD, double o)
{
    return fma(X, invD, o);
}

// One view of the 3D parallel beam: unit direction d, detector axes e_u, e_v
// and 1/d per component (0 where d has none).
struct View3 {
    double dx, dy, dz, ux, uy, uz, vx, vy, vz, idx, idy, idz;
};

// Optional stored transpose A^T in a sliced-ELLPACK form whose slices are
// 8 x 8 voxel tiles of one z-plane (one wavefront each; tiles ordered x,
// then y, then z; lane l = 8 (y % 8) + x % 8; entry k of lane l of slice s
// at off[s] + 64 k + l): values a_ij = length |D_i| as T, ray indices int32.
// A tile's voxels project onto a compact detector patch in every view, so a
// wavefront's gathers of r stay within few cache lines.
constexpr int MAT_T = 8;  // tile side

__host__ __device__ __forceinline__ int64_t mat_slices(int nx, int ny, int nz)
{
    return (int64_t)((nx + MAT_T - 1) / MAT_T) * ((ny + MAT_T - 1) / MAT_T) * nz;
}

// slice and lane of voxel (x, y, z)
__host__ __device__ __forceinline__ void mat_slot(int nx, int ny, int x, int y, int z, int64_t &s,
                                                  int &l)
{
    const int tx = (nx + MAT_T - 1) / MAT_T, ty = (ny + MAT_T - 1) / MAT_T;
    s = ((int64_t)z * ty + y / MAT_T) * tx + x / MAT_T;
    l = (y % MAT_T) * MAT_T + x % MAT_T;
}

// voxel of lane l of slice s; false for lanes of an edge tile past the volume
__host__ __device__ __forceinline__ bool mat_voxel(int nx, int ny, int64_t s, int l, int &x,
                                                   int &y, int &z)
{
    const int tx = (nx + MAT_T - 1) / MAT_T, ty = (ny + MAT_T - 1) / MAT_T;
    x = (int)(s % tx) * MAT_T + l % MAT_T;
    y = (int)((s / tx) % ty) * MAT_T + l / MAT_T;
    z = (int)(s / ((int64_t)tx * ty));
    return x < nx && y < ny;
}

// Symmetry of a circular scan.  With views evenly spaced over the full
// circle (V divisible by 4), a square even volume and an even detector, the
// turn of the volume by a quarter about z carries ray (v, row, col) onto ray
// (v + V/4, row, col) and voxel (i, j, k) onto (nx - 1 - j, i, k) with the
// same length; with V even and an even volume, the half turn carries view v
// onto v + V/2 and (i, j) onto (nx - 1 - i, ny - 1 - j); with an even nz and
// an even detector, the mirror z -> -z carries row r onto rows - 1 - r and
// k onto nz - 1 - k.  The stored transpose then holds only the voxels of one
// cell i < mx, j < my, k < mz of the group (a quadrant or half of the plane,
// the lower half in z) and each entry serves rot * (mir ? 2 : 1) voxels.
// Entries of such a layout carry a packed ray key (view << (kc + kr)) |
// (row << kc) | col instead of the ray index.
struct MatDev {
    int present;                     // 0: A^T evaluated on the fly
    int64_t sv;                      // slices of voxels
    const int64_t *off_v;            // first entry of each slice
    const int32_t *w_v;              // slice widths (max entries of a lane)
    const int32_t *cnt_v;            // entries of each stored voxel (mx x my x mz)
    const void *val_v;               // a_ij
    const int32_t *idx_v;            // ray index (rot = 1, mir = 0) or packed ray key
    int rot;                         // 1, 2 (half turns) or 4 (quarter turns)
    int mir;                         // 1: the z mirror is used
    int mx, my, mz;                  // stored cell (the whole volume when rot = 1, mir = 0)
    int kc, kr;                      // bits of the column and row fields of a key
};

struct GeomDev {
    int nx, ny, nz;
    int nviews, cols, rows;
    int cone;
    double pu, pv, ipu, ipv;   // detector pitches and their inverses
    double R, SDD;             // cone only
    double cu0, rv0;           // (cols - 1) / 2, (rows - 1) / 2
    double hx, hy, hz;         // nx / 2, ny / 2, nz / 2
    const double2 *cs;         // [nviews] (cos theta, sin theta); 3D beam: (d_x, d_y)
    const ColEntry *col;       // [nviews * cols]
    const RowEntry *row;       // [rows]
    const double *dnorm;       // |D|: cone [rows * cols], parallel [nviews]
    MatDev mat;                // stored A^T when present
    int beam3d;                // 3D parallel beam: rays from v3, not from col / row
    const View3 *v3;           // [nviews] (3D parallel beam only)
    int pj_wc;                 // projector: detector columns of a wave's ray tile (1, 2, 8, 16, 32, 64)
    int pj_ty;                 // projector: ray tiles (waves) per block, stacked along rows (1, 2, 4, 8)
    int bp_cz;                 // on-the-fly backprojector: voxels per thread along z (4, 8, 16)
    int flat_row;              // cone: the detector row with w = 0 (invDz = 0), else -1
    int sym_rot;               // the scan's symmetry group a stored A^T may use (see MatDev):
    int sym_mir;               // turns (1, 2 or 4) and the z mirror (0 or 1)
};

// Default tile shapes.  The projector's default ray tile is two detector
// columns x 32 rows where the detector has a multiple of 32 rows (no idle
// lanes), else 64 columns x 1 row.
constexpr int PJ_TY_DEFAULT = 4;
constexpr int BP_CZ_DEFAULT = 8;
inline int default_tile_cols(int rows) { return rows % 32 == 0 ? 2 : 64; }

// The projector's companion copy of the volume (see launch_project): column
// tiles (1 or 2 detector columns per wave) read a z-fastest copy
// [y][x][z]; row tiles (8 or more columns) read the y-fastest copy [z][x][y]
// for the views whose rays run mostly along x.
__host__ __device__ constexpr bool column_tiles(int pj_wc) { return pj_wc <= 2; }

// The feasible set Q = [lo, hi]^N (lo = 0, hi = +inf: the nonnegative
// orthant) and its projection, a clip evaluated in double.
struct Box {
    double lo, hi;
};
constexpr Box ORTHANT{0.0, __builtin_inf()};

__host__ __device__ __forceinline__ double clip_box(double v, const Box &b)
{
    return v > b.lo ? (v < b.hi ? v : b.hi) : b.lo;
}

// Double-precision reduction results live in fixed slots; every kernel that
// reduces writes one partial per block into partials[slot * pstride + block]
// and finalize_slots() sums each slot in a fixed order.
enum Slot : int {
    S_R2 = 0,        // sum r_i^2 of the projected residual
    S_RD2,           // sum (r_i - rref_i)^2
    S_XD2,           // |xbar - z|^2 (trial)
    S_GD,            // g^T (z - xbar) (trial)
    S_TVB,           // T_tau(xbar) (trial)
    S_BRB,           // Bregman_T(xbar, z) (trial)
    S_GM2,           // |z - P_Q(z - s g)|^2 (GPBB gradient map)
    S_TVY,           // T_tau(y) (gradient pass)
    S_BRY,           // Bregman_T(xref, y) (gradient pass)
    S_XY2,           // |xref - y|^2 (gradient pass)
    S_RY2,           // sum (r_y - r_xbar)^2 (extrapolation)
    S_SS,            // |s|^2 (BB)
    S_SY,            // <s, dg> (BB)
    S_AD1,           // <v, grad T(y)> (TV Hessian pass of the adjoint)
    S_AD2,           // <ybar, x_new - x_old> (extrapolation adjoint)
    S_COUNT
};

struct SlotList {
    int n;
    int slot[S_COUNT];
    int count[S_COUNT];     // partials written for the slot
    double *dst[S_COUNT];   // device destination of the slot's sum
};

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the launch error.  `T` is float (FP32 storage with
// FP64 reductions) or double.

// out = A x (- b); xt, when not NULL, is the companion copy of x for the
// geometry's ray tile (launch_companion).  Without it the walk reads x
// itself (the same values, at a lower rate).
template <typename T>
hipError_t launch_project(const GeomDev &g, const T *x, const T *xt, const T *b, T *out,
                          const T *rref, double *partials, int pstride, hipStream_t st,
                          int *nblocks);

// xc = the companion copy of x for the geometry's ray tile: xc[y][x][z] =
// x[z][y][x] for column tiles, xc[z][x][y] = x[z][y][x] for row tiles
template <typename T>
hipError_t launch_companion(const GeomDev &g, const T *x, T *xc, hipStream_t st);

template <typename T>
hipError_t launch_backproject(const GeomDev &g, const T *r, T *out, hipStream_t st);

// gout = (gin ? gin + alpha * grad T(y) : grad T(y)); slots S_TVY (with
// `value`) and, with xref, S_BRY and S_XY2.  gout may be NULL (value only).
template <typename T>
hipError_t launch_tv(int nx, int ny, int nz, double tau, double alpha, const T *y, const T *xref,
                     const T *gin, T *gout, double *partials, int pstride, hipStream_t st,
                     int *nblocks, bool value = true);

// xbar = P_Q(z - step g); slots S_XD2, S_GD, S_TVB, S_BRB and (gm_step > 0) S_GM2.
template <typename T>
hipError_t launch_trial(int nx, int ny, int nz, double tau, const T *z, const T *g, double step,
                        double gm_step, Box box, T *xbar, double *partials, int pstride,
                        hipStream_t st, int *nblocks);

// y = xn + beta (xn - xo) over n entries; with part != NULL adds sum (y - xn)^2 to S_RY2.
template <typename T>
hipError_t launch_extrapolate(int64_t n, double beta, const T *xn, const T *xo, T *y,
                              double *partials, int pstride, hipStream_t st, int *nblocks);
// the volume's and the residual's extrapolation in one launch (partials of
// the second as launch_extrapolate writes them; *nblocks2 = their count)
template <typename T>
hipError_t launch_extrapolate2(int64_t n1, const T *xn1, const T *xo1, T *y1, int64_t n2,
                               const T *xn2, const T *xo2, T *y2, double beta, double *partials,
                               int pstride, hipStream_t st, int *nblocks2);

// slots S_SS, S_SY of s = x - xp, dg = g - gp.
template <typename T>
hipError_t launch_bb_dots(int64_t n, const T *x, const T *xp, const T *g, const T *gp,
                          double *partials, int pstride, hipStream_t st, int *nblocks);

// out = P_Q(in)
template <typename T>
hipError_t launch_clip(int64_t n, const T *in, T *out, Box box, hipStream_t st);

hipError_t launch_finalize(const SlotList &sl, const double *partials, int pstride,
                           hipStream_t st);

// *out = 0.5 * (*r2) + alpha * (*tv)
hipError_t launch_combine_phi(const double *r2, const double *tv, double alpha, double *out,
                              hipStream_t st);

// ------------------------------------------------- stored system matrix
// x = A^T r from the stored transpose; called by launch_backproject when
// g.mat.present.
template <typename T>
hipError_t launch_backproject_matrix(const GeomDev &g, const T *r, T *out, hipStream_t st);
// entries per voxel (the counting pass of the build)
hipError_t launch_matrix_count(const GeomDev &g, int32_t *cnt_v, hipStream_t st);
// slice widths w[s] = max of cnt (natural voxel order) over the slice's lanes
hipError_t launch_slice_widths(const GeomDev &g, const int32_t *cnt, int32_t *w, hipStream_t st);
// fills values and ray indices at the offsets of g.mat
template <typename T>
hipError_t launch_matrix_fill(const GeomDev &g, T *val_v, int32_t *idx_v, hipStream_t st);

// ---------------------------------------------------- differentiated form
// out = in + ca u + cb w + ch H_T(y) u with H_T the smoothed-TV Hessian
// (in, w may be NULL; out may be in); slot S_AD1 = <u, grad T(y)>.
template <typename T>
hipError_t launch_hessvec(int nx, int ny, int nz, double tau, const T *y, const T *u, const T *in,
                          const T *w, double ca, double cb, double ch, T *out, double *partials,
                          int pstride, hipStream_t st, int *nblocks);
// out = (x > 0) ? g : 0
template <typename T>
hipError_t launch_mask(int64_t n, const T *x, const T *g, T *out, hipStream_t st);
// out = in + a u + b v (NULL operands are zero)
template <typename T>
hipError_t launch_lincomb(int64_t n, const T *in, double a, const T *u, double b, const T *v,
                          T *out, hipStream_t st);
// xbar_n += (1 + beta) ybar, xbar_o -= beta ybar; slot S_AD2 = <ybar, xn - xo>
template <typename T>
hipError_t launch_adj_extrap(int64_t n, double beta, const T *ybar, const T *xn, const T *xo,
                             T *xbar_n, T *xbar_o, double *partials, int pstride, hipStream_t st,
                             int *nblocks);

// grid limits used to size the partial-sum buffer (for the geometry's tile
// shapes; project_blocks_max: the largest over the projector's shapes)
int project_blocks(const GeomDev &g);
int project_blocks_max(const GeomDev &g);
int max_reduce_blocks_vol(int nx, int ny, int nz);
int elementwise_blocks(int64_t n);
int backproject_blocks(const GeomDev &g);
int backproject_depth(const GeomDev &g);  // the geometry's voxel depth: 4, 8 or 16
// Whether the on-the-fly backprojector gathers through the scan's symmetry
// (cone beam with GeomDev sym_rot > 1 or sym_mir), and its blocks.
bool backproject_symmetric(const GeomDev &g);
int backproject_sym_blocks(const GeomDev &g);
int companion_blocks(const GeomDev &g);  // blocks of the grouped companion copy

// ------------------------------------------------------------ batched solve
// One problem of a batch, resident in device memory.  Every phase of a UPN /
// GP round is one grouped launch over all problems; a block finds its
// problem in a prefix table of block counts and reads its operands here.
// The control kernel (one thread per problem) takes the line-search and
// momentum decisions in double and swaps the pointers for the next round,
// so a captured graph of the round can be replayed unchanged.
enum BatchState : int { B_RUNNING = 0, B_CONVERGED = 1, B_NOTCONV = 2, B_STALL = 3 };

template <typename T>
struct BatchProblem {
    GeomDev g;
    int N, m;
    int nb_vox, nb_proj, nb_ew, pstride;
    T *X, *XB, *YB, *G, *XT, *RX, *RXB, *RYB;
    T *Y, *RY;        // current auxiliary point and its residual (alias X/RX or YB/RYB)
    const T *b;
    double *part;     // per-block partial sums [S_COUNT][pstride]
    double *sum;      // finalised sums [S_COUNT]
    double alpha, tau, eps, rho, mu_bar;
    Box box;          // Q
    double L, mu, theta, beta, gm0, gm, phi;
    int method, stop_mode, max_iter, max_trials;
    int state, first, need_grad, ex, distinct, have_ry2, ry2_pending, trials;
    int iters, grad_evals, func_evals;
};

// Grouped launches; offs[p] = first block of problem p (n + 1 entries).  The
// on-the-fly backprojector takes the problems of one voxel depth (4 or 8).
template <typename T>
hipError_t launch_backproject_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                      int depth, hipStream_t st);
// the problems whose on-the-fly gather uses the scan's symmetry (rot, mir)
template <typename T>
hipError_t launch_backproject_sym_grouped(BatchProblem<T> *probs, const int *offs, int n,
                                          int blocks, int rot, int mir, hipStream_t st);
// the problems with a stored transpose (the on-the-fly kernels above take the others)
template <typename T>
hipError_t launch_spmv_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                               hipStream_t st);
int matrix_product_blocks(const GeomDev &g);
template <typename T>
hipError_t launch_tv_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                             hipStream_t st);
template <typename T>
hipError_t launch_trial_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                hipStream_t st);
template <typename T>
hipError_t launch_transpose_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                    hipStream_t st);
// the problems whose ray tile is `cols` columns x `waves` waves per block
// (buf: every problem's volume fits the walk's buffer-resource loads)
template <typename T>
hipError_t launch_project_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                  int cols, int waves, bool buf, hipStream_t st);
template <typename T>
hipError_t launch_extrapolate_grouped(BatchProblem<T> *probs, const int *offs, int n,
                                      int blocks, hipStream_t st);
template <typename T>
hipError_t launch_finalize_grouped(BatchProblem<T> *probs, int n, hipStream_t st);
template <typename T>
hipError_t launch_control_batched(BatchProblem<T> *probs, int n, int *running, hipStream_t st);

}  // namespace tvr

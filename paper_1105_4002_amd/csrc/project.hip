// Forward projector y = A x: one thread per ray, exact path lengths through
// the unit-voxel grid (Siddon's radiological path, walked incrementally).
//
// The paper only calls A "the system matrix" (Sec. II-A) and the data "the
// forward mapping of the discretized image" (Sec. IV-A); the exact
// intersection length of each pixel-centre ray with each voxel is the
// reading taken here.  Ray geometry and the ray sum are double in both
// precisions; only x and the output are stored as T.
//
// Fused epilogue for the solvers: with b the output is the residual
// r = A x - b, and the block writes FP64 partial sums of r_i^2 and, with
// rref, of (r_i - rref_i)^2 (the data part of the Bregman distance used by
// the line search).
#include <algorithm>

#include "ray3d.hpp"
#include "raywalk.hpp"
#include "reduce.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

// Ray tiles.  A wavefront of 64 threads walks the rays of a WC x (64 / WC)
// patch of detector pixels (columns x rows); a block stacks TY such patches
// along the rows.  A wave runs until its longest ray ends, and its lanes
// read the volume together, so a tile trades balance against locality.
// Along a detector row the ray lengths vary widely (a 64 x 1 strip mixes
// rays through the middle of the volume with rays that only clip an edge:
// 77 % of the lane steps are useful at 256^3), while down a detector column
// they barely change (96 %): the rays of one column share their path across
// the xy plane and differ only in slope along z.  Column tiles (WC = 1, 2)
// therefore keep nearly every lane busy, and read the z-fastest companion
// copy [y][x][z], in which the lanes of a wave, at neighbouring heights of
// the same xy cells, touch adjacent addresses.  Row tiles (WC >= 8) read x
// itself, or its y-fastest companion [z][x][y] for views whose rays run
// mostly along x.
template <int WC>
struct RayTile {
    static constexpr int rows = 64 / WC;  // detector rows per wave
};

// Block order.  Logical block L walks the column blocks of one row band
// through every view before moving to the next band: the rays of a band
// cross a thin z-slab of the volume, whatever the view.  The hardware deals
// consecutive blocks round-robin to the 8 XCDs, each with its own L2; the
// launch remaps that so each XCD runs a contiguous range of logical blocks,
// and its L2 holds the slab of its current band instead of the whole
// volume.  A block's work depends only on L (also the index of its partial
// sums), so the batched kernel, which numbers blocks without the remap,
// computes the same values.
constexpr int N_XCD = 8;

__device__ __forceinline__ int xcd_contiguous(int p, int nb)
{
    const int q = nb / N_XCD, rem = nb % N_XCD, k = p % N_XCD;
    return k * q + min(k, rem) + p / N_XCD;
}

__device__ __forceinline__ void decode_block(int L, int gx, int nviews, int &bx, int &by, int &v)
{
    bx = L % gx;
    v = (L / gx) % nviews;
    by = L / (gx * nviews);
}

// One block: WC detector columns x (TY * 64 / WC) rows of view v; BUF picks
// the walk's load path (see ray_walk).
template <typename T, bool CONE, int WC, int TY, bool BUF>
__device__ __forceinline__ void project_block(const GeomDev &g, const T *__restrict__ x,
                                              const T *__restrict__ xt, const T *__restrict__ b,
                                              T *__restrict__ out, const T *__restrict__ rref,
                                              double *__restrict__ partials, int pstride,
                                              int bx, int by, int v, int bid)
{
    const int col0 = bx * WC + (int)threadIdx.x % WC;
    const int row0 = (by * TY + (int)threadIdx.y) * RayTile<WC>::rows + (int)threadIdx.x / WC;
    // a lane past the detector's edge walks the edge ray and writes nothing,
    // so the walk runs outside any divergent branch
    const bool live = col0 < g.cols && row0 < g.rows;
    const int col = min(col0, g.cols - 1), row = min(row0, g.rows - 1);
    double red[2] = {0.0, 0.0};
    {
        ColEntry ce;
        RowEntry re;
        if (g.beam3d) {  // launch-uniform
            ray3d_entries(g, v, row, col, ce, re);
        } else {
            ce = g.col[(size_t)v * g.cols + col];
            re = g.row[row];
        }
        // the companion copy when one is given (block-uniform choice)
        const T *xs = x;
        int sx = 1, sy = g.nx, sz = g.nx * g.ny;
        if (xt != nullptr && column_tiles(WC)) {
            xs = xt;
            sx = g.nz;
            sy = g.nx * g.nz;
            sz = 1;
        } else if (xt != nullptr && fabs(g.cs[v].x) > fabs(g.cs[v].y)) {
            xs = xt;
            sx = g.ny;
            sy = 1;
        }
        const double s = ray_walk<T, CONE, BUF, sizeof(T) == 4 && column_tiles(WC)>(
            g, xs, ce, re, sx, sy, sz);
        if (live) {
            const double dn = CONE ? g.dnorm[(size_t)row * g.cols + col] : g.dnorm[v];
            const size_t i = ((size_t)v * g.rows + row) * g.cols + col;
            double ri = s * dn;
            if (b)
                ri -= (double)b[i];
            out[i] = (T)ri;
            red[0] = ri * ri;
            if (rref) {
                const double d = ri - (double)rref[i];
                red[1] = d * d;
            }
        }
    }
    if (partials) {
        const int slots[2] = {S_R2, S_RD2};
        block_reduce_store<2>(red, partials, pstride, slots, bid);
    }
}

template <typename T, bool CONE, int WC, int TY, bool BUF>
__global__ __launch_bounds__(64 * TY) void project_kernel(GeomDev g, const T *__restrict__ x,
                                                              const T *__restrict__ xt,
                                                              const T *__restrict__ b,
                                                              T *__restrict__ out,
                                                              const T *__restrict__ rref,
                                                              double *__restrict__ partials,
                                                              int pstride)
{
    const int L = xcd_contiguous(blockIdx.x, gridDim.x);
    int bx, by, v;
    decode_block(L, (g.cols + WC - 1) / WC, g.nviews, bx, by, v);
    project_block<T, CONE, WC, TY, BUF>(g, x, xt, b, out, rref, partials, pstride, bx, by, v, L);
}

// Batched: the trial points XB of every running problem (residual against
// b, Bregman data term against RY), one launch per ray tile shape (WC
// columns, TY waves) over the problems of that shape; BUF: every problem's
// volume fits the buffer-resource loads.
template <typename T, int WC, int TY, bool BUF>
__global__ __launch_bounds__(64 * TY) void project_grouped(BatchProblem<T> *probs,
                                                          const int *offs, int n)
{
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING)
        return;
    const int local = blockIdx.x - offs[p];
    int bx, by, v;
    decode_block(local, (P.g.cols + WC - 1) / WC, P.g.nviews, bx, by, v);
    if (P.g.cone)  // block-uniform
        project_block<T, true, WC, TY, BUF>(P.g, P.XB, P.XT, P.b, P.RXB, P.RY, P.part,
                                            P.pstride, bx, by, v, local);
    else
        project_block<T, false, WC, TY, BUF>(P.g, P.XB, P.XT, P.b, P.RXB, P.RY, P.part,
                                             P.pstride, bx, by, v, local);
}

template <typename T, int WC, bool BUF>
hipError_t launch_grouped_wc(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                             int waves, hipStream_t st)
{
    switch (waves) {
    case 1:
        hipLaunchKernelGGL((project_grouped<T, WC, 1, BUF>), dim3(blocks), dim3(64, 1), 0, st, probs,
                           offs, n);
        break;
    case 2:
        hipLaunchKernelGGL((project_grouped<T, WC, 2, BUF>), dim3(blocks), dim3(64, 2), 0, st, probs,
                           offs, n);
        break;
    case 8:
        hipLaunchKernelGGL((project_grouped<T, WC, 8, BUF>), dim3(blocks), dim3(64, 8), 0, st, probs,
                           offs, n);
        break;
    default:
        hipLaunchKernelGGL((project_grouped<T, WC, 4, BUF>), dim3(blocks), dim3(64, 4), 0, st, probs,
                           offs, n);
        break;
    }
    return hipGetLastError();
}

template <typename T, bool BUF>
hipError_t launch_grouped_buf(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                              int cols, int waves, hipStream_t st)
{
    switch (cols) {
    case 1:
        return launch_grouped_wc<T, 1, BUF>(probs, offs, n, blocks, waves, st);
    case 2:
        return launch_grouped_wc<T, 2, BUF>(probs, offs, n, blocks, waves, st);
    case 8:
        return launch_grouped_wc<T, 8, BUF>(probs, offs, n, blocks, waves, st);
    case 16:
        return launch_grouped_wc<T, 16, BUF>(probs, offs, n, blocks, waves, st);
    case 32:
        return launch_grouped_wc<T, 32, BUF>(probs, offs, n, blocks, waves, st);
    default:
        return launch_grouped_wc<T, 64, BUF>(probs, offs, n, blocks, waves, st);
    }
}

}  // namespace

template <typename T>
hipError_t launch_project_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                  int cols, int waves, bool buf, hipStream_t st)
{
    return buf ? launch_grouped_buf<T, true>(probs, offs, n, blocks, cols, waves, st)
               : launch_grouped_buf<T, false>(probs, offs, n, blocks, cols, waves, st);
}

template hipError_t launch_project_grouped<float>(BatchProblem<float> *, const int *, int, int,
                                                  int, int, bool, hipStream_t);
template hipError_t launch_project_grouped<double>(BatchProblem<double> *, const int *, int, int,
                                                   int, int, bool, hipStream_t);

namespace {

int grid_blocks(const GeomDev &g, int wc, int ty)
{
    const int br = ty * (64 / wc);
    return ((g.cols + wc - 1) / wc) * ((g.rows + br - 1) / br) * g.nviews;
}

template <typename T, int WC, int TY>
void launch_shape(const GeomDev &g, const T *x, const T *xt, const T *b, T *out, const T *rref,
                  double *partials, int pstride, hipStream_t st)
{
    dim3 block(64, TY, 1);
    dim3 grid(grid_blocks(g, WC, TY), 1, 1);  // decoded in the kernel
    const bool buf = walk_buffer_ok(g, sizeof(T));
    if (g.cone && buf)
        hipLaunchKernelGGL((project_kernel<T, true, WC, TY, true>), grid, block, 0, st, g, x, xt,
                           b, out, rref, partials, pstride);
    else if (g.cone)
        hipLaunchKernelGGL((project_kernel<T, true, WC, TY, false>), grid, block, 0, st, g, x, xt,
                           b, out, rref, partials, pstride);
    else if (buf)
        hipLaunchKernelGGL((project_kernel<T, false, WC, TY, true>), grid, block, 0, st, g, x,
                           xt, b, out, rref, partials, pstride);
    else
        hipLaunchKernelGGL((project_kernel<T, false, WC, TY, false>), grid, block, 0, st, g, x,
                           xt, b, out, rref, partials, pstride);
}

template <typename T, int WC>
void launch_wc(const GeomDev &g, const T *x, const T *xt, const T *b, T *out, const T *rref,
               double *partials, int pstride, hipStream_t st)
{
    switch (g.pj_ty) {
    case 1:
        launch_shape<T, WC, 1>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    case 2:
        launch_shape<T, WC, 2>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    case 8:
        launch_shape<T, WC, 8>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    default:
        launch_shape<T, WC, 4>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    }
}

int valid_ty(int ty) { return ty == 1 || ty == 2 || ty == 8 ? ty : 4; }
int valid_wc(int wc) { return wc == 1 || wc == 2 || wc == 8 || wc == 16 || wc == 32 ? wc : 64; }

}  // namespace

template <typename T>
hipError_t launch_project(const GeomDev &g, const T *x, const T *xt, const T *b, T *out,
                          const T *rref, double *partials, int pstride, hipStream_t st,
                          int *nblocks)
{
    if (nblocks)
        *nblocks = project_blocks(g);
    switch (valid_wc(g.pj_wc)) {
    case 1:
        launch_wc<T, 1>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    case 2:
        launch_wc<T, 2>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    case 8:
        launch_wc<T, 8>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    case 16:
        launch_wc<T, 16>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    case 32:
        launch_wc<T, 32>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    default:
        launch_wc<T, 64>(g, x, xt, b, out, rref, partials, pstride, st);
        break;
    }
    return hipGetLastError();
}

int project_blocks(const GeomDev &g) { return grid_blocks(g, valid_wc(g.pj_wc), valid_ty(g.pj_ty)); }

int project_blocks_max(const GeomDev &g)
{
    int mx = 0;
    for (int wc : {1, 2, 8, 16, 32, 64})  // one wave per block gives the most blocks
        mx = std::max(mx, grid_blocks(g, wc, 1));
    return mx;
}

template hipError_t launch_project<float>(const GeomDev &, const float *, const float *,
                                          const float *, float *, const float *, double *, int,
                                          hipStream_t, int *);
template hipError_t launch_project<double>(const GeomDev &, const double *, const double *,
                                           const double *, double *, const double *, double *,
                                           int, hipStream_t, int *);

}  // namespace tvr

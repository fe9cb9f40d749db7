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
#include "reduce.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

constexpr int PJ_TX = 64;  // detector columns per block (one wavefront)
constexpr int PJ_TY = 4;   // detector rows per block

// Slab entry/exit of the ray with the volume along one axis; a ray parallel
// to the axis (invD = 0) is inside iff S lies in the half-open range.
__device__ __forceinline__ void slab(double lo, double hi, double S, double invD, double o,
                                     double &tmin, double &tmax, bool &hit)
{
    if (invD != 0.0) {
        const double t0 = plane_t(lo, invD, o), t1 = plane_t(hi, invD, o);
        tmin = fmax(tmin, fmin(t0, t1));
        tmax = fmin(tmax, fmax(t0, t1));
    } else {
        hit = hit && (S >= lo) && (S < hi);
    }
}

// Sum of dt * x along the ray inside the volume, dt in units of the ray
// parameter (multiply by |D| for lengths).  Walks voxel to voxel: the next
// crossing of each axis is plane_t(X) of the next plane X, the segment ends
// at the nearest one, and every axis whose crossing is reached advances (a
// tie of two axes is one crossing, so no zero-length piece is visited).
// The exit crossing of each axis is computed with the same formula as the
// slab exit, so no index leaves the volume before t reaches tmax.
// The volume is read through strides (sx, sy) so that a y-fastest copy can
// serve views whose rays run mostly along x (adjacent detector columns then
// touch adjacent addresses).
template <typename T, bool CONE>
__device__ __forceinline__ double ray_walk(const GeomDev &g, const T *__restrict__ x,
                                           const ColEntry &ce, const RowEntry &re, int sx,
                                           int sy)
{
    const double lox = -g.hx, loy = -g.hy, loz = -g.hz;
    double tmin = CONE ? 0.0 : -INFINITY;
    double tmax = CONE ? 1.0 : INFINITY;
    bool hit = true;
    slab(lox, g.hx, ce.Sx, ce.invDx, ce.ox, tmin, tmax, hit);
    slab(loy, g.hy, ce.Sy, ce.invDy, ce.oy, tmin, tmax, hit);
    slab(loz, g.hz, re.Sz, re.invDz, re.oz, tmin, tmax, hit);
    if (!hit || !(tmax > tmin))
        return 0.0;

    // entry voxel (an axis the ray runs parallel to keeps its coordinate;
    // the clamp absorbs rounding at the entry face)
    int ix = (int)floor((ce.invDx != 0.0 ? ce.Sx + tmin * ce.Dx : ce.Sx) - lox);
    int iy = (int)floor((ce.invDy != 0.0 ? ce.Sy + tmin * ce.Dy : ce.Sy) - loy);
    int iz = (int)floor((re.invDz != 0.0 ? re.Sz + tmin * re.Dz : re.Sz) - loz);
    ix = min(max(ix, 0), g.nx - 1);
    iy = min(max(iy, 0), g.ny - 1);
    iz = min(max(iz, 0), g.nz - 1);

    const bool px = ce.Dx > 0.0, py = ce.Dy > 0.0, pz = re.Dz > 0.0;
    const double sxd = px ? 1.0 : -1.0, syd = py ? 1.0 : -1.0, szd = pz ? 1.0 : -1.0;
    double Xn = lox + (double)(ix + (px ? 1 : 0));
    double Yn = loy + (double)(iy + (py ? 1 : 0));
    double Zn = loz + (double)(iz + (pz ? 1 : 0));
    double tnx = ce.invDx != 0.0 ? plane_t(Xn, ce.invDx, ce.ox) : INFINITY;
    double tny = ce.invDy != 0.0 ? plane_t(Yn, ce.invDy, ce.oy) : INFINITY;
    double tnz = re.invDz != 0.0 ? plane_t(Zn, re.invDz, re.oz) : INFINITY;
    const int sz = g.nx * g.ny;
    const int stx = px ? sx : -sx;
    const int sty = py ? sy : -sy;
    const int stz = pz ? sz : -sz;
    const unsigned last = (unsigned)(g.nx * g.ny * g.nz - 1);
    int idx = ix * sx + iy * sy + iz * sz;

    double t = tmin, acc = 0.0;
    const int cap = g.nx + g.ny + g.nz + 2;  // hard bound on the number of voxels
    for (int it = 0; it < cap; ++it) {
        const double tn = fmin(fmin(tnx, tny), fmin(tnz, tmax));
        acc = fma(fmax(tn - t, 0.0), (double)x[min((unsigned)idx, last)], acc);
        t = tn;
        if (!(t < tmax))
            break;
        const bool ax = tnx <= tn, ay = tny <= tn, az = tnz <= tn;
        idx += (ax ? stx : 0) + (ay ? sty : 0) + (az ? stz : 0);
        const double Xa = Xn + sxd, Ya = Yn + syd, Za = Zn + szd;
        const double ta = plane_t(Xa, ce.invDx, ce.ox);
        const double tb = plane_t(Ya, ce.invDy, ce.oy);
        const double tc = plane_t(Za, re.invDz, re.oz);
        Xn = ax ? Xa : Xn;
        Yn = ay ? Ya : Yn;
        Zn = az ? Za : Zn;
        tnx = ax ? ta : tnx;
        tny = ay ? tb : tny;
        tnz = az ? tc : tnz;
    }
    return acc;
}

// One block: PJ_TX detector columns x PJ_TY rows of view v.
template <typename T, bool CONE>
__device__ __forceinline__ void project_block(const GeomDev &g, const T *__restrict__ x,
                                              const T *__restrict__ xt, const T *__restrict__ b,
                                              T *__restrict__ out, const T *__restrict__ rref,
                                              double *__restrict__ partials, int pstride,
                                              int bx, int by, int v, int bid)
{
    const int col = bx * PJ_TX + threadIdx.x;
    const int row = by * PJ_TY + threadIdx.y;
    double red[2] = {0.0, 0.0};
    if (col < g.cols && row < g.rows) {
        const ColEntry ce = g.col[(size_t)v * g.cols + col];
        const RowEntry re = g.row[row];
        // rays mostly along x read the y-fastest copy when one is given
        const double cv = g.cs[v].x, sv = g.cs[v].y;
        const bool use_t = xt != nullptr && fabs(cv) > fabs(sv);
        const double s = ray_walk<T, CONE>(g, use_t ? xt : x, ce, re, use_t ? g.ny : 1,
                                           use_t ? 1 : g.nx);
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
    if (partials) {
        const int slots[2] = {S_R2, S_RD2};
        block_reduce_store<2>(red, partials, pstride, slots, bid);
    }
}

template <typename T, bool CONE>
__global__ __launch_bounds__(PJ_TX *PJ_TY) void project_kernel(GeomDev g, const T *__restrict__ x,
                                                              const T *__restrict__ xt,
                                                              const T *__restrict__ b,
                                                              T *__restrict__ out,
                                                              const T *__restrict__ rref,
                                                              double *__restrict__ partials,
                                                              int pstride)
{
    project_block<T, CONE>(g, x, xt, b, out, rref, partials, pstride, blockIdx.x, blockIdx.y,
                           blockIdx.z, block_linear_id());
}

// Batched: the trial points XB of every running problem (residual against
// b, Bregman data term against RY).
template <typename T>
__global__ __launch_bounds__(PJ_TX *PJ_TY) void project_grouped(BatchProblem<T> *probs,
                                                               const int *offs, int n)
{
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING)
        return;
    const int local = blockIdx.x - offs[p];
    const int gx = (P.g.cols + PJ_TX - 1) / PJ_TX, gy = (P.g.rows + PJ_TY - 1) / PJ_TY;
    const int bx = local % gx, by = (local / gx) % gy, v = local / (gx * gy);
    if (P.g.cone)
        project_block<T, true>(P.g, P.XB, P.XT, P.b, P.RXB, P.RY, P.part, P.pstride, bx, by, v,
                               local);
    else
        project_block<T, false>(P.g, P.XB, P.XT, P.b, P.RXB, P.RY, P.part, P.pstride, bx, by, v,
                                local);
}

}  // namespace

template <typename T>
hipError_t launch_project_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                  hipStream_t st)
{
    hipLaunchKernelGGL((project_grouped<T>), dim3(blocks), dim3(PJ_TX, PJ_TY), 0, st, probs,
                       offs, n);
    return hipGetLastError();
}

template hipError_t launch_project_grouped<float>(BatchProblem<float> *, const int *, int, int,
                                                  hipStream_t);
template hipError_t launch_project_grouped<double>(BatchProblem<double> *, const int *, int, int,
                                                   hipStream_t);

template <typename T>
hipError_t launch_project(const GeomDev &g, const T *x, const T *xt, const T *b, T *out,
                          const T *rref, double *partials, int pstride, hipStream_t st,
                          int *nblocks)
{
    dim3 block(PJ_TX, PJ_TY, 1);
    dim3 grid((g.cols + PJ_TX - 1) / PJ_TX, (g.rows + PJ_TY - 1) / PJ_TY, g.nviews);
    if (nblocks)
        *nblocks = (int)(grid.x * grid.y * grid.z);
    if (g.cone)
        hipLaunchKernelGGL((project_kernel<T, true>), grid, block, 0, st, g, x, xt, b, out,
                           rref, partials, pstride);
    else
        hipLaunchKernelGGL((project_kernel<T, false>), grid, block, 0, st, g, x, xt, b, out,
                           rref, partials, pstride);
    return hipGetLastError();
}

int project_blocks(const GeomDev &g)
{
    return ((g.cols + PJ_TX - 1) / PJ_TX) * ((g.rows + PJ_TY - 1) / PJ_TY) * g.nviews;
}

template hipError_t launch_project<float>(const GeomDev &, const float *, const float *,
                                          const float *, float *, const float *, double *, int,
                                          hipStream_t, int *);
template hipError_t launch_project<double>(const GeomDev &, const double *, const double *,
                                           const double *, double *, const double *, double *,
                                           int, hipStream_t, int *);

}  // namespace tvr

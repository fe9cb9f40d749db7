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

// Sum of dt * x along the ray inside the volume, dt in units of the ray
// parameter (multiply by |D| for lengths).  t(X) = (X - S) * invD is the
// plane-crossing formula shared with the backprojector.
template <typename T, bool CONE>
__device__ __forceinline__ double ray_walk(const GeomDev &g, const T *__restrict__ x,
                                           double Sx, double Sy, double Sz, double Dx,
                                           double Dy, double Dz, double iDx, double iDy,
                                           double iDz)
{
    const double lox = -g.hx, loy = -g.hy, loz = -g.hz;
    double tmin = CONE ? 0.0 : -INFINITY;
    double tmax = CONE ? 1.0 : INFINITY;
    bool hit = true;
    if (Dx != 0.0) {
        double t0 = (lox - Sx) * iDx, t1 = (lox + (double)g.nx - Sx) * iDx;
        tmin = fmax(tmin, fmin(t0, t1));
        tmax = fmin(tmax, fmax(t0, t1));
    } else {
        hit = hit && (Sx >= lox) && (Sx < lox + (double)g.nx);
    }
    if (Dy != 0.0) {
        double t0 = (loy - Sy) * iDy, t1 = (loy + (double)g.ny - Sy) * iDy;
        tmin = fmax(tmin, fmin(t0, t1));
        tmax = fmin(tmax, fmax(t0, t1));
    } else {
        hit = hit && (Sy >= loy) && (Sy < loy + (double)g.ny);
    }
    if (Dz != 0.0) {
        double t0 = (loz - Sz) * iDz, t1 = (loz + (double)g.nz - Sz) * iDz;
        tmin = fmax(tmin, fmin(t0, t1));
        tmax = fmin(tmax, fmax(t0, t1));
    } else {
        hit = hit && (Sz >= loz) && (Sz < loz + (double)g.nz);
    }
    if (!hit || !(tmax > tmin))
        return 0.0;

    // first voxel: the entry point, clamped into the grid
    // (an axis the ray runs parallel to keeps its coordinate; the clamp also
    // guards against S - lo rounding up to the upper face)
    int ix = (int)floor((Dx != 0.0 ? Sx + tmin * Dx : Sx) - lox);
    int iy = (int)floor((Dy != 0.0 ? Sy + tmin * Dy : Sy) - loy);
    int iz = (int)floor((Dz != 0.0 ? Sz + tmin * Dz : Sz) - loz);
    ix = min(max(ix, 0), g.nx - 1);
    iy = min(max(iy, 0), g.ny - 1);
    iz = min(max(iz, 0), g.nz - 1);

    const int sx = Dx > 0.0 ? 1 : -1, sy = Dy > 0.0 ? 1 : -1, sz = Dz > 0.0 ? 1 : -1;
    const int ox = Dx > 0.0 ? 1 : 0, oy = Dy > 0.0 ? 1 : 0, oz = Dz > 0.0 ? 1 : 0;
    double tnx = Dx != 0.0 ? (lox + (double)(ix + ox) - Sx) * iDx : INFINITY;
    double tny = Dy != 0.0 ? (loy + (double)(iy + oy) - Sy) * iDy : INFINITY;
    double tnz = Dz != 0.0 ? (loz + (double)(iz + oz) - Sz) * iDz : INFINITY;
    const int stx = sx, sty = sy * g.nx, stz = sz * g.nx * g.ny;
    int idx = ix + g.nx * (iy + g.ny * iz);

    double t = tmin, acc = 0.0;
    // every pass advances at least one index monotonically, so the walk
    // ends after at most nx + ny + nz passes
    const int cap = g.nx + g.ny + g.nz + 2;
    for (int it = 0; it < cap && t < tmax; ++it) {
        const double tn = fmin(fmin(tnx, tny), fmin(tnz, tmax));
        acc += fmax(tn - t, 0.0) * (double)x[idx];
        t = fmax(t, tn);
        const bool ax = tnx <= tn, ay = tny <= tn, az = tnz <= tn;
        if (ax) {
            ix += sx;
            idx += stx;
            tnx = (lox + (double)(ix + ox) - Sx) * iDx;
        }
        if (ay) {
            iy += sy;
            idx += sty;
            tny = (loy + (double)(iy + oy) - Sy) * iDy;
        }
        if (az) {
            iz += sz;
            idx += stz;
            tnz = (loz + (double)(iz + oz) - Sz) * iDz;
        }
        if ((unsigned)ix >= (unsigned)g.nx || (unsigned)iy >= (unsigned)g.ny ||
            (unsigned)iz >= (unsigned)g.nz)
            break;
    }
    return acc;
}

template <typename T, bool CONE>
__global__ __launch_bounds__(PJ_TX *PJ_TY) void project_kernel(GeomDev g, const T *__restrict__ x,
                                                              const T *__restrict__ b,
                                                              T *__restrict__ out,
                                                              const T *__restrict__ rref,
                                                              double *__restrict__ partials,
                                                              int pstride)
{
    const int col = blockIdx.x * PJ_TX + threadIdx.x;
    const int row = blockIdx.y * PJ_TY + threadIdx.y;
    const int v = blockIdx.z;
    double red[2] = {0.0, 0.0};
    if (col < g.cols && row < g.rows) {
        const ColEntry ce = g.col[(size_t)v * g.cols + col];
        const RowEntry re = g.row[row];
        double s = ray_walk<T, CONE>(g, x, ce.Sx, ce.Sy, re.Sz, ce.Dx, ce.Dy, re.Dz, ce.invDx,
                                     ce.invDy, re.invDz);
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
        block_reduce_store<2>(red, partials, pstride, slots);
    }
}

}  // namespace

template <typename T>
hipError_t launch_project(const GeomDev &g, const T *x, const T *b, T *out, const T *rref,
                          double *partials, int pstride, hipStream_t st, int *nblocks)
{
    dim3 block(PJ_TX, PJ_TY, 1);
    dim3 grid((g.cols + PJ_TX - 1) / PJ_TX, (g.rows + PJ_TY - 1) / PJ_TY, g.nviews);
    if (nblocks)
        *nblocks = (int)(grid.x * grid.y * grid.z);
    if (g.cone)
        hipLaunchKernelGGL((project_kernel<T, true>), grid, block, 0, st, g, x, b, out, rref,
                           partials, pstride);
    else
        hipLaunchKernelGGL((project_kernel<T, false>), grid, block, 0, st, g, x, b, out, rref,
                           partials, pstride);
    return hipGetLastError();
}

int project_blocks(const GeomDev &g)
{
    return ((g.cols + PJ_TX - 1) / PJ_TX) * ((g.rows + PJ_TY - 1) / PJ_TY) * g.nviews;
}

template hipError_t launch_project<float>(const GeomDev &, const float *, const float *, float *,
                                          const float *, double *, int, hipStream_t, int *);
template hipError_t launch_project<double>(const GeomDev &, const double *, const double *,
                                           double *, const double *, double *, int, hipStream_t,
                                           int *);

}  // namespace tvr

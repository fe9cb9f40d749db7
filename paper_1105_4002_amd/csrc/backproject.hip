// Matched backprojector x = A^T r as a deterministic gather.
//
// The data term of grad phi (eq. 1, needed by every method of Sec. III) is
// A^T (A x - b).  Each thread owns one (x, y) voxel column and a chunk of CZ
// voxels along z.  For every view it finds the detector columns whose rays
// can cross the column (the projected footprint of the column's square,
// widened by a tiny margin), evaluates each such ray's entry/exit
// parameters through the square with the projector's own crossing formula
// t(X) = (X - S) * invD, and then, per voxel of the chunk, the detector rows
// whose rays cross that voxel.  The contribution of ray i to voxel j is
// (t_exit - t_enter) |D_i| r_i: the same length the projector's walk assigns
// to (i, j).  Views, columns and rows are visited in a fixed order, so the
// result is bitwise reproducible, and no atomics are used.
#include "reduce.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

constexpr int BP_TX = 16;   // voxel columns per block along x
constexpr int BP_TY = 16;   // ... along y
constexpr int BP_CZ = 8;    // voxels per thread along z

// Candidate index range [lo, hi] of detector samples whose centre
// coordinate, in units of the pitch, lies within [fmin, fmax] (with margin).
__device__ __forceinline__ void index_range(double fmin_, double fmax_, int n, int &lo, int &hi)
{
    const double margin = 1e-6;
    double a = ceil(fmin_ - margin), b = floor(fmax_ + margin);
    a = fmax(a, 0.0);
    b = fmin(b, (double)(n - 1));
    lo = (int)a;
    hi = (int)b;
    if (!(b >= a)) {
        lo = 0;
        hi = -1;
    }
}

template <typename T, bool CONE>
__global__ __launch_bounds__(BP_TX *BP_TY) void backproject_kernel(GeomDev g,
                                                                  const T *__restrict__ r,
                                                                  T *__restrict__ out)
{
    const int ix = blockIdx.x * BP_TX + (threadIdx.x % BP_TX);
    const int iy = blockIdx.y * BP_TY + (threadIdx.x / BP_TX);
    const int iz0 = blockIdx.z * BP_CZ;
    if (ix >= g.nx || iy >= g.ny)
        return;  // no block-level synchronisation below

    double acc[BP_CZ];
#pragma unroll
    for (int k = 0; k < BP_CZ; ++k)
        acc[k] = 0.0;

    const double X0 = -g.hx + (double)ix, X1 = X0 + 1.0;
    const double Y0 = -g.hy + (double)iy, Y1 = Y0 + 1.0;
    const size_t view_stride = (size_t)g.rows * g.cols;

    for (int v = 0; v < g.nviews; ++v) {
        const double c = g.cs[v].x, s = g.cs[v].y;
        // footprint of the column's square on the detector u axis
        const double a00 = -X0 * s + Y0 * c, a10 = -X1 * s + Y0 * c;
        const double a01 = -X0 * s + Y1 * c, a11 = -X1 * s + Y1 * c;
        double umin, umax;
        if (CONE) {
            const double b00 = X0 * c + Y0 * s, b10 = X1 * c + Y0 * s;
            const double b01 = X0 * c + Y1 * s, b11 = X1 * c + Y1 * s;
            const double u00 = g.SDD * a00 / (g.R - b00), u10 = g.SDD * a10 / (g.R - b10);
            const double u01 = g.SDD * a01 / (g.R - b01), u11 = g.SDD * a11 / (g.R - b11);
            umin = fmin(fmin(u00, u10), fmin(u01, u11));
            umax = fmax(fmax(u00, u10), fmax(u01, u11));
        } else {
            umin = fmin(fmin(a00, a10), fmin(a01, a11));
            umax = fmax(fmax(a00, a10), fmax(a01, a11));
        }
        int c_lo, c_hi;
        index_range(umin * g.ipu + g.cu0, umax * g.ipu + g.cu0, g.cols, c_lo, c_hi);
        const T *rv = r + (size_t)v * view_stride;
        const double dnv = CONE ? 0.0 : g.dnorm[v];

        for (int col = c_lo; col <= c_hi; ++col) {
            const ColEntry ce = g.col[(size_t)v * g.cols + col];
            double tl = CONE ? 0.0 : -INFINITY, th = CONE ? 1.0 : INFINITY;
            if (ce.Dx != 0.0) {
                const double t0 = (X0 - ce.Sx) * ce.invDx, t1 = (X1 - ce.Sx) * ce.invDx;
                tl = fmax(tl, fmin(t0, t1));
                th = fmin(th, fmax(t0, t1));
            } else if (!(ce.Sx >= X0 && ce.Sx < X1)) {
                continue;
            }
            if (ce.Dy != 0.0) {
                const double t0 = (Y0 - ce.Sy) * ce.invDy, t1 = (Y1 - ce.Sy) * ce.invDy;
                tl = fmax(tl, fmin(t0, t1));
                th = fmin(th, fmax(t0, t1));
            } else if (!(ce.Sy >= Y0 && ce.Sy < Y1)) {
                continue;
            }
            if (!(th > tl))
                continue;
            const T *rc = rv + col;

            if (CONE) {
                // z(t) = t w_row on this ray; rows reaching voxel layer [Z0, Z1]
                // within t in [tl, th] (tl > 0: the source is outside the volume)
                const double itl = 1.0 / tl, ith = 1.0 / th;
#pragma unroll
                for (int k = 0; k < BP_CZ; ++k) {
                    const int iz = iz0 + k;
                    if (iz < g.nz) {
                        const double Z0 = -g.hz + (double)iz, Z1 = Z0 + 1.0;
                        const double wlo = fmin(Z0 * itl, Z0 * ith);
                        const double whi = fmax(Z1 * itl, Z1 * ith);
                        int r_lo, r_hi;
                        index_range(wlo * g.ipv + g.rv0, whi * g.ipv + g.rv0, g.rows, r_lo, r_hi);
                        for (int row = r_lo; row <= r_hi; ++row) {
                            const RowEntry re = g.row[row];
                            double lo = tl, hi = th;
                            if (re.Dz != 0.0) {
                                const double t0 = (Z0 - re.Sz) * re.invDz;
                                const double t1 = (Z1 - re.Sz) * re.invDz;
                                lo = fmax(lo, fmin(t0, t1));
                                hi = fmin(hi, fmax(t0, t1));
                            } else if (!(re.Sz >= Z0 && re.Sz < Z1)) {
                                continue;
                            }
                            if (hi > lo) {
                                const size_t p = (size_t)row * g.cols;
                                acc[k] += ((hi - lo) * g.dnorm[p + col]) * (double)rc[p];
                            }
                        }
                    }
                }
            } else {
                // parallel rays are horizontal: row belongs to the layer containing Sz
                const double len = (th - tl) * dnv;
#pragma unroll
                for (int k = 0; k < BP_CZ; ++k) {
                    const int iz = iz0 + k;
                    if (iz < g.nz) {
                        const double Z0 = -g.hz + (double)iz, Z1 = Z0 + 1.0;
                        int r_lo, r_hi;
                        index_range(Z0 * g.ipv + g.rv0, Z1 * g.ipv + g.rv0, g.rows, r_lo, r_hi);
                        for (int row = r_lo; row <= r_hi; ++row) {
                            const double sz = g.row[row].Sz;
                            if (sz >= Z0 && sz < Z1)
                                acc[k] += len * (double)rc[(size_t)row * g.cols];
                        }
                    }
                }
            }
        }
    }

    const size_t plane = (size_t)g.nx * g.ny;
#pragma unroll
    for (int k = 0; k < BP_CZ; ++k) {
        const int iz = iz0 + k;
        if (iz < g.nz)
            out[(size_t)iz * plane + (size_t)iy * g.nx + ix] = (T)acc[k];
    }
}

}  // namespace

template <typename T>
hipError_t launch_backproject(const GeomDev &g, const T *r, T *out, hipStream_t st)
{
    dim3 block(BP_TX * BP_TY, 1, 1);
    dim3 grid((g.nx + BP_TX - 1) / BP_TX, (g.ny + BP_TY - 1) / BP_TY,
              (g.nz + BP_CZ - 1) / BP_CZ);
    if (g.cone)
        hipLaunchKernelGGL((backproject_kernel<T, true>), grid, block, 0, st, g, r, out);
    else
        hipLaunchKernelGGL((backproject_kernel<T, false>), grid, block, 0, st, g, r, out);
    return hipGetLastError();
}

template hipError_t launch_backproject<float>(const GeomDev &, const float *, float *,
                                              hipStream_t);
template hipError_t launch_backproject<double>(const GeomDev &, const double *, double *,
                                               hipStream_t);

}  // namespace tvr

// Voxel-driven enumeration of the rays crossing a voxel column, shared by
// the gather backprojector and the system-matrix builder: the detector
// footprint of a column, the candidate index ranges and the exact ray/voxel
// intervals from the ray tables' crossing formula plane_t.
#pragma once

#include "tvreg_internal.hpp"

namespace tvr {

// 1/x to full double accuracy from the hardware estimate and one Newton step
// (only used for candidate ranges, which carry a margin).
__device__ __forceinline__ double rcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(e, y, y);
}

// Candidate index range [lo, hi] of detector samples whose centre
// coordinate, in units of the pitch, lies within [f0, f1] (with margin),
// intersected with [lim_lo, lim_hi].
__device__ __forceinline__ void index_range(double f0, double f1, int lim_lo, int lim_hi,
                                            int &lo, int &hi)
{
    const double margin = 1e-6;
    const double a = fmax(ceil(f0 - margin), (double)lim_lo);
    const double b = fmin(floor(f1 + margin), (double)lim_hi);
    lo = (int)a;
    hi = b >= a ? (int)b : lo - 1;
}

// Footprint of the box [X0, X1] x [Y0, Y1] (any z) on the detector u axis in
// column units, and the box's depth range b = p.e_s (cone).  A linear or
// linear-fractional function of the point takes its extremes at the corners.
template <bool CONE>
__device__ __forceinline__ void u_footprint(const GeomDev &g, double c, double s, double X0,
                                            double X1, double Y0, double Y1, double &f0,
                                            double &f1, double &bmin, double &bmax)
{
    const double a00 = -X0 * s + Y0 * c, a10 = -X1 * s + Y0 * c;
    const double a01 = -X0 * s + Y1 * c, a11 = -X1 * s + Y1 * c;
    double u00 = a00, u10 = a10, u01 = a01, u11 = a11;
    bmin = bmax = 0.0;
    if (CONE) {
        const double b00 = X0 * c + Y0 * s, b10 = X1 * c + Y0 * s;
        const double b01 = X0 * c + Y1 * s, b11 = X1 * c + Y1 * s;
        u00 = g.SDD * a00 * rcp(g.R - b00);
        u10 = g.SDD * a10 * rcp(g.R - b10);
        u01 = g.SDD * a01 * rcp(g.R - b01);
        u11 = g.SDD * a11 * rcp(g.R - b11);
        bmin = fmin(fmin(b00, b10), fmin(b01, b11));
        bmax = fmax(fmax(b00, b10), fmax(b01, b11));
    }
    f0 = fmin(fmin(u00, u10), fmin(u01, u11)) * g.ipu + g.cu0;
    f1 = fmax(fmax(u00, u10), fmax(u01, u11)) * g.ipu + g.cu0;
}

template <typename T, bool CONE>
struct GlobalSrc {
    const GeomDev *g;
    const ColEntry *colv;  // this view's column entries
    const T *rv;           // this view's data
    double dnv;            // parallel beam |D| of the view
    __device__ ColEntry column(int c) const { return colv[c]; }
    __device__ double Sz(int r) const { return g->row[r].Sz; }
    __device__ double invDz(int r) const { return g->row[r].invDz; }
    __device__ double oz_(int r) const { return g->row[r].oz; }
    __device__ double value(int r, int c) const
    {
        const size_t p = (size_t)r * g->cols + c;
        return (double)rv[p] * (CONE ? g->dnorm[p] : dnv);
    }
};

// Exact ray/column interval [tl, th] through the square (cone: clipped to
// the source-detector segment t in [0, 1]); empty when th <= tl.
template <bool CONE>
__device__ __forceinline__ void xy_interval(double X0, double X1, double Y0, double Y1, double Sx,
                                            double Sy, double iDx, double iDy, double ox,
                                            double oy, double &tl, double &th)
{
    tl = CONE ? 0.0 : -INFINITY;
    th = CONE ? 1.0 : INFINITY;
    if (iDx != 0.0) {
        const double t0 = plane_t(X0, iDx, ox), t1 = plane_t(X1, iDx, ox);
        tl = fmax(tl, fmin(t0, t1));
        th = fmin(th, fmax(t0, t1));
    } else if (!(Sx >= X0 && Sx < X1)) {
        th = -INFINITY;
    }
    if (iDy != 0.0) {
        const double t0 = plane_t(Y0, iDy, oy), t1 = plane_t(Y1, iDy, oy);
        tl = fmax(tl, fmin(t0, t1));
        th = fmin(th, fmax(t0, t1));
    } else if (!(Sy >= Y0 && Sy < Y1)) {
        th = -INFINITY;
    }
}

// Generic enumeration of one view's rays through a voxel column chunk (both
// beams, any source of ray tables); detector indices limited to
// [cl0, ch0] x [rl0, rh0].  Calls visit(k, row, col, t_exit - t_enter) for
// every ray with a non-empty interval in voxel iz0 + k.
template <bool CONE, int CZ, class Src, class Visit>
__device__ __forceinline__ void gather_view_visit(const GeomDev &g, const Src &src, double c,
                                                  double s, double X0, double X1, double Y0,
                                                  double Y1, int iz0, int cl0, int ch0, int rl0,
                                                  int rh0, Visit &&visit)
{
    double f0, f1, bmin, bmax;
    u_footprint<CONE>(g, c, s, X0, X1, Y0, Y1, f0, f1, bmin, bmax);
    int c_lo, c_hi;
    index_range(f0, f1, cl0, ch0, c_lo, c_hi);
    for (int col = c_lo; col <= c_hi; ++col) {
        const ColEntry ce = src.column(col);
        double tl, th;
        xy_interval<CONE>(X0, X1, Y0, Y1, ce.Sx, ce.Sy, ce.invDx, ce.invDy, ce.ox, ce.oy, tl, th);
        if (!(th > tl))
            continue;
        const double itl = CONE ? rcp(tl) * g.ipv : 0.0, ith = CONE ? rcp(th) * g.ipv : 0.0;
#pragma unroll
        for (int k = 0; k < CZ; ++k) {
            const int iz = iz0 + k;
            if (iz < g.nz) {
                const double Z0 = -g.hz + (double)iz, Z1 = Z0 + 1.0;
                int r_lo, r_hi;
                if (CONE)   // rows reaching layer [Z0, Z1] have w in [Z0/t, Z1/t]
                    index_range(fmin(Z0 * itl, Z0 * ith) + g.rv0,
                                fmax(Z1 * itl, Z1 * ith) + g.rv0, rl0, rh0, r_lo, r_hi);
                else        // parallel rays are horizontal
                    index_range(Z0 * g.ipv + g.rv0, Z1 * g.ipv + g.rv0, rl0, rh0, r_lo, r_hi);
                for (int row = r_lo; row <= r_hi; ++row) {
                    const double idz = src.invDz(row);
                    double lo = tl, hi = th;
                    if (idz != 0.0) {
                        const double oz = src.oz_(row);
                        const double t0 = plane_t(Z0, idz, oz), t1 = plane_t(Z1, idz, oz);
                        lo = fmax(lo, fmin(t0, t1));
                        hi = fmin(hi, fmax(t0, t1));
                    } else {
                        const double sz = src.Sz(row);
                        if (!(sz >= Z0 && sz < Z1))
                            continue;
                    }
                    if (hi > lo)
                        visit(k, row, col, hi - lo);
                }
            }
        }
    }
}

// Generic gather of one view: acc[k] += sum of length * r |D| over the rays.
template <bool CONE, int CZ, class Src>
__device__ __forceinline__ void gather_view(const GeomDev &g, const Src &src, double c, double s,
                                            double X0, double X1, double Y0, double Y1,
                                            int iz0, int cl0, int ch0, int rl0, int rh0,
                                            double (&acc)[CZ])
{
    gather_view_visit<CONE, CZ>(g, src, c, s, X0, X1, Y0, Y1, iz0, cl0, ch0, rl0, rh0,
                                [&](int k, int row, int col, double len) {
                                    acc[k] = fma(len, src.value(row, col), acc[k]);
                                });
}

}  // namespace tvr

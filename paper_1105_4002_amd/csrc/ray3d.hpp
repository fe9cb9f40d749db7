// The 3D parallel beam of the paper's experiment (Sec. IV-A: parallel rays
// whose view directions are spread over the unit sphere).
//
// View v has a unit direction d and detector axes e_u = e_z x d / |e_z x d|
// (e_x when d runs along z) and e_v = d x e_u; pixel (row, col) is the line
// S + t d with S = u e_u + w e_v.  A ray's table entries (S, d, 1/d and the
// plane offsets -S/d) are formed here from the view's table, by the one
// function both the walk and the voxel-driven gather call, so A and A^T see
// bitwise identical crossing parameters t(X) = fma(X, 1/d, -S/d).
#pragma once

#include "gather.hpp"
#include "raywalk.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

__device__ __forceinline__ void ray3d_entries(const GeomDev &g, int v, int row, int col,
                                              ColEntry &ce, RowEntry &re)
{
    const View3 &q = g.v3[v];
    const double u = ((double)col - g.cu0) * g.pu;
    const double w = ((double)row - g.rv0) * g.pv;
    ce.Sx = fma(w, q.vx, u * q.ux);
    ce.Sy = fma(w, q.vy, u * q.uy);
    re.Sz = fma(w, q.vz, u * q.uz);
    ce.Dx = q.dx;
    ce.Dy = q.dy;
    re.Dz = q.dz;
    ce.invDx = q.idx;
    ce.invDy = q.idy;
    re.invDz = q.idz;
    ce.ox = -ce.Sx * q.idx;
    ce.oy = -ce.Sy * q.idy;
    re.oz = -re.Sz * q.idz;
}

// Voxel-driven enumeration for one view: for each voxel k of the column
// chunk [X0, X1] x [Y0, Y1] x layers iz0 .. iz0 + CZ - 1, the pixels whose
// rays can cross it (the voxel's projection onto e_u and e_v, with the
// candidate margin), then each candidate ray's exact interval through the
// voxel from the slab crossings; visit(k, row, col, len) for every
// non-empty interval, rows then columns.  The interval is the walk's
// segment in that voxel: both take the largest entering and the smallest
// leaving crossing of the same planes.
template <int CZ, class Visit>
__device__ __forceinline__ void gather3d_visit(const GeomDev &g, int v, double X0, double X1,
                                               double Y0, double Y1, int iz0, Visit &&visit)
{
    const View3 &q = g.v3[v];
    const double ur = 0.5 * (fabs(q.ux) + fabs(q.uy) + fabs(q.uz));
    const double wr = 0.5 * (fabs(q.vx) + fabs(q.vy) + fabs(q.vz));
    const double cx = 0.5 * (X0 + X1), cy = 0.5 * (Y0 + Y1);
#pragma unroll
    for (int k = 0; k < CZ; ++k) {
        if (iz0 + k < g.nz) {
            const double Z0 = -g.hz + (double)(iz0 + k), Z1 = Z0 + 1.0;
            const double cz = 0.5 * (Z0 + Z1);
            const double uc = cx * q.ux + cy * q.uy + cz * q.uz;
            const double wc = cx * q.vx + cy * q.vy + cz * q.vz;
            int c_lo, c_hi, r_lo, r_hi;
            index_range((uc - ur) * g.ipu + g.cu0, (uc + ur) * g.ipu + g.cu0, 0, g.cols - 1,
                        c_lo, c_hi);
            index_range((wc - wr) * g.ipv + g.rv0, (wc + wr) * g.ipv + g.rv0, 0, g.rows - 1,
                        r_lo, r_hi);
            for (int row = r_lo; row <= r_hi; ++row)
                for (int col = c_lo; col <= c_hi; ++col) {
                    ColEntry ce;
                    RowEntry re;
                    ray3d_entries(g, v, row, col, ce, re);
                    double tl = -INFINITY, th = INFINITY;
                    bool hit = true;
                    slab(X0, X1, ce.Sx, ce.invDx, ce.ox, tl, th, hit);
                    slab(Y0, Y1, ce.Sy, ce.invDy, ce.oy, tl, th, hit);
                    slab(Z0, Z1, re.Sz, re.invDz, re.oz, tl, th, hit);
                    if (hit && th > tl)
                        visit(k, row, col, th - tl);
                }
        }
    }
}

}  // namespace tvr

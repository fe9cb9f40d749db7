// Siddon walk of the projector: the slab clip of a ray against the volume
// and the voxel-to-voxel traversal, both from the ray tables' crossing
// formula plane_t, with a visitor per voxel segment.
#pragma once

#include "tvreg_internal.hpp"

namespace tvr {

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

// The walk itself.  Calls enter(ix, iy, iz, px, py, pz) once with the entry
// voxel and the direction of travel along each axis (true: increasing
// index), then, voxel by voxel, visit(dt) with dt >= 0 the parameter length
// inside the current voxel (multiply by |D| for the length; dt may be 0 where
// two crossings coincide) followed, unless the ray has left the volume, by
// move(ax, ay, az): which axes' planes the ray crosses into the next voxel.
// The next crossing of each axis is plane_t(X) of the next plane X, the
// segment ends at the nearest one, and every axis whose crossing is reached
// advances (a tie of two axes is one crossing, so no zero-length piece is
// visited).  The exit crossing of each axis is computed with the same formula
// as the slab exit, so no voxel outside the volume is reached before t
// reaches tmax.
template <bool CONE, class Enter, class Visit, class Move>
__device__ __forceinline__ void ray_walk_core(const GeomDev &g, const ColEntry &ce,
                                              const RowEntry &re, Enter &&enter, Visit &&visit,
                                              Move &&move)
{
    const double lox = -g.hx, loy = -g.hy, loz = -g.hz;
    double tmin = CONE ? 0.0 : -INFINITY;
    double tmax = CONE ? 1.0 : INFINITY;
    bool hit = true;
    slab(lox, g.hx, ce.Sx, ce.invDx, ce.ox, tmin, tmax, hit);
    slab(loy, g.hy, ce.Sy, ce.invDy, ce.oy, tmin, tmax, hit);
    slab(loz, g.hz, re.Sz, re.invDz, re.oz, tmin, tmax, hit);
    if (!hit || !(tmax > tmin))
        return;

    // entry voxel (an axis the ray runs parallel to keeps its coordinate;
    // the clamp absorbs rounding at the entry face)
    int ix = (int)floor((ce.invDx != 0.0 ? ce.Sx + tmin * ce.Dx : ce.Sx) - lox);
    int iy = (int)floor((ce.invDy != 0.0 ? ce.Sy + tmin * ce.Dy : ce.Sy) - loy);
    int iz = (int)floor((re.invDz != 0.0 ? re.Sz + tmin * re.Dz : re.Sz) - loz);
    ix = min(max(ix, 0), g.nx - 1);
    iy = min(max(iy, 0), g.ny - 1);
    iz = min(max(iz, 0), g.nz - 1);

    const bool px = ce.Dx > 0.0, py = ce.Dy > 0.0, pz = re.Dz > 0.0;
    enter(ix, iy, iz, px, py, pz);
    // An axis the ray runs parallel to gets the crossing offset +inf:
    // fma(X, 0, +inf) = +inf, so its crossing is never reached.
    const double ox = ce.invDx != 0.0 ? ce.ox : INFINITY;
    const double oy = ce.invDy != 0.0 ? ce.oy : INFINITY;
    const double oz = re.invDz != 0.0 ? re.oz : INFINITY;
    // Plane steps +-1.0 by their high words (the low word of +-1.0 is zero).
    const int hx = px ? 0x3ff00000 : (int)0xbff00000;
    const int hy = py ? 0x3ff00000 : (int)0xbff00000;
    const int hz = pz ? 0x3ff00000 : (int)0xbff00000;
    double Xn = lox + (double)(ix + (px ? 1 : 0));
    double Yn = loy + (double)(iy + (py ? 1 : 0));
    double Zn = loz + (double)(iz + (pz ? 1 : 0));
    double tnx = plane_t(Xn, ce.invDx, ox);
    double tny = plane_t(Yn, ce.invDy, oy);
    double tnz = plane_t(Zn, re.invDz, oz);

    // Every crossing after the first is >= the one before it (fma rounds
    // monotonically and invD has the sign of the plane step), so segment
    // lengths are >= 0; the first crossing may round to before tmin, and
    // starting t at the smaller of the two gives that segment length 0.
    double t = fmin(tmin, fmin(fmin(tnx, tny), fmin(tnz, tmax)));
    const int cap = g.nx + g.ny + g.nz + 2;  // hard bound on the number of voxels
    for (int it = 0; it < cap; ++it) {
        const double tn = fmin(fmin(tnx, tny), fmin(tnz, tmax));
        visit(tn - t);
        t = tn;
        if (!(t < tmax))
            break;
        const bool ax = tnx <= tn, ay = tny <= tn, az = tnz <= tn;
        move(ax, ay, az);
        // every reached axis moves to its next plane and the others add 0;
        // all three crossings are then recomputed, an unmoved plane giving
        // its previous crossing again bit for bit
        Xn += __hiloint2double(ax ? hx : 0, 0);
        Yn += __hiloint2double(ay ? hy : 0, 0);
        Zn += __hiloint2double(az ? hz : 0, 0);
        tnx = plane_t(Xn, ce.invDx, ox);
        tny = plane_t(Yn, ce.invDy, oy);
        tnz = plane_t(Zn, re.invDz, oz);
    }
}

// Visits the ray's voxels in order, calling visit(index, dt) (the walk of
// ray_walk_core with the voxel's index into the volume).  The volume is read
// through strides (sx, sy, sz), so that a copy stored in another axis order
// can serve rays whose neighbours then touch adjacent addresses.  CLAMP
// clamps each visited index to the volume as well (for loads without a
// hardware range check).
template <bool CONE, bool CLAMP, class Visit>
__device__ __forceinline__ void ray_walk_visit(const GeomDev &g, const ColEntry &ce,
                                               const RowEntry &re, int sx, int sy, int sz,
                                               Visit &&visit)
{
    const unsigned last = (unsigned)(g.nx * g.ny * g.nz - 1);
    int idx = 0, stx = 0, sty = 0, stz = 0;
    ray_walk_core<CONE>(
        g, ce, re,
        [&](int ix, int iy, int iz, bool px, bool py, bool pz) {
            stx = px ? sx : -sx;
            sty = py ? sy : -sy;
            stz = pz ? sz : -sz;
            idx = ix * sx + iy * sy + iz * sz;
        },
        [&](double dt) { visit(CLAMP ? min((unsigned)idx, last) : (unsigned)idx, dt); },
        [&](bool ax, bool ay, bool az) {
            idx += (ax ? stx : 0) + (ay ? sty : 0) + (az ? stz : 0);
        });
}

// Loads of x[idx] through a buffer resource: the hardware checks each offset
// against the volume's size (an offset past it reads 0), so the walk needs no
// clamp of its index and addresses with a 32-bit offset.  Word 3 of the
// descriptor is the gfx9-family value for raw dword access (32-bit data
// format, no swizzle).
constexpr int BUF_WORD3 = 0x00020000;

// (`off` in bytes: the walk then keeps its index in bytes, with no scaling per step)
template <typename T>
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned off);
template <>
__device__ __forceinline__ double buf_load<float>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
    return (double)__builtin_bit_cast(float, v);
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Sum of dt * x along the ray (the projector's ray sum before |D|).  With
// BUF (volumes under 2^31 bytes: a buffer offset is a signed 32-bit number)
// x is read through a range-checked buffer resource, otherwise through
// clamped global loads; both read the same values.
template <typename T, bool CONE, bool BUF>
__device__ __forceinline__ double ray_walk(const GeomDev &g, const T *__restrict__ x,
                                           const ColEntry &ce, const RowEntry &re, int sx,
                                           int sy, int sz)
{
    double acc = 0.0;
    if (BUF) {
        const int bytes = (int)(sizeof(T) * (size_t)g.nx * g.ny * g.nz);
        const __amdgpu_buffer_rsrc_t xr =
            __builtin_amdgcn_make_buffer_rsrc((void *)x, (short)0, bytes, BUF_WORD3);
        const int es = (int)sizeof(T);  // strides in bytes
        ray_walk_visit<CONE, false>(g, ce, re, sx * es, sy * es, sz * es,
                                    [&](unsigned off, double dt) {
                                        acc = fma(dt, buf_load<T>(xr, off), acc);
                                    });
    } else {
        ray_walk_visit<CONE, true>(g, ce, re, sx, sy, sz, [&](unsigned idx, double dt) {
            acc = fma(dt, (double)x[idx], acc);
        });
    }
    return acc;
}

// whether a volume of this geometry fits the buffer path
__host__ __device__ __forceinline__ bool walk_buffer_ok(const GeomDev &g, size_t elem)
{
    return elem * (size_t)g.nx * g.ny * g.nz < (size_t(1) << 31);
}

}  // namespace tvr

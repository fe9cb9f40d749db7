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

// One step of the walk: the segment from t to the nearest crossing (its
// parameter length is returned; inside: the ray is still in the volume after
// it), then the move across that crossing into the next voxel.
__device__ __forceinline__ double walk_step(double &t, double tmax, double &Xn, double &Yn,
                                            double &Zn, double &tnx, double &tny, double &tnz,
                                            int &idx, int stx, int sty, int stz, int hx, int hy,
                                            int hz, double ivx, double ivy, double ivz, double ox,
                                            double oy, double oz, bool &inside)
{
    const double tn = fmin(fmin(tnx, tny), fmin(tnz, tmax));
    const double dt = tn - t;
    t = tn;
    inside = t < tmax;
    // inside: tn is one of the three crossings, and if neither x's nor y's,
    // then z's
    const bool ax = tnx <= tn, ay = tny <= tn;
    // y moves where y is reached and x is not, z where neither is: both
    // formed from the wave's lane masks of the two compares (scalar mask
    // operations, no further per-lane compare or select)
    const uint64_t bx = __builtin_amdgcn_ballot_w64(ax), by = __builtin_amdgcn_ballot_w64(ay);
    const bool my = __builtin_amdgcn_inverse_ballot_w64(by & ~bx);
    const bool az = __builtin_amdgcn_inverse_ballot_w64(~(bx | by));
    idx += ax ? stx : (ay ? sty : stz);
    // the moving axis steps to its next plane and the others add 0; all
    // three crossings are then recomputed, an unmoved plane giving its
    // previous crossing again bit for bit
    Xn += __hiloint2double(ax ? hx : 0, 0);
    Yn += __hiloint2double(my ? hy : 0, 0);
    Zn += __hiloint2double(az ? hz : 0, 0);
    tnx = plane_t(Xn, ivx, ox);
    tny = plane_t(Yn, ivy, oy);
    tnz = plane_t(Zn, ivz, oz);
    return dt;
}

// The walk itself: the sum over the ray's voxels, in order, of dt times the
// voxel's value fetch(index), with dt >= 0 the parameter length inside the
// voxel (multiply by |D| for the length; dt may be 0, see below).  The
// volume is read through strides (sx, sy, sz), so that a copy stored in
// another axis order can serve rays whose neighbours then touch adjacent
// addresses; CLAMP clamps each fetched index to the volume as well (for
// loads without a hardware range check; with one, an index off the volume
// reads 0).  The next crossing of each axis is plane_t(X) of the next plane
// X and the segment ends at the nearest one.  One plane is crossed per step:
// where two or three crossings coincide (the ray passes through an edge or a
// corner) the first reached axis in the order x, y, z moves and the next
// step, in the voxel beside the edge, has length 0 -- a zero entry of A,
// which adds nothing to the sum.  The exit crossing of each axis is computed
// with the same formula as the slab exit, so no voxel outside the volume is
// reached before t reaches tmax.
//
// With AHEAD, each step fetches the next voxel's value before it adds the
// current one (the addresses do not depend on the data), so a load has a
// whole step to arrive.  The lanes of a wave then step together until the
// last of their rays has left the volume (a wave-uniform loop, no per-lane
// exit): after its exit crossing a ray's steps have length 0 (every crossing
// is then at or past tmax), and what they fetch, off the volume or not, adds
// nothing.  Without AHEAD a step fetches its own voxel and a lane leaves the
// loop at its exit.  Both add the same terms in the same order.
template <bool CONE, bool CLAMP, bool AHEAD, class Fetch>
__device__ __forceinline__ double ray_walk_sum(const GeomDev &g, const ColEntry &ce,
                                               const RowEntry &re, int sx, int sy, int sz,
                                               Fetch &&fetch)
{
    const double lox = -g.hx, loy = -g.hy, loz = -g.hz;
    double tmin = CONE ? 0.0 : -INFINITY;
    double tmax = CONE ? 1.0 : INFINITY;
    bool hit = true;
    slab(lox, g.hx, ce.Sx, ce.invDx, ce.ox, tmin, tmax, hit);
    slab(loy, g.hy, ce.Sy, ce.invDy, ce.oy, tmin, tmax, hit);
    slab(loz, g.hz, re.Sz, re.invDz, re.oz, tmin, tmax, hit);
    // a ray that misses the volume walks too (no divergent exit before the
    // loop): its tmax is set to its start below, so every step has length 0
    const bool ok = hit && (tmax > tmin);

    // entry voxel (an axis the ray runs parallel to keeps its coordinate;
    // the clamp absorbs rounding at the entry face, and keeps a missing
    // ray's far-off point in range before its conversion to int)
    const auto cell = [](double c, int n) { return (int)fmin(fmax(floor(c), 0.0), n - 1.0); };
    const int ix = cell((ce.invDx != 0.0 ? ce.Sx + tmin * ce.Dx : ce.Sx) - lox, g.nx);
    const int iy = cell((ce.invDy != 0.0 ? ce.Sy + tmin * ce.Dy : ce.Sy) - loy, g.ny);
    const int iz = cell((re.invDz != 0.0 ? re.Sz + tmin * re.Dz : re.Sz) - loz, g.nz);

    // directions of travel (true: increasing index) and the index steps
    const bool px = ce.Dx > 0.0, py = ce.Dy > 0.0, pz = re.Dz > 0.0;
    const int stx = px ? sx : -sx, sty = py ? sy : -sy, stz = pz ? sz : -sz;
    const unsigned last = (unsigned)(g.nx * g.ny * g.nz - 1);
    int idx = ix * sx + iy * sy + iz * sz;
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
    if (!ok)
        tmax = t;
    // hard bound on the steps: each moves one plane, at most n - 1 per axis
    // before the exit crossing
    const int cap = g.nx + g.ny + g.nz + 2;
    const auto at = [&](int i) { return CLAMP ? min((unsigned)i, last) : (unsigned)i; };
    double acc = 0.0;
    if (AHEAD) {
        // four steps per iteration, the fetched values alternating between
        // xa and xb; the wave leaves once none of its rays is still inside
        // after the fourth (a ray that left earlier adds steps of length 0)
        double xa = fetch(at(idx)), xb;
        for (int it = 0;;) {
            bool inside;
            // (two calls, not a loop: the steps' lane-mask operations keep
            // a compiler from unrolling one)
            const auto two = [&]() {
                const double d1 = walk_step(t, tmax, Xn, Yn, Zn, tnx, tny, tnz, idx, stx, sty,
                                            stz, hx, hy, hz, ce.invDx, ce.invDy, re.invDz, ox,
                                            oy, oz, inside);
                xb = fetch(at(idx));
                acc = fma(d1, xa, acc);
                const double d2 = walk_step(t, tmax, Xn, Yn, Zn, tnx, tny, tnz, idx, stx, sty,
                                            stz, hx, hy, hz, ce.invDx, ce.invDy, re.invDz, ox,
                                            oy, oz, inside);
                xa = fetch(at(idx));
                acc = fma(d2, xb, acc);
            };
            two();
            two();
            // one exit test for both conditions (a single uniform branch
            // keeps the step count in a scalar register)
            it += 4;
            if (!((__any(inside) != 0) & (it < cap)))
                break;
        }
    } else {
        bool inside = true;
        const auto one = [&]() {
            const unsigned cur = at(idx);
            const double dt = walk_step(t, tmax, Xn, Yn, Zn, tnx, tny, tnz, idx, stx, sty, stz,
                                        hx, hy, hz, ce.invDx, ce.invDy, re.invDz, ox, oy, oz,
                                        inside);
            acc = fma(dt, fetch(cur), acc);
        };
        // two steps per iteration, called twice as above
        for (int it = 0; it < cap; it += 2) {
            one();
            if (!inside)
                break;
            one();
            if (!inside)
                break;
        }
    }
    return acc;
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
// clamped global loads; both read the same values.  AHEAD selects the walk
// with its loads a step ahead (see ray_walk_sum).  It pays where a wave's
// rays have nearly equal lengths (the column ray tiles) in single
// precision; where they do not (row tiles), or for double (twice the bytes
// per fetch), the lanes that step on past their exit cost more than the
// early loads save.
template <typename T, bool CONE, bool BUF, bool AHEAD>
__device__ __forceinline__ double ray_walk(const GeomDev &g, const T *__restrict__ x,
                                           const ColEntry &ce, const RowEntry &re, int sx,
                                           int sy, int sz)
{
    if (BUF) {
        const int bytes = (int)(sizeof(T) * (size_t)g.nx * g.ny * g.nz);
        const __amdgpu_buffer_rsrc_t xr =
            __builtin_amdgcn_make_buffer_rsrc((void *)x, (short)0, bytes, BUF_WORD3);
        const int es = (int)sizeof(T);  // strides in bytes
        return ray_walk_sum<CONE, false, AHEAD>(
            g, ce, re, sx * es, sy * es, sz * es,
            [&](unsigned off) { return buf_load<T>(xr, off); });
    }
    return ray_walk_sum<CONE, true, AHEAD>(
        g, ce, re, sx, sy, sz, [&](unsigned idx) { return (double)x[idx]; });
}

// whether a volume of this geometry fits the buffer path
__host__ __device__ __forceinline__ bool walk_buffer_ok(const GeomDev &g, size_t elem)
{
    return elem * (size_t)g.nx * g.ny * g.nz < (size_t(1) << 31);
}

}  // namespace tvr

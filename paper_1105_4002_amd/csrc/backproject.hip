// Matched backprojector x = A^T r as a deterministic gather.
//
// The data term of grad phi (eq. 1, needed by every method of Sec. III) is
// A^T (A x - b).  Each thread owns one (x, y) voxel column and a chunk of CZ
// voxels along z.  For every view it finds the detector columns whose rays
// can cross the column (the projected footprint of the column's square,
// widened by a tiny margin), evaluates each such ray's entry/exit
// parameters through the square with the projector's own crossing formula
// plane_t, and then, per voxel of the chunk, the detector rows whose rays
// cross that voxel.  The contribution of ray i to voxel j is
// (t_exit - t_enter) |D_i| r_i: the same length the projector's walk assigns
// to (i, j).  Views, columns and rows are visited in a fixed order, so the
// result is bitwise reproducible, and no atomics are used.
//
// Memory: per view, a block (16 x 16 voxel columns x CZ) stages in LDS the
// detector tile its voxels can see -- r |D| in double, the tile's column ray
// entries (structure of arrays) and row entries -- so the inner loops read
// only LDS.  The cone-beam inner loop is branch free: every candidate row
// gets the exact interval arithmetic, selected to zero where it is empty.
// A view whose footprint exceeds the tile (unusual geometries) takes the
// generic arithmetic with global loads.
#include "reduce.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

constexpr int BP_TX = 16;   // voxel columns per block along x
constexpr int BP_TY = 16;   // ... along y
constexpr int BP_THREADS = BP_TX * BP_TY;
constexpr int BP_CZ = 8;    // voxels per thread along z
constexpr int TILE_C = 48;  // detector columns a block stages per view
constexpr int TILE_R = 32;  // detector rows a block stages per view
constexpr int TILE_S = TILE_C + 1;  // odd row stride (in doubles) against bank conflicts

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

// The block's LDS copy of one view.
struct Tile {
    double rt[TILE_R * TILE_S];                     // r |D|, [row - R0][col - C0]
    double Sx[TILE_C], Sy[TILE_C], iDx[TILE_C], iDy[TILE_C], ox[TILE_C], oy[TILE_C];
    double Sz[TILE_R], iDz[TILE_R], oz[TILE_R];
};

// Data sources of the generic gather: the block's tile, or global memory.
struct TileSrc {
    const Tile *t;
    int C0, R0;
    __device__ ColEntry column(int c) const
    {
        const int j = c - C0;
        ColEntry e;
        e.Sx = t->Sx[j];
        e.Sy = t->Sy[j];
        e.Dx = e.Dy = 0.0;
        e.invDx = t->iDx[j];
        e.invDy = t->iDy[j];
        e.ox = t->ox[j];
        e.oy = t->oy[j];
        return e;
    }
    __device__ double Sz(int r) const { return t->Sz[r - R0]; }
    __device__ double invDz(int r) const { return t->iDz[r - R0]; }
    __device__ double oz_(int r) const { return t->oz[r - R0]; }
    __device__ double value(int r, int c) const { return t->rt[(r - R0) * TILE_S + (c - C0)]; }
};

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

// Generic gather of one view (both beams, any data source); detector
// indices limited to [cl0, ch0] x [rl0, rh0].
template <bool CONE, int CZ, class Src>
__device__ __forceinline__ void gather_view(const GeomDev &g, const Src &src, double c, double s,
                                            double X0, double X1, double Y0, double Y1,
                                            int iz0, int cl0, int ch0, int rl0, int rh0,
                                            double (&acc)[CZ])
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
                        acc[k] = fma(hi - lo, src.value(row, col), acc[k]);
                }
            }
        }
    }
}

// Cone-beam gather of one view from the block's tile.  The source sits at
// z = 0 (Sz = 0, so the plane parameter is Z * invDz; a row with w = 0 runs
// in the plane z = 0 and belongs to the layer containing 0).
template <int CZ>
__device__ __forceinline__ void cone_row(const Tile &T_, int row, int R0, int cc, double Z0,
                                         double Z1, double tl, double th, bool in0, bool ok,
                                         double &acc)
{
    const int rr = ok ? row - R0 : 0;
    const double val = T_.rt[rr * TILE_S + cc];
    const double idz = T_.iDz[rr];
    const double t0 = Z0 * idz, t1 = Z1 * idz;
    const double lo = fmax(tl, fmin(t0, t1)), hi = fmin(th, fmax(t0, t1));
    double len = idz != 0.0 ? hi - lo : (in0 ? th - tl : 0.0);
    len = ok ? len : 0.0;
    acc += len > 0.0 ? len * val : 0.0;
}

template <int CZ>
__device__ __forceinline__ void gather_cone_tile(const GeomDev &g, const Tile &T_, double c,
                                                 double s, double X0, double X1, double Y0,
                                                 double Y1, int iz0, int C0, int C1, int R0,
                                                 int R1, double (&acc)[CZ])
{
    double f0, f1, bmin, bmax;
    u_footprint<true>(g, c, s, X0, X1, Y0, Y1, f0, f1, bmin, bmax);
    int c_lo, c_hi;
    index_range(f0, f1, C0, C1, c_lo, c_hi);
    for (int col = c_lo; col <= c_hi; ++col) {
        const int cc = col - C0;
        double tl, th;
        xy_interval<true>(X0, X1, Y0, Y1, T_.Sx[cc], T_.Sy[cc], T_.iDx[cc], T_.iDy[cc], T_.ox[cc],
                          T_.oy[cc], tl, th);
        if (!(th > tl))
            continue;
        // z(t) = t w: rows reaching layer [Z0, Z1] within t in [tl, th]
        // have w in [Z0/t, Z1/t] (tl > 0: the source is outside the volume)
        const double itl = rcp(tl) * g.ipv, ith = rcp(th) * g.ipv;
        double Z0 = -g.hz + (double)iz0;
        double qa = Z0 * itl, qb = Z0 * ith;
#pragma unroll
        for (int k = 0; k < CZ; ++k) {
            const double Z1 = Z0 + 1.0;
            const double pa = Z1 * itl, pb = Z1 * ith;
            if (iz0 + k < g.nz) {  // block-uniform
                int r_lo, r_hi;
                index_range(fmin(qa, qb) + g.rv0, fmax(pa, pb) + g.rv0, R0, R1, r_lo, r_hi);
                const bool in0 = Z0 <= 0.0 && 0.0 < Z1;
                cone_row<CZ>(T_, r_lo, R0, cc, Z0, Z1, tl, th, in0, r_lo <= r_hi, acc[k]);
                cone_row<CZ>(T_, r_lo + 1, R0, cc, Z0, Z1, tl, th, in0, r_lo + 1 <= r_hi, acc[k]);
                for (int row = r_lo + 2; row <= r_hi; ++row)  // wide footprints only
                    cone_row<CZ>(T_, row, R0, cc, Z0, Z1, tl, th, in0, true, acc[k]);
            }
            Z0 = Z1;
            qa = pa;
            qb = pb;
        }
    }
}

// One block: BP_TX x BP_TY voxel columns, CZ voxels deep, block (bx, by, bz).
template <typename T, bool CONE, int CZ>
__device__ __forceinline__ void backproject_block(const GeomDev &g, const T *__restrict__ r,
                                                  T *__restrict__ out, int bx, int by, int bz,
                                                  Tile &tile)
{
    const int tid = threadIdx.x;
    const int ix = bx * BP_TX + (tid % BP_TX);
    const int iy = by * BP_TY + (tid / BP_TX);
    const int iz0 = bz * CZ;
    // threads past the volume edge still stage data and meet every barrier
    const bool active = ix < g.nx && iy < g.ny;

    double acc[CZ];
#pragma unroll
    for (int k = 0; k < CZ; ++k)
        acc[k] = 0.0;

    const double X0 = -g.hx + (double)ix, X1 = X0 + 1.0;
    const double Y0 = -g.hy + (double)iy, Y1 = Y0 + 1.0;
    // the block's box
    const double bX0 = -g.hx + (double)(bx * BP_TX);
    const double bY0 = -g.hy + (double)(by * BP_TY);
    const double bZ0 = -g.hz + (double)iz0;
    const double bX1 = fmin(bX0 + BP_TX, g.hx), bY1 = fmin(bY0 + BP_TY, g.hy);
    const double bZ1 = fmin(bZ0 + CZ, g.hz);
    const size_t view_stride = (size_t)g.rows * g.cols;

    for (int v = 0; v < g.nviews; ++v) {
        const double c = g.cs[v].x, s = g.cs[v].y;
        double f0, f1, bmin, bmax;
        u_footprint<CONE>(g, c, s, bX0, bX1, bY0, bY1, f0, f1, bmin, bmax);
        int C0, C1, R0, R1;
        index_range(f0, f1, 0, g.cols - 1, C0, C1);
        if (CONE) {
            // w = SDD z / (R - b): extremes at the corners of [bZ0, bZ1] x [bmin, bmax]
            const double i0 = g.SDD * rcp(g.R - bmin), i1 = g.SDD * rcp(g.R - bmax);
            const double wlo = fmin(bZ0 * i0, bZ0 * i1), whi = fmax(bZ1 * i0, bZ1 * i1);
            index_range(wlo * g.ipv + g.rv0, whi * g.ipv + g.rv0, 0, g.rows - 1, R0, R1);
        } else {
            index_range(bZ0 * g.ipv + g.rv0, bZ1 * g.ipv + g.rv0, 0, g.rows - 1, R0, R1);
        }
        const int nc = C1 - C0 + 1, nr = R1 - R0 + 1;
        if (nc <= 0 || nr <= 0)
            continue;  // block-uniform: nothing of this view reaches the block
        const T *rv = r + (size_t)v * view_stride;
        const double dnv = CONE ? 1.0 : g.dnorm[v];
        if (nc <= TILE_C && nr <= TILE_R) {
            for (int i = tid; i < nr * nc; i += BP_THREADS) {
                const int rr = i / nc, cc = i - rr * nc;
                const size_t p = (size_t)(R0 + rr) * g.cols + (C0 + cc);
                tile.rt[rr * TILE_S + cc] = (double)rv[p] * (CONE ? g.dnorm[p] : dnv);
            }
            for (int i = tid; i < nc; i += BP_THREADS) {
                const ColEntry e = g.col[(size_t)v * g.cols + C0 + i];
                tile.Sx[i] = e.Sx;
                tile.Sy[i] = e.Sy;
                tile.iDx[i] = e.invDx;
                tile.iDy[i] = e.invDy;
                tile.ox[i] = e.ox;
                tile.oy[i] = e.oy;
            }
            for (int i = tid; i < nr; i += BP_THREADS) {
                const RowEntry e = g.row[R0 + i];
                tile.Sz[i] = e.Sz;
                tile.iDz[i] = e.invDz;
                tile.oz[i] = e.oz;
            }
            __syncthreads();
            if (active) {
                if (CONE) {
                    gather_cone_tile<CZ>(g, tile, c, s, X0, X1, Y0, Y1, iz0, C0, C1, R0, R1, acc);
                } else {
                    const TileSrc src{&tile, C0, R0};
                    gather_view<false, CZ>(g, src, c, s, X0, X1, Y0, Y1, iz0, C0, C1, R0, R1,
                                           acc);
                }
            }
            __syncthreads();
        } else if (active) {
            const GlobalSrc<T, CONE> src{&g, g.col + (size_t)v * g.cols, rv, dnv};
            gather_view<CONE, CZ>(g, src, c, s, X0, X1, Y0, Y1, iz0, 0, g.cols - 1, 0,
                                  g.rows - 1, acc);
        }
    }

    if (active) {
        const size_t plane = (size_t)g.nx * g.ny;
#pragma unroll
        for (int k = 0; k < CZ; ++k) {
            const int iz = iz0 + k;
            if (iz < g.nz)
                out[(size_t)iz * plane + (size_t)iy * g.nx + ix] = (T)acc[k];
        }
    }
}

template <typename T, bool CONE, int CZ>
__global__ __launch_bounds__(BP_THREADS) void backproject_kernel(GeomDev g,
                                                                const T *__restrict__ r,
                                                                T *__restrict__ out)
{
    __shared__ Tile tile;
    backproject_block<T, CONE, CZ>(g, r, out, blockIdx.x, blockIdx.y, blockIdx.z, tile);
}

// Batched: G = A^T RY for every problem whose gradient is due this round.
template <typename T>
__global__ __launch_bounds__(BP_THREADS) void backproject_grouped(BatchProblem<T> *probs,
                                                                 const int *offs, int n)
{
    __shared__ Tile tile;
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING || !P.need_grad)
        return;
    const int local = blockIdx.x - offs[p];
    const int gx = (P.g.nx + BP_TX - 1) / BP_TX, gy = (P.g.ny + BP_TY - 1) / BP_TY;
    const int bx = local % gx, by = (local / gx) % gy, bz = local / (gx * gy);
    if (P.g.cone)
        backproject_block<T, true, BP_CZ>(P.g, P.RY, P.G, bx, by, bz, tile);
    else
        backproject_block<T, false, BP_CZ>(P.g, P.RY, P.G, bx, by, bz, tile);
}

}  // namespace

int backproject_blocks(const GeomDev &g)
{
    return ((g.nx + BP_TX - 1) / BP_TX) * ((g.ny + BP_TY - 1) / BP_TY) *
           ((g.nz + BP_CZ - 1) / BP_CZ);
}

template <typename T>
hipError_t launch_backproject_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                      hipStream_t st)
{
    hipLaunchKernelGGL((backproject_grouped<T>), dim3(blocks), dim3(BP_THREADS), 0, st, probs,
                       offs, n);
    return hipGetLastError();
}

template hipError_t launch_backproject_grouped<float>(BatchProblem<float> *, const int *, int,
                                                      int, hipStream_t);
template hipError_t launch_backproject_grouped<double>(BatchProblem<double> *, const int *, int,
                                                       int, hipStream_t);

template <typename T>
hipError_t launch_backproject(const GeomDev &g, const T *r, T *out, hipStream_t st)
{
    dim3 block(BP_THREADS, 1, 1);
    dim3 grid((g.nx + BP_TX - 1) / BP_TX, (g.ny + BP_TY - 1) / BP_TY,
              (g.nz + BP_CZ - 1) / BP_CZ);
    if (g.cone)
        hipLaunchKernelGGL((backproject_kernel<T, true, BP_CZ>), grid, block, 0, st, g, r, out);
    else
        hipLaunchKernelGGL((backproject_kernel<T, false, BP_CZ>), grid, block, 0, st, g, r, out);
    return hipGetLastError();
}

template hipError_t launch_backproject<float>(const GeomDev &, const float *, float *,
                                              hipStream_t);
template hipError_t launch_backproject<double>(const GeomDev &, const double *, double *,
                                               hipStream_t);

}  // namespace tvr

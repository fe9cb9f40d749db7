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
// only LDS.  The cone-beam inner loop is branch free: the two candidate rows
// of each layer get the exact interval arithmetic, a row outside the range
// reads the tile's zero row, and a non-positive length adds nothing.
// A cone-beam view whose footprint exceeds the tile is gathered tile by
// tile; a parallel-beam one takes the generic arithmetic with global loads.
#include "gather.hpp"
#include "ray3d.hpp"
#include "reduce.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

constexpr int BP_TX = 16;   // voxel columns per block along x
constexpr int BP_TY = 16;   // ... along y
constexpr int BP_THREADS = BP_TX * BP_TY;
constexpr int TILE_C = 48;  // detector columns a block stages per view
constexpr int TILE_R = 32;  // detector rows a block stages per view
constexpr int TILE_S = TILE_C + 1;  // odd row stride (in doubles) against bank conflicts
// A flat detector row (invDz = 0: its rays run in the plane w = 0) is staged
// with this huge finite 1/Dz: its crossing parameters Z0 / Dz, Z1 / Dz are
// then -huge, 0 or +huge (|Z| FLAT_IDZ stays finite), and the interval clip
// leaves the whole xy interval th - tl exactly when Z0 <= 0 < Z1 and nothing
// otherwise -- the flat row's length, with no separate path.
constexpr double FLAT_IDZ = 1e300;

// The block's LDS copy of one view.  Row TILE_R of rt and iDz is a zero row
// (value 0, slope 1) that the cone gather reads for candidate rows outside
// a voxel's range: it adds exactly nothing.
struct Tile {
    double rt[(TILE_R + 1) * TILE_S];               // r |D|, [row - R0][col - C0]
    double Sx[TILE_C], Sy[TILE_C], iDx[TILE_C], iDy[TILE_C], ox[TILE_C], oy[TILE_C];
    double Sz[TILE_R], iDz[TILE_R + 1], oz[TILE_R];
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

// Cone-beam gather of one view from the block's tile.  The source sits at
// z = 0 (Sz = 0, so the plane parameter is Z * invDz; a flat row carries
// FLAT_IDZ).  A candidate row outside the voxel's range (ok false) reads the
// tile's zero row.  The interval length is clamped at 0 and weights the
// value in one fma.
__device__ __forceinline__ void cone_row(const Tile &T_, int rel, int cc, double Z0, double Z1,
                                         double tl, double th, bool ok, double &acc)
{
    const int rr = ok ? rel : TILE_R;
    const double val = T_.rt[rr * TILE_S + cc];
    const double idz = T_.iDz[rr];
    const double t0 = Z0 * idz, t1 = Z1 * idz;
    const double lo = fmax(tl, fmin(t0, t1)), hi = fmin(th, fmax(t0, t1));
    acc = fma(fmax(hi - lo, 0.0), val, acc);
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
    // row coordinate w / pv + rv0, shifted to the tile and widened by the
    // candidate margin, and the tile's last row
    const double row_lo_off = g.rv0 - (double)R0 - 1e-6, row_hi_off = g.rv0 - (double)R0 + 1e-6;
    const double row_last = (double)(R1 - R0);
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
                // candidate rows relative to the tile (empty when hi < lo)
                const int lo = (int)fmax(ceil(fmin(qa, qb) + row_lo_off), 0.0);
                const int hi = (int)fmin(floor(fmax(pa, pb) + row_hi_off), row_last);
                cone_row(T_, lo, cc, Z0, Z1, tl, th, lo <= hi, acc[k]);
                cone_row(T_, lo + 1, cc, Z0, Z1, tl, th, lo + 1 <= hi, acc[k]);
                for (int rel = lo + 2; rel <= hi; ++rel)  // wide footprints only
                    cone_row(T_, rel, cc, Z0, Z1, tl, th, true, acc[k]);
            }
            Z0 = Z1;
            qa = pa;
            qb = pb;
        }
    }
}

// One block: BP_TX x BP_TY voxel columns, CZ voxels deep, block (bx, by, bz).
// The 3D parallel beam: the same thread layout, each voxel's rays found by
// the voxel-driven enumeration of ray3d.hpp (no detector tile staging: a
// view's footprint on the block is not a row x column rectangle).
template <typename T, int CZ>
__device__ __forceinline__ void backproject_block3d(const GeomDev &g, const T *__restrict__ r,
                                                    T *__restrict__ out, int bx, int by, int bz)
{
    const int tid = threadIdx.x;
    const int ix = bx * BP_TX + (tid % BP_TX);
    const int iy = by * BP_TY + (tid / BP_TX);
    const int iz0 = bz * CZ;
    if (ix >= g.nx || iy >= g.ny)
        return;
    double acc[CZ];
#pragma unroll
    for (int k = 0; k < CZ; ++k)
        acc[k] = 0.0;
    const double X0 = -g.hx + (double)ix, X1 = X0 + 1.0;
    const double Y0 = -g.hy + (double)iy, Y1 = Y0 + 1.0;
    const size_t view_stride = (size_t)g.rows * g.cols;
    for (int v = 0; v < g.nviews; ++v) {
        const T *rv = r + (size_t)v * view_stride;
        const double dnv = g.dnorm[v];
        gather3d_visit<CZ>(g, v, X0, X1, Y0, Y1, iz0, [&](int k, int row, int col, double len) {
            acc[k] += len * ((double)rv[(size_t)row * g.cols + col] * dnv);
        });
    }
    const size_t plane = (size_t)g.nx * g.ny;
#pragma unroll
    for (int k = 0; k < CZ; ++k)
        if (iz0 + k < g.nz)
            out[(size_t)(iz0 + k) * plane + (size_t)iy * g.nx + ix] = (T)acc[k];
}

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
    if (CONE) {  // the zero row; the first view's barrier orders it before any read
        for (int i = tid; i < TILE_S; i += BP_THREADS)
            tile.rt[TILE_R * TILE_S + i] = 0.0;
        if (tid == 0)
            tile.iDz[TILE_R] = 1.0;
    }

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
        // the view's detector rectangle rows rb..re x columns cb..ce into the tile
        const auto stage = [&](int cb, int rb, int ncs, int nrs) {
            for (int i = tid; i < nrs * ncs; i += BP_THREADS) {
                const int rr = i / ncs, cc = i - rr * ncs;
                const size_t p = (size_t)(rb + rr) * g.cols + (cb + cc);
                tile.rt[rr * TILE_S + cc] = (double)rv[p] * (CONE ? g.dnorm[p] : dnv);
            }
            for (int i = tid; i < ncs; i += BP_THREADS) {
                const ColEntry e = g.col[(size_t)v * g.cols + cb + i];
                tile.Sx[i] = e.Sx;
                tile.Sy[i] = e.Sy;
                tile.iDx[i] = e.invDx;
                tile.iDy[i] = e.invDy;
                tile.ox[i] = e.ox;
                tile.oy[i] = e.oy;
            }
            for (int i = tid; i < nrs; i += BP_THREADS) {
                const RowEntry e = g.row[rb + i];
                tile.Sz[i] = e.Sz;
                // cone: a flat row (invDz = 0) gets a huge finite 1/Dz, whose
                // clip in cone_row gives its length (see FLAT_IDZ)
                tile.iDz[i] = CONE && e.invDz == 0.0 ? FLAT_IDZ : e.invDz;
                tile.oz[i] = e.oz;
            }
        };
        if (CONE) {
            // One path per view: the footprint in tiles (one when it fits;
            // else column-major chunks of TILE_C columns by TILE_R rows).  A
            // second path in the loop would hold the accumulators in other
            // registers on each and pay moves between them per view.
            for (int cb = C0; cb <= C1; cb += TILE_C) {  // block-uniform
                const int ce = min(cb + TILE_C - 1, C1);
                for (int rb = R0; rb <= R1; rb += TILE_R) {
                    const int re = min(rb + TILE_R - 1, R1);
                    stage(cb, rb, ce - cb + 1, re - rb + 1);
                    __syncthreads();
                    if (active)
                        gather_cone_tile<CZ>(g, tile, c, s, X0, X1, Y0, Y1, iz0, cb, ce, rb, re,
                                             acc);
                    __syncthreads();
                }
            }
        } else if (nc <= TILE_C && nr <= TILE_R) {
            stage(C0, R0, nc, nr);
            __syncthreads();
            if (active) {
                const TileSrc src{&tile, C0, R0};
                gather_view<false, CZ>(g, src, c, s, X0, X1, Y0, Y1, iz0, C0, C1, R0, R1, acc);
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

// ------------------------------------------------------------ symmetric scan
// A circular cone scan with the quarter-turn (or half-turn) symmetry and / or
// the z mirror of GeomDev sym_rot / sym_mir (the group the stored transpose
// uses): the rays through the image of voxel j under q turns, in view
// v + q V / ROT, are the rays through j in view v, with the same lengths, and
// the rays through its mirror image z -> -z are those of the mirrored
// detector rows R - 1 - row, with the same |D|.  A thread of the symmetric
// gather owns a voxel column of the cell the images tile the volume from
// (the stored transpose's cell), finds its rays and lengths once per view,
// and applies them to all NI = ROT (x 2 with the mirror) images, reading
// each image's detector tile -- the rotated views, the mirrored rows --
// from LDS (r |D| in double, as the plain gather stages it).  Each image
// sums its views in the order v + q V / ROT, v = 0 .. V - 1 (the identity
// image: the plain gather's order and values, wherever a view's footprint
// fits one tile; a larger one is gathered in tiles, its rows in a different
// order).
constexpr int STILE_R = 16;  // detector rows the symmetric gather stages per view
constexpr int STILE_C = 44;  // ... and columns
constexpr int STILE_S = STILE_C + 1;  // odd row stride (in doubles)

template <int NI>
struct SymTile {
    // r |D| of images 2p and 2p + 1 at [row - R0][col - C0] (one 16-byte LDS
    // read serves both); row STILE_R: 0
    double2 rt[NI / 2][(STILE_R + 1) * STILE_S];
    double Sx[STILE_C], Sy[STILE_C], iDx[STILE_C], iDy[STILE_C], ox[STILE_C], oy[STILE_C];
    double iDz[STILE_R + 1];
};

// One detector row of one column for voxel layer k: the ray's length in
// the voxel (its xy interval [tl, th] clipped by the layer's crossings
// Z / Dz; the flat row's huge 1/Dz gives th - tl or 0) applied to the NI
// images.  A row past the footprint (ok false) reads the zero row.
template <int NI, int CZ>
__device__ __forceinline__ void sym_row(const SymTile<NI> &S, int rel, int cc, double Z0,
                                        double Z1, double tl, double th, bool ok,
                                        double (&acc)[NI][CZ], int k)
{
    const int o = (ok ? rel : STILE_R) * STILE_S + cc;
    const double idz = S.iDz[ok ? rel : STILE_R];
    const double t0 = Z0 * idz, t1 = Z1 * idz;
    const double lo = fmax(tl, fmin(t0, t1)), hi = fmin(th, fmax(t0, t1));
    const double len = fmax(hi - lo, 0.0);
#pragma unroll
    for (int i = 0; i < NI / 2; ++i) {
        const double2 v = S.rt[i][o];
        acc[2 * i][k] = fma(len, v.x, acc[2 * i][k]);
        acc[2 * i + 1][k] = fma(len, v.y, acc[2 * i + 1][k]);
    }
}

// The cone-beam gather of gather_cone_tile for the cell's voxels iz0 ..
// iz0 + CZ - 1 below mz, every ray applied to the NI images.
template <int CZ, int NI>
__device__ __forceinline__ void gather_cone_sym(const GeomDev &g, const SymTile<NI> &S,
                                                double c, double s, double X0, double X1,
                                                double Y0, double Y1, int iz0, int mz, int C0,
                                                int C1, int R0, int R1, double (&acc)[NI][CZ])
{
    double f0, f1, bmin, bmax;
    u_footprint<true>(g, c, s, X0, X1, Y0, Y1, f0, f1, bmin, bmax);
    int c_lo, c_hi;
    index_range(f0, f1, C0, C1, c_lo, c_hi);
    const double row_lo_off = g.rv0 - (double)R0 - 1e-6, row_hi_off = g.rv0 - (double)R0 + 1e-6;
    const double row_last = (double)(R1 - R0);
    for (int col = c_lo; col <= c_hi; ++col) {
        const int cc = col - C0;
        double tl, th;
        xy_interval<true>(X0, X1, Y0, Y1, S.Sx[cc], S.Sy[cc], S.iDx[cc], S.iDy[cc], S.ox[cc],
                          S.oy[cc], tl, th);
        if (!(th > tl))
            continue;
        const double itl = rcp(tl) * g.ipv, ith = rcp(th) * g.ipv;
        double Z0 = -g.hz + (double)iz0;
        double qa = Z0 * itl, qb = Z0 * ith;
#pragma unroll
        for (int k = 0; k < CZ; ++k) {
            const double Z1 = Z0 + 1.0;
            const double pa = Z1 * itl, pb = Z1 * ith;
            if (iz0 + k < mz) {  // block-uniform
                const int lo = (int)fmax(ceil(fmin(qa, qb) + row_lo_off), 0.0);
                const int hi = (int)fmin(floor(fmax(pa, pb) + row_hi_off), row_last);
                sym_row(S, lo, cc, Z0, Z1, tl, th, lo <= hi, acc, k);
                sym_row(S, lo + 1, cc, Z0, Z1, tl, th, lo + 1 <= hi, acc, k);
                for (int rel = lo + 2; rel <= hi; ++rel)  // wide footprints only
                    sym_row(S, rel, cc, Z0, Z1, tl, th, true, acc, k);
            }
            Z0 = Z1;
            qa = pa;
            qb = pb;
        }
    }
}

// cell of the symmetric gather (the stored transpose's cell)
__host__ __device__ __forceinline__ void sym_cell(const GeomDev &g, int &mx, int &my, int &mz)
{
    mx = g.sym_rot == 4 ? g.nx / 2 : g.nx;
    my = g.sym_rot >= 2 ? g.ny / 2 : g.ny;
    mz = g.sym_mir ? g.nz / 2 : g.nz;
}

// One block of the symmetric gather: BP_TX x BP_TY voxel columns of the
// cell, CZ voxels deep, block (bx, by, bz) of the cell.
template <typename T, int ROT, bool MIR, int CZ>
__device__ __forceinline__ void backproject_sym_block(const GeomDev &g, const T *__restrict__ r,
                                                      T *__restrict__ out, int bx, int by, int bz,
                                                      SymTile<ROT *(MIR ? 2 : 1)> &S)
{
    constexpr int NM = MIR ? 2 : 1, NI = ROT * NM;
    int mx, my, mz;
    sym_cell(g, mx, my, mz);
    const int tid = threadIdx.x;
    const int ix = bx * BP_TX + (tid % BP_TX);
    const int iy = by * BP_TY + (tid / BP_TX);
    const int iz0 = bz * CZ;
    const bool active = ix < mx && iy < my;  // the others stage data and meet every barrier

    double acc[NI][CZ];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int k = 0; k < CZ; ++k)
            acc[i][k] = 0.0;

    const double X0 = -g.hx + (double)ix, X1 = X0 + 1.0;
    const double Y0 = -g.hy + (double)iy, Y1 = Y0 + 1.0;
    const double bX0 = -g.hx + (double)(bx * BP_TX);
    const double bY0 = -g.hy + (double)(by * BP_TY);
    const double bZ0 = -g.hz + (double)iz0;
    const double bX1 = fmin(bX0 + BP_TX, -g.hx + mx), bY1 = fmin(bY0 + BP_TY, -g.hy + my);
    const double bZ1 = fmin(bZ0 + CZ, -g.hz + mz);
    const size_t view_stride = (size_t)g.rows * g.cols;
    const int vstep = g.nviews / ROT;
    for (int i = tid; i < STILE_S; i += BP_THREADS) {  // the zero rows
#pragma unroll
        for (int q = 0; q < NI / 2; ++q)
            S.rt[q][STILE_R * STILE_S + i] = make_double2(0.0, 0.0);
    }
    if (tid == 0)
        S.iDz[STILE_R] = 1.0;

    // detector columns C0..C1 and rows R0..R1 the block's voxels project to
    // in view v (empty when C1 < C0 or R1 < R0)
    const auto footprint = [&](int v, int &C0, int &C1, int &R0, int &R1) {
        const double c = g.cs[v].x, s = g.cs[v].y;
        double f0, f1, bmin, bmax;
        u_footprint<true>(g, c, s, bX0, bX1, bY0, bY1, f0, f1, bmin, bmax);
        index_range(f0, f1, 0, g.cols - 1, C0, C1);
        const double i0 = g.SDD * rcp(g.R - bmin), i1 = g.SDD * rcp(g.R - bmax);
        const double wlo = fmin(bZ0 * i0, bZ0 * i1), whi = fmax(bZ1 * i0, bZ1 * i1);
        index_range(wlo * g.ipv + g.rv0, whi * g.ipv + g.rv0, 0, g.rows - 1, R0, R1);
    };
    // view v's NI detector tiles (r |D| in double) and its column and row
    // entries into LDS
    const auto stage = [&](int v, int C0, int R0, int nc, int nr) {
        for (int i = tid; i < nr * nc; i += BP_THREADS) {
            const int rr = i / nc, cc = i - rr * nc;
            const int row = R0 + rr, col = C0 + cc;
            const int o = rr * STILE_S + cc;
            // |D| of a mirrored row is that of the row (rows symmetric about w = 0)
            const double dn = g.dnorm[(size_t)row * g.cols + col];
            int vq = v;
#pragma unroll
            for (int q = 0; q < ROT; ++q) {
                const T *rq = r + (size_t)vq * view_stride;
                const double a = (double)rq[(size_t)row * g.cols + col] * dn;
                if (MIR) {
                    S.rt[q][o] =
                        make_double2(a, (double)rq[(size_t)(g.rows - 1 - row) * g.cols + col] * dn);
                } else if (q % 2 == 0) {
                    S.rt[q / 2][o].x = a;
                } else {
                    S.rt[q / 2][o].y = a;
                }
                vq += vstep;
                vq -= vq >= g.nviews ? g.nviews : 0;
            }
        }
        for (int i = tid; i < nc; i += BP_THREADS) {
            const ColEntry e = g.col[(size_t)v * g.cols + C0 + i];
            S.Sx[i] = e.Sx;
            S.Sy[i] = e.Sy;
            S.iDx[i] = e.invDx;
            S.iDy[i] = e.invDy;
            S.ox[i] = e.ox;
            S.oy[i] = e.oy;
        }
        // The flat row (invDz = 0: its rays run in the plane w = 0) gets a
        // huge finite 1/Dz instead: its crossing parameters Z0 / Dz, Z1 / Dz
        // are then -huge, 0 or +huge, and the clip of sym_row leaves the
        // whole xy interval th - tl exactly when Z0 <= 0 < Z1 and nothing
        // otherwise -- the flat row's length, with no separate path.
        for (int i = tid; i < nr; i += BP_THREADS) {
            const double idz = g.row[R0 + i].invDz;
            S.iDz[i] = idz != 0.0 ? idz : FLAT_IDZ;
        }
    };

    // One path per view: its footprint in LDS tiles (one tile when it fits,
    // as on the usual scans; else column-major chunks of STILE_C columns by
    // STILE_R rows), each staged and gathered from LDS.  (A second, generic
    // path in the loop would keep the accumulators in other registers on each
    // path and pay moves between them per view.)
    for (int v = 0; v < g.nviews; ++v) {
        int C0, C1, R0, R1;
        footprint(v, C0, C1, R0, R1);
        for (int cb = C0; cb <= C1; cb += STILE_C) {  // block-uniform
            const int ce = min(cb + STILE_C - 1, C1), nc = ce - cb + 1;
            for (int rb = R0; rb <= R1; rb += STILE_R) {
                const int re = min(rb + STILE_R - 1, R1), nr = re - rb + 1;
                stage(v, cb, rb, nc, nr);
                __syncthreads();
                if (active)
                    gather_cone_sym<CZ>(g, S, g.cs[v].x, g.cs[v].y, X0, X1, Y0, Y1, iz0, mz, cb,
                                        ce, rb, re, acc);
                __syncthreads();
            }
        }
    }

    if (!active)
        return;
    const size_t plane = (size_t)g.nx * g.ny;
    int xi = ix, yi = iy;
#pragma unroll
    for (int q = 0; q < ROT; ++q) {
#pragma unroll
        for (int k = 0; k < CZ; ++k) {
            const int iz = iz0 + k;
            if (iz < mz) {
                out[(size_t)iz * plane + (size_t)yi * g.nx + xi] = (T)acc[q * NM][k];
                if (MIR)
                    out[(size_t)(g.nz - 1 - iz) * plane + (size_t)yi * g.nx + xi] =
                        (T)acc[q * NM + 1][k];
            }
        }
        if (ROT == 4) {  // a quarter turn: (i, j) -> (nx - 1 - j, i)
            const int t = xi;
            xi = g.nx - 1 - yi;
            yi = t;
        } else if (ROT == 2) {  // a half turn: (i, j) -> (nx - 1 - i, ny - 1 - j)
            xi = g.nx - 1 - xi;
            yi = g.ny - 1 - yi;
        }
    }
}

// The hardware deals consecutive blocks round-robin to the 8 XCDs, each with
// its own L2; the kernel remaps block ids so that each XCD runs a contiguous
// range of bricks (x fastest, then y, then z): its L2 then serves the
// detector rows of a few z-chunks instead of every chunk in flight.
constexpr int N_XCD = 8;

template <typename T, bool CONE, int CZ>
__global__ __launch_bounds__(BP_THREADS) void backproject_kernel(GeomDev g,
                                                                const T *__restrict__ r,
                                                                T *__restrict__ out)
{
    __shared__ Tile tile;
    const int nb = gridDim.x, p = blockIdx.x;
    const int q = nb / N_XCD, rem = nb % N_XCD, k = p % N_XCD;
    const int L = k * q + min(k, rem) + p / N_XCD;
    const int gx = (g.nx + BP_TX - 1) / BP_TX, gy = (g.ny + BP_TY - 1) / BP_TY;
    if (g.beam3d)  // launch-uniform
        backproject_block3d<T, CZ>(g, r, out, L % gx, (L / gx) % gy, L / (gx * gy));
    else
        backproject_block<T, CONE, CZ>(g, r, out, L % gx, (L / gx) % gy, L / (gx * gy), tile);
}

// The symmetric gather (see backproject_sym_block), block ids remapped to
// XCD-contiguous ranges as in backproject_kernel.
template <typename T, int ROT, bool MIR, int CZ>
__global__ __launch_bounds__(BP_THREADS) void backproject_sym_kernel(GeomDev g,
                                                                    const T *__restrict__ r,
                                                                    T *__restrict__ out)
{
    __shared__ SymTile<ROT *(MIR ? 2 : 1)> S;
    const int nb = gridDim.x, p = blockIdx.x;
    const int q = nb / N_XCD, rem = nb % N_XCD, k = p % N_XCD;
    const int L = k * q + min(k, rem) + p / N_XCD;
    int mx, my, mz;
    sym_cell(g, mx, my, mz);
    const int gx = (mx + BP_TX - 1) / BP_TX, gy = (my + BP_TY - 1) / BP_TY;
    backproject_sym_block<T, ROT, MIR, CZ>(g, r, out, L % gx, (L / gx) % gy, L / (gx * gy), S);
}

// Batched: G = A^T RY for every problem whose gradient is due this round.
template <typename T, int CZ>
__device__ __forceinline__ void backproject_grouped_body(const BatchProblem<T> &P, int local,
                                                         Tile &tile)
{
    const int gx = (P.g.nx + BP_TX - 1) / BP_TX, gy = (P.g.ny + BP_TY - 1) / BP_TY;
    const int bx = local % gx, by = (local / gx) % gy, bz = local / (gx * gy);
    if (P.g.beam3d)  // block-uniform
        backproject_block3d<T, CZ>(P.g, P.RY, P.G, bx, by, bz);
    else if (P.g.cone)
        backproject_block<T, true, CZ>(P.g, P.RY, P.G, bx, by, bz, tile);
    else
        backproject_block<T, false, CZ>(P.g, P.RY, P.G, bx, by, bz, tile);
}

// One kernel per voxel depth CZ (4 or 8): a depth chosen per problem inside
// one kernel would size every block's registers for the deepest variant.
template <typename T, int CZ>
__global__ __launch_bounds__(BP_THREADS) void backproject_grouped(BatchProblem<T> *probs,
                                                                 const int *offs, int n)
{
    __shared__ Tile tile;
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING || !P.need_grad)
        return;
    backproject_grouped_body<T, CZ>(P, blockIdx.x - offs[p], tile);
}

// Batched symmetric gather: the problems whose scan has the symmetry
// (ROT, MIR), each block one block of its problem's cell.
template <typename T, int ROT, bool MIR, int CZ>
__global__ __launch_bounds__(BP_THREADS) void backproject_sym_grouped(BatchProblem<T> *probs,
                                                                     const int *offs, int n)
{
    __shared__ SymTile<ROT *(MIR ? 2 : 1)> S;
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING || !P.need_grad)
        return;
    const int local = blockIdx.x - offs[p];
    int mx, my, mz;
    sym_cell(P.g, mx, my, mz);
    const int gx = (mx + BP_TX - 1) / BP_TX, gy = (my + BP_TY - 1) / BP_TY;
    backproject_sym_block<T, ROT, MIR, CZ>(P.g, P.RY, P.G, local % gx, (local / gx) % gy,
                                           local / (gx * gy), S);
}

}  // namespace

int backproject_depth(const GeomDev &g) { return g.bp_cz == 4 || g.bp_cz == 16 ? g.bp_cz : 8; }

// blocks of the backprojector at the geometry's voxel depth
int backproject_blocks(const GeomDev &g)
{
    const int cz = backproject_depth(g);
    return ((g.nx + BP_TX - 1) / BP_TX) * ((g.ny + BP_TY - 1) / BP_TY) * ((g.nz + cz - 1) / cz);
}

bool backproject_symmetric(const GeomDev &g)
{
    return g.cone && !g.beam3d && (g.sym_rot > 1 || g.sym_mir);
}

// voxels per thread of the symmetric gather: 32 accumulators per thread, at
// most 8 voxels deep
constexpr int sym_depth(int rot, int mir) { return rot * (mir ? 2 : 1) >= 4 ? 32 / (rot * (mir ? 2 : 1)) : 8; }

int backproject_sym_blocks(const GeomDev &g)
{
    int mx, my, mz;
    sym_cell(g, mx, my, mz);
    const int cz = sym_depth(g.sym_rot, g.sym_mir);
    return ((mx + BP_TX - 1) / BP_TX) * ((my + BP_TY - 1) / BP_TY) * ((mz + cz - 1) / cz);
}

template <typename T>
hipError_t launch_backproject_sym_grouped(BatchProblem<T> *probs, const int *offs, int n,
                                          int blocks, int rot, int mir, hipStream_t st)
{
    const dim3 gr(blocks), bl(BP_THREADS);
    if (rot == 4 && mir)
        hipLaunchKernelGGL((backproject_sym_grouped<T, 4, true, sym_depth(4, 1)>), gr, bl, 0, st,
                           probs, offs, n);
    else if (rot == 4)
        hipLaunchKernelGGL((backproject_sym_grouped<T, 4, false, sym_depth(4, 0)>), gr, bl, 0,
                           st, probs, offs, n);
    else if (rot == 2 && mir)
        hipLaunchKernelGGL((backproject_sym_grouped<T, 2, true, sym_depth(2, 1)>), gr, bl, 0, st,
                           probs, offs, n);
    else if (rot == 2)
        hipLaunchKernelGGL((backproject_sym_grouped<T, 2, false, sym_depth(2, 0)>), gr, bl, 0,
                           st, probs, offs, n);
    else
        hipLaunchKernelGGL((backproject_sym_grouped<T, 1, true, sym_depth(1, 1)>), gr, bl, 0, st,
                           probs, offs, n);
    return hipGetLastError();
}

template hipError_t launch_backproject_sym_grouped<float>(BatchProblem<float> *, const int *,
                                                          int, int, int, int, hipStream_t);
template hipError_t launch_backproject_sym_grouped<double>(BatchProblem<double> *, const int *,
                                                           int, int, int, int, hipStream_t);

template <typename T>
hipError_t launch_backproject_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                      int depth, hipStream_t st)
{
    if (depth == 4)
        hipLaunchKernelGGL((backproject_grouped<T, 4>), dim3(blocks), dim3(BP_THREADS), 0, st,
                           probs, offs, n);
    else
        hipLaunchKernelGGL((backproject_grouped<T, 8>), dim3(blocks), dim3(BP_THREADS), 0, st,
                           probs, offs, n);
    return hipGetLastError();
}

template hipError_t launch_backproject_grouped<float>(BatchProblem<float> *, const int *, int,
                                                      int, int, hipStream_t);
template hipError_t launch_backproject_grouped<double>(BatchProblem<double> *, const int *, int,
                                                       int, int, hipStream_t);

template <typename T, int CZ>
static void launch_backproject_cz(const GeomDev &g, const T *r, T *out, hipStream_t st)
{
    dim3 block(BP_THREADS, 1, 1);
    dim3 grid(((g.nx + BP_TX - 1) / BP_TX) * ((g.ny + BP_TY - 1) / BP_TY) *
                  ((g.nz + CZ - 1) / CZ),
              1, 1);
    if (g.cone)
        hipLaunchKernelGGL((backproject_kernel<T, true, CZ>), grid, block, 0, st, g, r, out);
    else
        hipLaunchKernelGGL((backproject_kernel<T, false, CZ>), grid, block, 0, st, g, r, out);
}

template <typename T, int ROT, bool MIR>
static void launch_backproject_sym(const GeomDev &g, const T *r, T *out, hipStream_t st)
{
    hipLaunchKernelGGL((backproject_sym_kernel<T, ROT, MIR, sym_depth(ROT, MIR)>),
                       dim3(backproject_sym_blocks(g)), dim3(BP_THREADS), 0, st, g, r, out);
}

template <typename T>
hipError_t launch_backproject(const GeomDev &g, const T *r, T *out, hipStream_t st)
{
    if (g.mat.present)
        return launch_backproject_matrix<T>(g, r, out, st);
    if (backproject_symmetric(g)) {
        if (g.sym_rot == 4)
            g.sym_mir ? launch_backproject_sym<T, 4, true>(g, r, out, st)
                      : launch_backproject_sym<T, 4, false>(g, r, out, st);
        else if (g.sym_rot == 2)
            g.sym_mir ? launch_backproject_sym<T, 2, true>(g, r, out, st)
                      : launch_backproject_sym<T, 2, false>(g, r, out, st);
        else
            launch_backproject_sym<T, 1, true>(g, r, out, st);
        return hipGetLastError();
    }
    switch (g.bp_cz) {
    case 4:
        launch_backproject_cz<T, 4>(g, r, out, st);
        break;
    case 16:
        launch_backproject_cz<T, 16>(g, r, out, st);
        break;
    default:
        launch_backproject_cz<T, 8>(g, r, out, st);
        break;
    }
    return hipGetLastError();
}

template hipError_t launch_backproject<float>(const GeomDev &, const float *, float *,
                                              hipStream_t);
template hipError_t launch_backproject<double>(const GeomDev &, const double *, double *,
                                               hipStream_t);

}  // namespace tvr

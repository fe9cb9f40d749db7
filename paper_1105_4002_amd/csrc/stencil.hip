// Voxel-space kernels: the smoothed-TV stencil (value, gradient, Bregman
// distance), the projected trial step, UPN's extrapolation, the
// Barzilai-Borwein inner products, the y-fastest transpose and the slot
// finaliser.
//
// TV (eq. 2, Huber-smoothed with parameter tau):
//   T_tau(x) = sum_j Phi(D_j x),  Phi(z) = |z| - tau/2 (|z| >= tau),
//   |z|^2 / (2 tau) otherwise, D_j x = forward differences along x, y, z,
//   a component being 0 where the neighbour is outside the volume;
//   grad T_tau(x) = sum_j D_j^T q_j,  q_j = D_j x / max(tau, |D_j x|).
// The stencil arithmetic (differences, q, per-voxel Phi and Bregman terms)
// runs in the storage type T -- with one hardware reciprocal square root per
// normalisation for float -- and every sum over voxels runs in double.
//
// The TV and trial kernels give each thread one (x, y) column and march up
// a chunk of z, carrying the values the next plane reuses.
#include "reduce.hpp"
#include "stencil_math.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

template <typename C>
__device__ __forceinline__ C huber_c(C d2, C tau, C itau)
{
    const C n = SM<C>::norm(d2);
    return n >= tau ? n - C(0.5) * tau : C(0.5) * d2 * itau;
}

// Bregman distance Phi(a) - Phi(b) - grad Phi(b)^T (a - b) with d = a - b,
// written per smoothing regime so that it is formed from d without
// cancellation (each case follows from |a|^2 = |b|^2 + 2 b.d + |d|^2):
//   both quadratic: |d|^2 / (2 tau);  both linear: |a|/2 |a/|a| - b/|b||^2;
//   a linear, b quadratic: (|d|^2 - (|a| - tau)^2) / (2 tau);
//   a quadratic, b linear: |a - tau b/|b||^2 / (2 tau).
template <typename C>
__device__ __forceinline__ C huber_bregman(C a0, C a1, C a2, C b0, C b1, C b2, C d0, C d1, C d2,
                                           C tau, C itau)
{
    const C na = SM<C>::norm(a0 * a0 + a1 * a1 + a2 * a2);
    const C nb = SM<C>::norm(b0 * b0 + b1 * b1 + b2 * b2);
    const C dd = d0 * d0 + d1 * d1 + d2 * d2;
    if (na < tau && nb < tau)
        return C(0.5) * dd * itau;
    if (na >= tau && nb >= tau) {
        // unit-vector difference d/|a| - (b/|b|) ((a + b).d) / (|a| (|a| + |b|))
        const C ia = SM<C>::inv(na), ib = SM<C>::inv(nb);
        const C sc = ((a0 + b0) * d0 + (a1 + b1) * d1 + (a2 + b2) * d2) * ia * SM<C>::inv(na + nb);
        const C e0 = d0 * ia - b0 * ib * sc;
        const C e1 = d1 * ia - b1 * ib * sc;
        const C e2 = d2 * ia - b2 * ib * sc;
        return C(0.5) * na * (e0 * e0 + e1 * e1 + e2 * e2);
    }
    if (na >= tau) {
        const C t = na - tau;
        const C v = C(0.5) * (dd - t * t) * itau;
        return v > C(0) ? v : C(0);
    }
    const C s = tau * SM<C>::inv(nb);
    const C e0 = a0 - b0 * s, e1 = a1 - b1 * s, e2 = a2 - b2 * s;
    return C(0.5) * (e0 * e0 + e1 * e1 + e2 * e2) * itau;
}

// gout = (gin ? gin : 0) + alpha grad T(y); with partials also the sums
// T(y) and, with xref, Bregman_T(xref, y) and |xref - y|^2.  The block's
// 64 x 4 columns march up VZ planes.  Each thread reads the neighbours its
// terms need (+x, +y, +z for its own forward differences; the left voxel's
// +y and +z, the front voxel's +x and +z for their q components) straight
// from global memory, where L1 and L2 serve the re-reads of adjacent
// columns: no LDS staging and no barrier.  The values of plane z + 1 that
// plane z already needs (own, left and front) are carried up; the next
// plane's other loads are issued before the current plane's arithmetic.
// Neighbours outside the volume read as 0 and only enter through the same
// masks as the forward differences, so every voxel's arithmetic and every
// block's sum order are those of a zero-padded volume.
template <typename T>
__device__ __forceinline__ void tv_block(int nx, int ny, int nz, double tau, double alpha,
                                                const T *__restrict__ y, const T *__restrict__ xref,
                                                const T *__restrict__ gin, T *__restrict__ gout,
                                                double *__restrict__ partials, int pstride, int bx,
                                                int by, int bz, int bid, bool value)
{
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int ix = bx * VX + tx, iy = by * VY + ty;
    const int z0 = bz * VZ;
    const int z1 = min(z0 + VZ, nz);
    const bool active = ix < nx && iy < ny;
    double red[3] = {0.0, 0.0, 0.0};
    const T ct = (T)tau, itau = T(1) / ct;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    const bool hx = ix + 1 < nx, hy = iy + 1 < ny, lx = ix > 0, ly = iy > 0;
    const bool hxly = hx && ly, lxhy = lx && hy;
    const bool hasx = xref != nullptr, addg = gin != nullptr && gout != nullptr;
    T qz_prev = T(0);
    if (active && z0 > 0) {
        const size_t jb = (size_t)ix + sy * iy + sz * (z0 - 1);
        const T yb = y[jb];
        const T dx = hx ? y[jb + 1] - yb : T(0);
        const T dy = hy ? y[jb + sy] - yb : T(0);
        const T dz = y[jb + sz] - yb;
        qz_prev = dz * SM<T>::inv_clamped(dx * dx + dy * dy + dz * dz, ct, itau);
    }
    const size_t j0 = active ? (size_t)ix + sy * iy + sz * z0 : 0;
    // plane z values
    T c = T(0), l = T(0), f = T(0), r = T(0), b = T(0), lb = T(0), rf = T(0);
    T xj = T(0), xa = T(0), xb = T(0), g0 = T(0);
    // plane z + 1 values
    T cn = T(0), ln = T(0), fn = T(0), xc = T(0);
    if (active && z0 < z1) {
        const size_t j = j0;
        c = y[j];
        l = lx ? y[j - 1] : T(0);
        f = ly ? y[j - sy] : T(0);
        r = hx ? y[j + 1] : T(0);
        b = hy ? y[j + sy] : T(0);
        lb = lxhy ? y[j - 1 + sy] : T(0);
        rf = hxly ? y[j + 1 - sy] : T(0);
        if (hasx) {
            xj = xref[j];
            xa = hx ? xref[j + 1] : T(0);
            xb = hy ? xref[j + sy] : T(0);
        }
        if (addg)
            g0 = gin[j];
        if (z0 + 1 < nz) {
            cn = y[j + sz];
            ln = lx ? y[j + sz - 1] : T(0);
            fn = ly ? y[j + sz - sy] : T(0);
            if (hasx)
                xc = xref[j + sz];
        }
    }
    for (int z = z0; z < z1; ++z) {
        const bool hz = z + 1 < nz;
        const size_t j = j0 + sz * (size_t)(z - z0);
        // next plane's lateral values and the plane after it, loaded ahead
        T r1 = T(0), b1 = T(0), lb1 = T(0), rf1 = T(0), xa1 = T(0), xb1 = T(0), g1 = T(0);
        T c2 = T(0), l2 = T(0), f2 = T(0), xc2 = T(0);
        const bool nxt = active && z + 1 < z1;
        if (nxt) {
            const size_t k = j + sz;
            r1 = hx ? y[k + 1] : T(0);
            b1 = hy ? y[k + sy] : T(0);
            lb1 = lxhy ? y[k - 1 + sy] : T(0);
            rf1 = hxly ? y[k + 1 - sy] : T(0);
            if (hasx) {
                xa1 = hx ? xref[k + 1] : T(0);
                xb1 = hy ? xref[k + sy] : T(0);
            }
            if (addg)
                g1 = gin[k];
            if (z + 2 < nz) {
                const size_t k2 = k + sz;
                c2 = y[k2];
                l2 = lx ? y[k2 - 1] : T(0);
                f2 = ly ? y[k2 - sy] : T(0);
                if (hasx)
                    xc2 = xref[k2];
            }
        }
        if (active) {
            const T yj = c;
            const T dx = hx ? r - yj : T(0);
            const T dy = hy ? b - yj : T(0);
            const T dz = hz ? cn - yj : T(0);
            const T d2 = dx * dx + dy * dy + dz * dz;
            const T inv = SM<T>::inv_clamped(d2, ct, itau);
            T gsum = -(dx + dy + dz) * inv + qz_prev;
            qz_prev = dz * inv;
            {
                const T yk = l;
                const T ex = yj - yk;
                const T ey = hy ? lb - yk : T(0);
                const T ez = hz ? ln - yk : T(0);
                const T t = ex * SM<T>::inv_clamped(ex * ex + ey * ey + ez * ez, ct, itau);
                gsum += lx ? t : T(0);
            }
            {
                const T yk = f;
                const T ex = hx ? rf - yk : T(0);
                const T ey = yj - yk;
                const T ez = hz ? fn - yk : T(0);
                const T t = ey * SM<T>::inv_clamped(ex * ex + ey * ey + ez * ez, ct, itau);
                gsum += ly ? t : T(0);
            }
            if (gout)
                gout[j] = gin ? (T)((double)g0 + alpha * (double)gsum)
                              : (T)(alpha * (double)gsum);
            if (partials) {
                if (value)
                    red[0] += (double)huber_c<T>(d2, ct, itau);
                if (hasx) {
                    const T ej = xj - yj;
                    const T a0 = hx ? xa - xj : T(0);
                    const T e0 = hx ? (xa - r) - ej : T(0);
                    const T a1 = hy ? xb - xj : T(0);
                    const T e1 = hy ? (xb - b) - ej : T(0);
                    const T a2 = hz ? xc - xj : T(0);
                    const T e2 = hz ? (xc - cn) - ej : T(0);
                    red[1] += (double)huber_bregman<T>(a0, a1, a2, dx, dy, dz, e0, e1, e2, ct, itau);
                    const double ed = (double)xj - (double)yj;
                    red[2] += ed * ed;
                }
            }
        }
        c = cn; l = ln; f = fn; xj = xc;
        r = r1; b = b1; lb = lb1; rf = rf1; xa = xa1; xb = xb1; g0 = g1;
        cn = c2; ln = l2; fn = f2; xc = xc2;
    }
    if (partials && value) {
        const int slots[3] = {S_TVY, S_BRY, S_XY2};
        block_reduce_store<3>(red, partials, pstride, slots, bid);
    } else if (partials && xref) {  // the Bregman terms only
        const int slots[2] = {S_BRY, S_XY2};
        double r2[2] = {red[1], red[2]};
        block_reduce_store<2>(r2, partials, pstride, slots, bid);
    }
}

template <typename T>
__global__ __launch_bounds__(VX *VY) void tv_kernel(int nx, int ny, int nz, double tau,
                                                    double alpha, const T *__restrict__ y,
                                                    const T *__restrict__ xref,
                                                    const T *__restrict__ gin,
                                                    T *__restrict__ gout,
                                                    double *__restrict__ partials, int pstride,
                                                    bool value)
{
    tv_block<T>(nx, ny, nz, tau, alpha, y, xref, gin, gout, partials, pstride, blockIdx.x,
                blockIdx.y, blockIdx.z, block_linear_id(), value);
}

// local block -> (bx, by, bz) of a voxel grid
__device__ __forceinline__ void voxel_block_coords(int local, int nx, int ny, int &bx, int &by,
                                                   int &bz)
{
    const int gx = (nx + VX - 1) / VX, gy = (ny + VY - 1) / VY;
    bx = local % gx;
    by = (local / gx) % gy;
    bz = local / (gx * gy);
}

// Batched gradient assembly G += alpha grad T(Y), with the Bregman terms
// against X once Y has moved away from X (UPN, the batched method, needs no
// value of T(Y)).
template <typename T>
__global__ __launch_bounds__(VX *VY) void tv_grouped(BatchProblem<T> *probs, const int *offs,
                                                     int n)
{
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING || !P.need_grad)
        return;
    const int local = blockIdx.x - offs[p];
    int bx, by, bz;
    voxel_block_coords(local, P.g.nx, P.g.ny, bx, by, bz);
    tv_block<T>(P.g.nx, P.g.ny, P.g.nz, P.tau, P.alpha, P.Y, P.distinct ? P.X : nullptr, P.G,
                P.G, P.part, P.pstride, bx, by, bz, local, false);
}

template <typename T>
__device__ __forceinline__ T pstep(T z, T g, double step, const Box &box)
{
    return (T)clip_box((double)z - step * (double)g, box);
}

// xbar = P_Q(z - step g) (Q = [lo, hi]^N, a clip) with the sums |xbar - z|^2,
// g^T (z - xbar), T(xbar), Bregman_T(xbar, z) and, for gm_step > 0,
// |z - P_Q(z - gm_step g)|^2 (the GPBB gradient map).  As in the TV stencil
// each thread reads its high-side neighbours of z and g from global memory
// with no barrier, the next plane's loads issued before the current plane's
// arithmetic; the value above becomes the next plane's own.
template <typename T>
__device__ __forceinline__ void trial_block(int nx, int ny, int nz, double tau,
                                            const T *__restrict__ zv, const T *__restrict__ g,
                                            double step, double gm_step, const Box box,
                                            T *__restrict__ xbar, double *__restrict__ partials,
                                            int pstride, int bx, int by, int bz, int bid)
{
    const int ix = bx * VX + (int)threadIdx.x, iy = by * VY + (int)threadIdx.y;
    const int z0 = bz * VZ;
    const int z1 = min(z0 + VZ, nz);
    const bool active = ix < nx && iy < ny;
    double red[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const T ct = (T)tau, itau = T(1) / ct;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    const bool hx = ix + 1 < nx, hy = iy + 1 < ny;
    const size_t j0 = active ? (size_t)ix + sy * iy + sz * z0 : 0;
    // plane z: own, +x and +y values; plane z + 1: own value
    T zc = T(0), gc = T(0), zr = T(0), gr = T(0), zb = T(0), gb = T(0), zn = T(0), gn = T(0);
    if (active && z0 < z1) {
        zc = zv[j0];
        gc = g[j0];
        if (hx) {
            zr = zv[j0 + 1];
            gr = g[j0 + 1];
        }
        if (hy) {
            zb = zv[j0 + sy];
            gb = g[j0 + sy];
        }
        if (z0 + 1 < nz) {
            zn = zv[j0 + sz];
            gn = g[j0 + sz];
        }
    }
    for (int z = z0; z < z1; ++z) {
        const bool hz = z + 1 < nz;
        const size_t j = j0 + sz * (size_t)(z - z0);
        T zr1 = T(0), gr1 = T(0), zb1 = T(0), gb1 = T(0), zn2 = T(0), gn2 = T(0);
        if (active && z + 1 < z1) {
            const size_t k = j + sz;
            if (hx) {
                zr1 = zv[k + 1];
                gr1 = g[k + 1];
            }
            if (hy) {
                zb1 = zv[k + sy];
                gb1 = g[k + sy];
            }
            if (z + 2 < nz) {
                zn2 = zv[k + sz];
                gn2 = g[k + sz];
            }
        }
        if (active) {
            const T zj = zc, gj = gc;
            const T xj = pstep(zj, gj, step, box);
            const T zxp = hx ? zr : zj;
            const T xxp = hx ? pstep(zxp, gr, step, box) : xj;
            const T zyp = hy ? zb : zj;
            const T xyp = hy ? pstep(zyp, gb, step, box) : xj;
            const T zzp = hz ? zn : zj;
            const T xzp = hz ? pstep(zzp, gn, step, box) : xj;
            xbar[j] = xj;
            const double ed = (double)xj - (double)zj;
            red[0] += ed * ed;
            red[1] -= (double)gj * ed;
            const T a0 = xxp - xj, a1 = xyp - xj, a2 = xzp - xj;
            const T b0 = zxp - zj, b1 = zyp - zj, b2 = zzp - zj;
            const T ej = xj - zj;
            const T d0 = (xxp - zxp) - ej, d1 = (xyp - zyp) - ej, d2 = (xzp - zzp) - ej;
            red[2] += (double)huber_c<T>(a0 * a0 + a1 * a1 + a2 * a2, ct, itau);
            red[3] += (double)huber_bregman<T>(a0, a1, a2, b0, b1, b2, d0, d1, d2, ct, itau);
            if (gm_step > 0.0) {
                const double zd = (double)zj;
                const double p = zd - clip_box(zd - gm_step * (double)gj, box);
                red[4] += p * p;
            }
        }
        zc = zn;
        gc = gn;
        zr = zr1;
        gr = gr1;
        zb = zb1;
        gb = gb1;
        zn = zn2;
        gn = gn2;
    }
    const int slots[5] = {S_XD2, S_GD, S_TVB, S_BRB, S_GM2};
    block_reduce_store<5>(red, partials, pstride, slots, bid);
}

template <typename T>
__global__ __launch_bounds__(VX *VY) void trial_kernel(int nx, int ny, int nz, double tau,
                                                       const T *__restrict__ zv,
                                                       const T *__restrict__ g, double step,
                                                       double gm_step, Box box,
                                                       T *__restrict__ xbar,
                                                       double *__restrict__ partials,
                                                       int pstride)
{
    trial_block<T>(nx, ny, nz, tau, zv, g, step, gm_step, box, xbar, partials, pstride,
                   blockIdx.x, blockIdx.y, blockIdx.z, block_linear_id());
}

// Batched trial XB = P_Q(Y - G / L) of every running problem.
template <typename T>
__global__ __launch_bounds__(VX *VY) void trial_grouped(BatchProblem<T> *probs, const int *offs,
                                                        int n)
{
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING)
        return;
    const int local = blockIdx.x - offs[p];
    int bx, by, bz;
    voxel_block_coords(local, P.g.nx, P.g.ny, bx, by, bz);
    trial_block<T>(P.g.nx, P.g.ny, P.g.nz, P.tau, P.Y, P.G, 1.0 / P.L, 0.0, P.box, P.XB,
                   P.part, P.pstride, bx, by, bz, local);
}

// Slice z of a stack of ny x nx matrices, transposed: xt[z][x][y] =
// x[z][y][x], through a 32 x 32 LDS tile per block (both the read and the
// write are coalesced); the padding column avoids bank conflicts.
constexpr int TR = 32;

template <typename T>
__device__ __forceinline__ void transpose_block(int nx, int ny, const T *__restrict__ x,
                                                T *__restrict__ xt, int gbx, int gby, int z,
                                                T (&tile)[TR][TR + 1])
{
    const size_t plane = (size_t)nx * ny;
    const T *xs = x + (size_t)z * plane;
    T *xd = xt + (size_t)z * plane;
    const int bx = gbx * TR, by = gby * TR;
    const int tx = threadIdx.x % TR, ty = threadIdx.x / TR;  // 32 x 8 threads
    for (int j = ty; j < TR; j += 8) {
        const int ix = bx + tx, iy = by + j;
        if (ix < nx && iy < ny)
            tile[j][tx] = xs[(size_t)iy * nx + ix];
    }
    __syncthreads();
    for (int j = ty; j < TR; j += 8) {
        const int iy = by + tx, ix = bx + j;
        if (ix < nx && iy < ny)
            xd[(size_t)ix * ny + iy] = tile[tx][j];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(int nx, int ny, const T *__restrict__ x,
                                                           T *__restrict__ xt)
{
    __shared__ T tile[TR][TR + 1];
    transpose_block<T>(nx, ny, x, xt, blockIdx.x, blockIdx.y, blockIdx.z, tile);
}

// The companion copy of a problem's trial point for its ray tile: for column
// tiles the z-fastest copy, which is the transpose of x seen as an nz x
// (ny nx) matrix (one slice of transpose_block); for row tiles the y-fastest
// copy, one transpose per z slice.
template <typename T>
__global__ __launch_bounds__(256) void transpose_grouped(BatchProblem<T> *probs, const int *offs,
                                                         int n)
{
    __shared__ T tile[TR][TR + 1];
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING)
        return;
    const int local = blockIdx.x - offs[p];
    if (column_tiles(P.g.pj_wc)) {  // block-uniform
        const int cols = P.g.nx * P.g.ny, gx = (cols + TR - 1) / TR;
        transpose_block<T>(cols, P.g.nz, P.XB, P.XT, local % gx, local / gx, 0, tile);
    } else {
        const int gx = (P.g.nx + TR - 1) / TR, gy = (P.g.ny + TR - 1) / TR;
        transpose_block<T>(P.g.nx, P.g.ny, P.XB, P.XT, local % gx, (local / gx) % gy,
                           local / (gx * gy), tile);
    }
}

// Batched UPN extrapolation after an accepted step (the control kernel has
// already made X the new iterate and XB the previous one):
// YB = X + beta (X - XB), RYB = RX + beta (RX - RXB), sum (RYB - RX)^2.
template <typename T>
__global__ __launch_bounds__(256) void extrapolate_grouped(BatchProblem<T> *probs,
                                                           const int *offs, int n)
{
    const int p = find_problem(offs, n, blockIdx.x);
    BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING || !P.ex)
        return;
    // the first blocks cover the volume, the rest the data, partitioned
    // exactly as the single-problem launches do (same partial sums)
    const int local = blockIdx.x - offs[p];
    const int nbN = elementwise_blocks_dev(P.N), nbM = P.nb_ew;
    const double beta = P.beta;
    if (local < nbN) {
        for (int64_t i = (int64_t)local * VB + threadIdx.x; i < P.N; i += (int64_t)nbN * VB) {
            const double a = (double)P.X[i];
            P.YB[i] = (T)(a + beta * (a - (double)P.XB[i]));
        }
        return;  // block-uniform
    }
    const int lb = local - nbN;
    double red[1] = {0.0};
    for (int64_t k = (int64_t)lb * VB + threadIdx.x; k < P.m; k += (int64_t)nbM * VB) {
        const double a = (double)P.RX[k];
        const T yi = (T)(a + beta * (a - (double)P.RXB[k]));
        P.RYB[k] = yi;
        const double d = (double)yi - a;
        red[0] += d * d;
    }
    const int slots[1] = {S_RY2};
    block_reduce_store<1>(red, P.part, P.pstride, slots, lb);
}

// Finalisers: one block of FB threads per slot sums the slot's per-block
// partials in a fixed order, so every sum is bitwise reproducible.  Thread t
// adds the partials t, t + FB, t + 2 FB, ... in four interleaved chains (four
// loads in flight), the chains combine pairwise, each wave reduces by a fixed
// shuffle tree and thread 0 adds the wave totals in order.  The single and
// batched finalisers share it, so a batched problem's sums equal its own
// solve's.
constexpr int FB = 1024;

__device__ __forceinline__ double fixed_order_sum(const double *__restrict__ src, int count)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * FB < count; i += 4 * FB) {
        a0 += src[i];
        a1 += src[i + FB];
        a2 += src[i + 2 * FB];
        a3 += src[i + 3 * FB];
    }
    for (; i < count; i += FB)
        a0 += src[i];
    const double s = wave_sum((a0 + a1) + (a2 + a3));
    __shared__ double sh[FB / 64];
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < FB / 64; ++w)
            t += sh[w];
    return t;
}

// Batched finaliser: one block per (problem, slot) of the slots the round
// produced.
constexpr int NFIN = 9;
__constant__ const int fin_slots[NFIN] = {S_XD2, S_GD, S_TVB, S_BRB, S_R2, S_RD2,
                                          S_BRY, S_XY2, S_RY2};

template <typename T>
__global__ __launch_bounds__(FB) void finalize_grouped(BatchProblem<T> *probs)
{
    const int p = blockIdx.x / NFIN, q = blockIdx.x % NFIN;
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING)
        return;
    const int slot = fin_slots[q];
    int count;
    if (slot == S_R2 || slot == S_RD2)
        count = P.nb_proj;
    else if (slot == S_BRY || slot == S_XY2)
        count = P.need_grad ? P.nb_vox : 0;
    else if (slot == S_RY2)
        count = P.ry2_pending ? P.nb_ew : 0;
    else
        count = P.nb_vox;
    if (count == 0)
        return;
    const double t = fixed_order_sum(P.part + (size_t)slot * P.pstride, count);
    if (threadIdx.x == 0)
        P.sum[slot] = t;
}

template <typename T>
__global__ __launch_bounds__(VB) void extrapolate_kernel(int64_t n, double beta,
                                                         const T *__restrict__ xn,
                                                         const T *__restrict__ xo,
                                                         T *__restrict__ y,
                                                         double *__restrict__ partials,
                                                         int pstride)
{
    double red[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VB) {
        const double a = (double)xn[i];
        const T yi = (T)(a + beta * (a - (double)xo[i]));
        y[i] = yi;
        const double d = (double)yi - a;
        red[0] += d * d;
    }
    if (partials) {
        const int slots[1] = {S_RY2};
        block_reduce_store<1>(red, partials, pstride, slots);
    }
}

// UPN's extrapolation of the volume and of its residual in one launch:
// blocks [0, nb1) take y1 = xn1 + beta (xn1 - xo1) over n1 voxels; blocks
// [nb1, nb1 + nb2) take y2 likewise over n2 rays and write the partial sums
// of (y2 - xn2)^2 exactly as a launch of nb2 blocks of extrapolate_kernel
// would (same elements per block, same slots).
template <typename T>
__global__ __launch_bounds__(VB) void extrapolate2_kernel(
    int64_t n1, const T *__restrict__ xn1, const T *__restrict__ xo1, T *__restrict__ y1, int nb1,
    int64_t n2, const T *__restrict__ xn2, const T *__restrict__ xo2, T *__restrict__ y2, int nb2,
    double beta, double *__restrict__ partials, int pstride)
{
    if ((int)blockIdx.x < nb1) {  // block-uniform
        for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n1; i += (int64_t)nb1 * VB) {
            const double a = (double)xn1[i];
            y1[i] = (T)(a + beta * (a - (double)xo1[i]));
        }
        return;
    }
    const int b = (int)blockIdx.x - nb1;
    double red[1] = {0.0};
    for (int64_t i = (int64_t)b * VB + threadIdx.x; i < n2; i += (int64_t)nb2 * VB) {
        const double a = (double)xn2[i];
        const T yi = (T)(a + beta * (a - (double)xo2[i]));
        y2[i] = yi;
        const double d = (double)yi - a;
        red[0] += d * d;
    }
    const int slots[1] = {S_RY2};
    block_reduce_store<1>(red, partials, pstride, slots, b);
}

template <typename T>
__global__ __launch_bounds__(VB) void bb_dots_kernel(int64_t n, const T *__restrict__ x,
                                                     const T *__restrict__ xp,
                                                     const T *__restrict__ g,
                                                     const T *__restrict__ gp,
                                                     double *__restrict__ partials, int pstride)
{
    double red[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VB) {
        const double s = (double)x[i] - (double)xp[i];
        const double dg = (double)g[i] - (double)gp[i];
        red[0] += s * s;
        red[1] += s * dg;
    }
    const int slots[2] = {S_SS, S_SY};
    block_reduce_store<2>(red, partials, pstride, slots);
}

template <typename T>
__global__ __launch_bounds__(VB) void clip_kernel(int64_t n, const T *__restrict__ in,
                                                  T *__restrict__ out, Box box)
{
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VB)
        out[i] = (T)clip_box((double)in[i], box);
}

__global__ __launch_bounds__(FB) void finalize_kernel(SlotList sl, const double *__restrict__ partials,
                                                      int pstride)
{
    const int q = blockIdx.x;
    const double t = fixed_order_sum(partials + (size_t)sl.slot[q] * pstride, sl.count[q]);
    if (threadIdx.x == 0)
        *sl.dst[q] = t;
}

__global__ void combine_phi_kernel(const double *r2, const double *tv, double alpha, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *out = 0.5 * (*r2) + alpha * (*tv);
}

dim3 voxel_grid(int nx, int ny, int nz)
{
    return dim3((nx + VX - 1) / VX, (ny + VY - 1) / VY, (nz + VZ - 1) / VZ);
}

}  // namespace

int elementwise_blocks(int64_t n)
{
    int64_t b = (n + VB - 1) / VB;
    if (b > EW_MAX_BLOCKS)
        b = EW_MAX_BLOCKS;
    return (int)(b < 1 ? 1 : b);
}

int max_reduce_blocks_vol(int nx, int ny, int nz)
{
    const dim3 gr = voxel_grid(nx, ny, nz);
    return (int)(gr.x * gr.y * gr.z);
}

template <typename T>
hipError_t launch_tv(int nx, int ny, int nz, double tau, double alpha, const T *y, const T *xref,
                     const T *gin, T *gout, double *partials, int pstride, hipStream_t st,
                     int *nblocks, bool value)
{
    const dim3 gr = voxel_grid(nx, ny, nz);
    if (nblocks)
        *nblocks = (int)(gr.x * gr.y * gr.z);
    hipLaunchKernelGGL((tv_kernel<T>), gr, dim3(VX, VY), 0, st, nx, ny, nz, tau, alpha, y, xref,
                       gin, gout, partials, pstride, value);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_trial(int nx, int ny, int nz, double tau, const T *z, const T *g, double step,
                        double gm_step, Box box, T *xbar, double *partials, int pstride,
                        hipStream_t st, int *nblocks)
{
    const dim3 gr = voxel_grid(nx, ny, nz);
    if (nblocks)
        *nblocks = (int)(gr.x * gr.y * gr.z);
    hipLaunchKernelGGL((trial_kernel<T>), gr, dim3(VX, VY), 0, st, nx, ny, nz, tau, z, g, step,
                       gm_step, box, xbar, partials, pstride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_extrapolate(int64_t n, double beta, const T *xn, const T *xo, T *y,
                              double *partials, int pstride, hipStream_t st, int *nblocks)
{
    const int nb = elementwise_blocks(n);
    if (nblocks)
        *nblocks = nb;
    hipLaunchKernelGGL((extrapolate_kernel<T>), dim3(nb), dim3(VB), 0, st, n, beta, xn, xo, y,
                       partials, pstride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_extrapolate2(int64_t n1, const T *xn1, const T *xo1, T *y1, int64_t n2,
                               const T *xn2, const T *xo2, T *y2, double beta, double *partials,
                               int pstride, hipStream_t st, int *nblocks2)
{
    const int nb1 = elementwise_blocks(n1), nb2 = elementwise_blocks(n2);
    *nblocks2 = nb2;
    hipLaunchKernelGGL((extrapolate2_kernel<T>), dim3(nb1 + nb2), dim3(VB), 0, st, n1, xn1, xo1, y1,
                       nb1, n2, xn2, xo2, y2, nb2, beta, partials, pstride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bb_dots(int64_t n, const T *x, const T *xp, const T *g, const T *gp,
                          double *partials, int pstride, hipStream_t st, int *nblocks)
{
    const int nb = elementwise_blocks(n);
    if (nblocks)
        *nblocks = nb;
    hipLaunchKernelGGL((bb_dots_kernel<T>), dim3(nb), dim3(VB), 0, st, n, x, xp, g, gp, partials,
                       pstride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_companion(const GeomDev &g, const T *x, T *xc, hipStream_t st)
{
    if (column_tiles(g.pj_wc)) {
        // x as an nz x (ny nx) matrix, transposed
        const int cols = g.nx * g.ny;
        dim3 grid((cols + TR - 1) / TR, (g.nz + TR - 1) / TR, 1);
        hipLaunchKernelGGL((transpose_kernel<T>), grid, dim3(256), 0, st, cols, g.nz, x, xc);
    } else {
        dim3 grid((g.nx + TR - 1) / TR, (g.ny + TR - 1) / TR, g.nz);
        hipLaunchKernelGGL((transpose_kernel<T>), grid, dim3(256), 0, st, g.nx, g.ny, x, xc);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_clip(int64_t n, const T *in, T *out, Box box, hipStream_t st)
{
    hipLaunchKernelGGL((clip_kernel<T>), dim3(elementwise_blocks(n)), dim3(VB), 0, st, n, in, out,
                       box);
    return hipGetLastError();
}

hipError_t launch_finalize(const SlotList &sl, const double *partials, int pstride,
                           hipStream_t st)
{
    if (sl.n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(sl.n), dim3(FB), 0, st, sl, partials, pstride);
    return hipGetLastError();
}

hipError_t launch_combine_phi(const double *r2, const double *tv, double alpha, double *out,
                              hipStream_t st)
{
    hipLaunchKernelGGL(combine_phi_kernel, dim3(1), dim3(64), 0, st, r2, tv, alpha, out);
    return hipGetLastError();
}

int companion_blocks(const GeomDev &g)
{
    if (column_tiles(g.pj_wc))
        return ((g.nx * g.ny + TR - 1) / TR) * ((g.nz + TR - 1) / TR);
    return ((g.nx + TR - 1) / TR) * ((g.ny + TR - 1) / TR) * g.nz;
}

template <typename T>
hipError_t launch_tv_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                             hipStream_t st)
{
    hipLaunchKernelGGL((tv_grouped<T>), dim3(blocks), dim3(VX, VY), 0, st, probs, offs, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_trial_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                hipStream_t st)
{
    hipLaunchKernelGGL((trial_grouped<T>), dim3(blocks), dim3(VX, VY), 0, st, probs, offs, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_transpose_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                                    hipStream_t st)
{
    hipLaunchKernelGGL((transpose_grouped<T>), dim3(blocks), dim3(256), 0, st, probs, offs, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_extrapolate_grouped(BatchProblem<T> *probs, const int *offs, int n,
                                      int blocks, hipStream_t st)
{
    hipLaunchKernelGGL((extrapolate_grouped<T>), dim3(blocks), dim3(VB), 0, st, probs, offs, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize_grouped(BatchProblem<T> *probs, int n, hipStream_t st)
{
    hipLaunchKernelGGL((finalize_grouped<T>), dim3(n * NFIN), dim3(FB), 0, st, probs);
    return hipGetLastError();
}

#define TVR_INST_GROUPED(T)                                                                      \
    template hipError_t launch_tv_grouped<T>(BatchProblem<T> *, const int *, int, int,           \
                                             hipStream_t);                                       \
    template hipError_t launch_trial_grouped<T>(BatchProblem<T> *, const int *, int, int,        \
                                                hipStream_t);                                    \
    template hipError_t launch_transpose_grouped<T>(BatchProblem<T> *, const int *, int, int,    \
                                                    hipStream_t);                                \
    template hipError_t launch_extrapolate_grouped<T>(BatchProblem<T> *, const int *, int, int,  \
                                                      hipStream_t);                              \
    template hipError_t launch_finalize_grouped<T>(BatchProblem<T> *, int, hipStream_t);

TVR_INST_GROUPED(float)
TVR_INST_GROUPED(double)

#define TVR_INST(T)                                                                              \
    template hipError_t launch_tv<T>(int, int, int, double, double, const T *, const T *,       \
                                     const T *, T *, double *, int, hipStream_t, int *, bool);        \
    template hipError_t launch_trial<T>(int, int, int, double, const T *, const T *, double,     \
                                        double, Box, T *, double *, int, hipStream_t, int *);   \
    template hipError_t launch_extrapolate<T>(int64_t, double, const T *, const T *, T *,       \
                                              double *, int, hipStream_t, int *);               \
    template hipError_t launch_extrapolate2<T>(int64_t, const T *, const T *, T *, int64_t,      \
                                               const T *, const T *, T *, double, double *, int,  \
                                               hipStream_t, int *);                              \
    template hipError_t launch_bb_dots<T>(int64_t, const T *, const T *, const T *, const T *,  \
                                          double *, int, hipStream_t, int *);                   \
    template hipError_t launch_clip<T>(int64_t, const T *, T *, Box, hipStream_t);              \
    template hipError_t launch_companion<T>(const GeomDev &, const T *, T *, hipStream_t);

TVR_INST(float)
TVR_INST(double)

}  // namespace tvr

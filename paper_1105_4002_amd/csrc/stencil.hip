// Voxel-space kernels: the smoothed-TV stencil (value, gradient, Bregman
// distance), the projected trial step, UPN's extrapolation, the
// Barzilai-Borwein inner products and the slot finaliser.
//
// TV (eq. 2, Huber-smoothed with parameter tau):
//   T_tau(x) = sum_j Phi(D_j x),  Phi(z) = |z| - tau/2 (|z| >= tau),
//   |z|^2 / (2 tau) otherwise, D_j x = forward differences along x, y, z,
//   a component being 0 where the neighbour is outside the volume;
//   grad T_tau(x) = sum_j D_j^T q_j,  q_j = D_j x / max(tau, |D_j x|).
// The gradient stencil runs in the storage type T; Phi values, Bregman
// distances and every sum run in double.
#include "reduce.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

constexpr int VB = 256;  // threads per block for voxel kernels

__device__ __forceinline__ double huber(double n, double tau)
{
    return n >= tau ? n - 0.5 * tau : n * n / (2.0 * tau);
}

// Bregman distance Phi(a) - Phi(b) - grad Phi(b)^T (a - b) with d = a - b,
// written per smoothing regime so that it is formed from d without
// cancellation (each case follows from |a|^2 = |b|^2 + 2 b.d + |d|^2).
__device__ __forceinline__ double huber_bregman(double a0, double a1, double a2, double b0,
                                                double b1, double b2, double d0, double d1,
                                                double d2, double tau)
{
    const double na = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
    const double nb = sqrt(b0 * b0 + b1 * b1 + b2 * b2);
    const double dd = d0 * d0 + d1 * d1 + d2 * d2;
    if (na < tau && nb < tau)
        return dd / (2.0 * tau);
    if (na >= tau && nb >= tau) {
        // |a| (1 - cos) = |a|/2 |a/|a| - b/|b||^2, the unit-vector difference
        // expanded as d/|a| - (b/|b|) ((a + b).d) / (|a| (|a| + |b|))
        const double sc = ((a0 + b0) * d0 + (a1 + b1) * d1 + (a2 + b2) * d2) / (na * (na + nb));
        const double ib = 1.0 / nb, ia = 1.0 / na;
        const double e0 = d0 * ia - b0 * ib * sc;
        const double e1 = d1 * ia - b1 * ib * sc;
        const double e2 = d2 * ia - b2 * ib * sc;
        return 0.5 * na * (e0 * e0 + e1 * e1 + e2 * e2);
    }
    if (na >= tau) {
        const double t = na - tau;
        return fmax((dd - t * t) / (2.0 * tau), 0.0);
    }
    const double ib = tau / nb;
    const double e0 = a0 - b0 * ib, e1 = a1 - b1 * ib, e2 = a2 - b2 * ib;
    return (e0 * e0 + e1 * e1 + e2 * e2) / (2.0 * tau);
}

// q = D / max(tau, |D|) at voxel j in storage precision
template <typename T>
__device__ __forceinline__ void qvec(const T *__restrict__ y, size_t j, bool hx, bool hy, bool hz,
                                     size_t sy, size_t sz, T tau, T &qx, T &qy, T &qz)
{
    const T yj = y[j];
    const T dx = hx ? y[j + 1] - yj : T(0);
    const T dy = hy ? y[j + sy] - yj : T(0);
    const T dz = hz ? y[j + sz] - yj : T(0);
    const T n = sqrt(dx * dx + dy * dy + dz * dz);
    const T den = n > tau ? n : tau;
    qx = dx / den;
    qy = dy / den;
    qz = dz / den;
}

template <typename T>
__global__ __launch_bounds__(VB) void tv_kernel(int nx, int ny, int nz, double tau, double alpha,
                                                const T *__restrict__ y,
                                                const T *__restrict__ xref,
                                                const T *__restrict__ gin, T *__restrict__ gout,
                                                double *__restrict__ partials, int pstride)
{
    const size_t N = (size_t)nx * ny * nz;
    const size_t j = (size_t)blockIdx.x * VB + threadIdx.x;
    double red[3] = {0.0, 0.0, 0.0};
    if (j < N) {
        const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
        const int ix = (int)(j % nx);
        const int iy = (int)((j / nx) % ny);
        const int iz = (int)(j / sz);
        const bool hx = ix + 1 < nx, hy = iy + 1 < ny, hz = iz + 1 < nz;
        const T tt = (T)tau;
        // own differences (value, Bregman, own q)
        const T yj = y[j];
        const T dx = hx ? y[j + 1] - yj : T(0);
        const T dy = hy ? y[j + sy] - yj : T(0);
        const T dz = hz ? y[j + sz] - yj : T(0);
        // the value's differences are formed in double (exact for FP32 data)
        const double yd = (double)yj;
        const double b0 = hx ? (double)y[j + 1] - yd : 0.0;
        const double b1 = hy ? (double)y[j + sy] - yd : 0.0;
        const double b2 = hz ? (double)y[j + sz] - yd : 0.0;
        red[0] = huber(sqrt(b0 * b0 + b1 * b1 + b2 * b2), tau);
        if (gout) {
            const T n = sqrt(dx * dx + dy * dy + dz * dz);
            const T den = n > tt ? n : tt;
            T gj = -(dx + dy + dz) / den;
            T qx, qy, qz;
            if (ix > 0) {
                qvec(y, j - 1, true, hy, hz, sy, sz, tt, qx, qy, qz);
                gj += qx;
            }
            if (iy > 0) {
                qvec(y, j - sy, hx, true, hz, sy, sz, tt, qx, qy, qz);
                gj += qy;
            }
            if (iz > 0) {
                qvec(y, j - sz, hx, hy, true, sy, sz, tt, qx, qy, qz);
                gj += qz;
            }
            if (gin)
                gout[j] = (T)((double)gin[j] + alpha * (double)gj);
            else
                gout[j] = (T)(alpha * (double)gj);
        }
        if (xref) {
            const double ej = (double)xref[j] - (double)yj;
            const double xj = (double)xref[j];
            const double a0 = hx ? (double)xref[j + 1] - xj : 0.0;
            const double a1 = hy ? (double)xref[j + sy] - xj : 0.0;
            const double a2 = hz ? (double)xref[j + sz] - xj : 0.0;
            const double d0 = hx ? ((double)xref[j + 1] - (double)y[j + 1]) - ej : 0.0;
            const double d1 = hy ? ((double)xref[j + sy] - (double)y[j + sy]) - ej : 0.0;
            const double d2 = hz ? ((double)xref[j + sz] - (double)y[j + sz]) - ej : 0.0;
            red[1] = huber_bregman(a0, a1, a2, b0, b1, b2, d0, d1, d2, tau);
            red[2] = ej * ej;
        }
    }
    if (partials) {
        const int slots[3] = {S_TVY, S_BRY, S_XY2};
        block_reduce_store<3>(red, partials, pstride, slots);
    }
}

template <typename T>
__device__ __forceinline__ T pstep(const T *__restrict__ z, const T *__restrict__ g, size_t k,
                                   double step)
{
    return (T)fmax((double)z[k] - step * (double)g[k], 0.0);
}

template <typename T>
__global__ __launch_bounds__(VB) void trial_kernel(int nx, int ny, int nz, double tau,
                                                   const T *__restrict__ z,
                                                   const T *__restrict__ g, double step,
                                                   double gm_step, T *__restrict__ xbar,
                                                   double *__restrict__ partials, int pstride)
{
    const size_t N = (size_t)nx * ny * nz;
    const size_t j = (size_t)blockIdx.x * VB + threadIdx.x;
    double red[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (j < N) {
        const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
        const int ix = (int)(j % nx);
        const int iy = (int)((j / nx) % ny);
        const int iz = (int)(j / sz);
        const bool hx = ix + 1 < nx, hy = iy + 1 < ny, hz = iz + 1 < nz;
        const T xj = pstep(z, g, j, step);
        xbar[j] = xj;
        const double zj = (double)z[j];
        const double ej = (double)xj - zj;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
        if (hx) {
            const T xn = pstep(z, g, j + 1, step);
            const double zn = (double)z[j + 1];
            a0 = (double)xn - (double)xj;
            b0 = zn - zj;
            d0 = ((double)xn - zn) - ej;
        }
        if (hy) {
            const T xn = pstep(z, g, j + sy, step);
            const double zn = (double)z[j + sy];
            a1 = (double)xn - (double)xj;
            b1 = zn - zj;
            d1 = ((double)xn - zn) - ej;
        }
        if (hz) {
            const T xn = pstep(z, g, j + sz, step);
            const double zn = (double)z[j + sz];
            a2 = (double)xn - (double)xj;
            b2 = zn - zj;
            d2 = ((double)xn - zn) - ej;
        }
        const double gj = (double)g[j];
        red[0] = ej * ej;
        red[1] = -gj * ej;
        red[2] = huber(sqrt(a0 * a0 + a1 * a1 + a2 * a2), tau);
        red[3] = huber_bregman(a0, a1, a2, b0, b1, b2, d0, d1, d2, tau);
        if (gm_step > 0.0) {
            const double p = zj - fmax(zj - gm_step * gj, 0.0);
            red[4] = p * p;
        }
    }
    const int slots[5] = {S_XD2, S_GD, S_TVB, S_BRB, S_GM2};
    block_reduce_store<5>(red, partials, pstride, slots);
}

constexpr int EW_MAX_BLOCKS = 4096;

// xt[z][x][y] = x[z][y][x] through a 32 x 32 LDS tile per block (both the
// read and the write are coalesced); the padding column avoids bank conflicts.
constexpr int TR = 32;

template <typename T>
__global__ __launch_bounds__(256) void transpose_xy_kernel(int nx, int ny, const T *__restrict__ x,
                                                           T *__restrict__ xt)
{
    __shared__ T tile[TR][TR + 1];
    const size_t plane = (size_t)nx * ny;
    const T *xs = x + (size_t)blockIdx.z * plane;
    T *xd = xt + (size_t)blockIdx.z * plane;
    const int bx = blockIdx.x * TR, by = blockIdx.y * TR;
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
                                                  T *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VB) {
        const T v = in[i];
        out[i] = v > T(0) ? v : T(0);
    }
}

__global__ __launch_bounds__(VB) void finalize_kernel(SlotList sl, const double *__restrict__ partials,
                                                      int pstride)
{
    const int q = blockIdx.x;
    const int slot = sl.slot[q], count = sl.count[q];
    const double *p = partials + (size_t)slot * pstride;
    double red[1] = {0.0};
    for (int i = threadIdx.x; i < count; i += VB)
        red[0] += p[i];
    __shared__ double sh[VB / 64];
    double s = wave_sum(red[0]);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < VB / 64; ++w)
            t += sh[w];
        *sl.dst[q] = t;
    }
}

__global__ void combine_phi_kernel(const double *r2, const double *tv, double alpha, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *out = 0.5 * (*r2) + alpha * (*tv);
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
    const int64_t N = (int64_t)nx * ny * nz;
    return (int)((N + VB - 1) / VB);
}

template <typename T>
hipError_t launch_tv(int nx, int ny, int nz, double tau, double alpha, const T *y, const T *xref,
                     const T *gin, T *gout, double *partials, int pstride, hipStream_t st,
                     int *nblocks)
{
    const int nb = max_reduce_blocks_vol(nx, ny, nz);
    if (nblocks)
        *nblocks = nb;
    hipLaunchKernelGGL((tv_kernel<T>), dim3(nb), dim3(VB), 0, st, nx, ny, nz, tau, alpha, y, xref,
                       gin, gout, partials, pstride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_trial(int nx, int ny, int nz, double tau, const T *z, const T *g, double step,
                        double gm_step, T *xbar, double *partials, int pstride, hipStream_t st,
                        int *nblocks)
{
    const int nb = max_reduce_blocks_vol(nx, ny, nz);
    if (nblocks)
        *nblocks = nb;
    hipLaunchKernelGGL((trial_kernel<T>), dim3(nb), dim3(VB), 0, st, nx, ny, nz, tau, z, g, step,
                       gm_step, xbar, partials, pstride);
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
hipError_t launch_transpose_xy(int nx, int ny, int nz, const T *x, T *xt, hipStream_t st)
{
    dim3 grid((nx + TR - 1) / TR, (ny + TR - 1) / TR, nz);
    hipLaunchKernelGGL((transpose_xy_kernel<T>), grid, dim3(256), 0, st, nx, ny, x, xt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_clip(int64_t n, const T *in, T *out, hipStream_t st)
{
    hipLaunchKernelGGL((clip_kernel<T>), dim3(elementwise_blocks(n)), dim3(VB), 0, st, n, in, out);
    return hipGetLastError();
}

hipError_t launch_finalize(const SlotList &sl, const double *partials, int pstride,
                           hipStream_t st)
{
    if (sl.n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(sl.n), dim3(VB), 0, st, sl, partials, pstride);
    return hipGetLastError();
}

hipError_t launch_combine_phi(const double *r2, const double *tv, double alpha, double *out,
                              hipStream_t st)
{
    hipLaunchKernelGGL(combine_phi_kernel, dim3(1), dim3(64), 0, st, r2, tv, alpha, out);
    return hipGetLastError();
}

#define TVR_INST(T)                                                                              \
    template hipError_t launch_tv<T>(int, int, int, double, double, const T *, const T *,       \
                                     const T *, T *, double *, int, hipStream_t, int *);        \
    template hipError_t launch_trial<T>(int, int, int, double, const T *, const T *, double,     \
                                        double, T *, double *, int, hipStream_t, int *);        \
    template hipError_t launch_extrapolate<T>(int64_t, double, const T *, const T *, T *,       \
                                              double *, int, hipStream_t, int *);               \
    template hipError_t launch_bb_dots<T>(int64_t, const T *, const T *, const T *, const T *,  \
                                          double *, int, hipStream_t, int *);                   \
    template hipError_t launch_clip<T>(int64_t, const T *, T *, hipStream_t);                   \
    template hipError_t launch_transpose_xy<T>(int, int, int, const T *, T *, hipStream_t);

TVR_INST(float)
TVR_INST(double)

}  // namespace tvr

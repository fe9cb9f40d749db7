// Voxel- and ray-space kernels of the differentiated form (reverse mode
// through unrolled UPN steps): the Hessian-vector product of the smoothed TV
// fused with the adjoint update it feeds, the projection mask, linear
// combinations, and the adjoint of the extrapolation step of Alg. 3.
//
// TV Hessian: with a_j = D_j y, e_j = D_j v and n_j = |a_j|,
//   H(y) v = sum_j D_j^T dq_j,
//   dq_j = e_j / tau                                  (n_j <  tau)
//   dq_j = (e_j - a_j (a_j . e_j) / n_j^2) / n_j       (n_j >= tau),
// the derivative of q_j = a_j / max(tau, n_j) along v.  The same pass gives
// <v, grad T(y)> = sum_j q_j . e_j (the adjoint identity of D), so the
// gradient itself is never formed.
#include "reduce.hpp"
#include "stencil_math.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

// dq of one voxel from its differences a (of y) and e (of v); q . e on the side
template <typename T>
__device__ __forceinline__ void hess_dq(T a0, T a1, T a2, T e0, T e1, T e2, T ct, T itau, T &d0,
                                        T &d1, T &d2, T &qe)
{
    const T s2 = a0 * a0 + a1 * a1 + a2 * a2;
    const T inv = SM<T>::inv_clamped(s2, ct, itau);  // 1 / max(tau, n)
    const T ae = a0 * e0 + a1 * e1 + a2 * e2;
    qe = ae * inv;
    const T k = SM<T>::norm(s2) >= ct ? ae * inv * inv : T(0);
    d0 = (e0 - a0 * k) * inv;
    d1 = (e1 - a1 * k) * inv;
    d2 = (e2 - a2 * k) * inv;
}

// out = in + ca u + cb w + ch H(y) u  (in, w may be NULL; out may be in); with
// partials, slot S_AD1 gets <u, grad T(y)>.  One thread per (x, y) column marching up VZ planes, the
// z component of the plane below carried along.
template <typename T>
__global__ __launch_bounds__(VX *VY) void hessvec_kernel(int nx, int ny, int nz, double tau,
                                                         const T *__restrict__ y,
                                                         const T *__restrict__ u,
                                                         const T *in,
                                                         const T *__restrict__ w, double ca,
                                                         double cb, double ch, T *out,
                                                         double *__restrict__ partials,
                                                         int pstride)
{
    const int ix = blockIdx.x * VX + threadIdx.x;
    const int iy = blockIdx.y * VY + threadIdx.y;
    const int z0 = blockIdx.z * VZ;
    const int z1 = min(z0 + VZ, nz);
    double red[1] = {0.0};
    if (ix < nx && iy < ny) {
        const T ct = (T)tau, itau = T(1) / ct;
        const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
        const bool hx = ix + 1 < nx, hy = iy + 1 < ny, lx = ix > 0, ly = iy > 0;
        T dz_prev = T(0);
        T t0, t1, qe;
        if (z0 > 0) {
            const size_t jb = (size_t)ix + sy * iy + sz * (z0 - 1);
            const T yb = y[jb], ub = u[jb];
            const T a0 = hx ? y[jb + 1] - yb : T(0), e0 = hx ? u[jb + 1] - ub : T(0);
            const T a1 = hy ? y[jb + sy] - yb : T(0), e1 = hy ? u[jb + sy] - ub : T(0);
            const T a2 = y[jb + sz] - yb, e2 = u[jb + sz] - ub;
            hess_dq<T>(a0, a1, a2, e0, e1, e2, ct, itau, t0, t1, dz_prev, qe);
        }
        for (int z = z0; z < z1; ++z) {
            const size_t j = (size_t)ix + sy * iy + sz * z;
            const bool hz = z + 1 < nz;
            const T yj = y[j], uj = u[j];
            const T a0 = hx ? y[j + 1] - yj : T(0), e0 = hx ? u[j + 1] - uj : T(0);
            const T a1 = hy ? y[j + sy] - yj : T(0), e1 = hy ? u[j + sy] - uj : T(0);
            const T a2 = hz ? y[j + sz] - yj : T(0), e2 = hz ? u[j + sz] - uj : T(0);
            T d0, d1, d2;
            hess_dq<T>(a0, a1, a2, e0, e1, e2, ct, itau, d0, d1, d2, qe);
            red[0] += (double)qe;
            T h = -(d0 + d1 + d2) + dz_prev;
            dz_prev = d2;
            if (lx) {  // x component of dq at the voxel on the left
                const size_t k = j - 1;
                const T yk = y[k], uk = u[k];
                const T b1 = hy ? y[k + sy] - yk : T(0), f1 = hy ? u[k + sy] - uk : T(0);
                const T b2 = hz ? y[k + sz] - yk : T(0), f2 = hz ? u[k + sz] - uk : T(0);
                T c0, c1, c2, q;
                hess_dq<T>(yj - yk, b1, b2, uj - uk, f1, f2, ct, itau, c0, c1, c2, q);
                h += c0;
            }
            if (ly) {  // y component of dq at the voxel in front
                const size_t k = j - sy;
                const T yk = y[k], uk = u[k];
                const T b0 = hx ? y[k + 1] - yk : T(0), f0 = hx ? u[k + 1] - uk : T(0);
                const T b2 = hz ? y[k + sz] - yk : T(0), f2 = hz ? u[k + sz] - uk : T(0);
                T c0, c1, c2, q;
                hess_dq<T>(b0, yj - yk, b2, f0, uj - uk, f2, ct, itau, c0, c1, c2, q);
                h += c1;
            }
            double o = in ? (double)in[j] : 0.0;
            o += ca * (double)uj + ch * (double)h;
            if (w)
                o += cb * (double)w[j];
            out[j] = (T)o;
        }
    }
    if (partials) {
        const int slots[1] = {S_AD1};
        block_reduce_store<1>(red, partials, pstride, slots);
    }
}

// out = (x > 0) ? g : 0   (the Jacobian of P_Q applied to an adjoint)
template <typename T>
__global__ __launch_bounds__(VB) void mask_kernel(int64_t n, const T *__restrict__ x,
                                                  const T *__restrict__ g, T *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n; i += (int64_t)gridDim.x * VB)
        out[i] = x[i] > T(0) ? g[i] : T(0);
}

// out = in + a u + b v (in, u, v may be NULL: zero)
template <typename T>
__global__ __launch_bounds__(VB) void lincomb_kernel(int64_t n, const T *in, double a, const T *u,
                                                     double b, const T *v, T *out)
{
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VB) {
        double o = in ? (double)in[i] : 0.0;
        if (u)
            o += a * (double)u[i];
        if (v)
            o += b * (double)v[i];
        out[i] = (T)o;
    }
}

// Adjoint of y+ = x+ + beta (x+ - x): xbar+ += (1 + beta) ybar,
// xbar += -beta ybar, and slot S_AD2 = <ybar, x+ - x> (the adjoint of beta).
template <typename T>
__global__ __launch_bounds__(VB) void adj_extrap_kernel(int64_t n, double beta,
                                                        const T *__restrict__ ybar,
                                                        const T *__restrict__ xn,
                                                        const T *__restrict__ xo,
                                                        T *__restrict__ xbar_n,
                                                        T *__restrict__ xbar_o,
                                                        double *__restrict__ partials,
                                                        int pstride)
{
    double red[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * VB + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * VB) {
        const double yb = (double)ybar[i];
        red[0] += yb * ((double)xn[i] - (double)xo[i]);
        xbar_n[i] = (T)((double)xbar_n[i] + (1.0 + beta) * yb);
        xbar_o[i] = (T)((double)xbar_o[i] - beta * yb);
    }
    const int slots[1] = {S_AD2};
    block_reduce_store<1>(red, partials, pstride, slots);
}

}  // namespace

template <typename T>
hipError_t launch_hessvec(int nx, int ny, int nz, double tau, const T *y, const T *u, const T *in,
                          const T *w, double ca, double cb, double ch, T *out, double *partials,
                          int pstride, hipStream_t st, int *nblocks)
{
    const dim3 gr((nx + VX - 1) / VX, (ny + VY - 1) / VY, (nz + VZ - 1) / VZ);
    if (nblocks)
        *nblocks = (int)(gr.x * gr.y * gr.z);
    hipLaunchKernelGGL((hessvec_kernel<T>), gr, dim3(VX, VY), 0, st, nx, ny, nz, tau, y, u, in, w,
                       ca, cb, ch, out, partials, pstride);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mask(int64_t n, const T *x, const T *g, T *out, hipStream_t st)
{
    hipLaunchKernelGGL((mask_kernel<T>), dim3(elementwise_blocks_dev(n)), dim3(VB), 0, st, n, x, g,
                       out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lincomb(int64_t n, const T *in, double a, const T *u, double b, const T *v,
                          T *out, hipStream_t st)
{
    hipLaunchKernelGGL((lincomb_kernel<T>), dim3(elementwise_blocks_dev(n)), dim3(VB), 0, st, n, in,
                       a, u, b, v, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_extrap(int64_t n, double beta, const T *ybar, const T *xn, const T *xo,
                             T *xbar_n, T *xbar_o, double *partials, int pstride, hipStream_t st,
                             int *nblocks)
{
    const int nb = elementwise_blocks_dev(n);
    if (nblocks)
        *nblocks = nb;
    hipLaunchKernelGGL((adj_extrap_kernel<T>), dim3(nb), dim3(VB), 0, st, n, beta, ybar, xn, xo,
                       xbar_n, xbar_o, partials, pstride);
    return hipGetLastError();
}

#define TVR_INST_ADJ(T)                                                                          \
    template hipError_t launch_hessvec<T>(int, int, int, double, const T *, const T *, const T *, \
                                          const T *, double, double, double, T *, double *, int, \
                                          hipStream_t, int *);                                   \
    template hipError_t launch_mask<T>(int64_t, const T *, const T *, T *, hipStream_t);         \
    template hipError_t launch_lincomb<T>(int64_t, const T *, double, const T *, double,         \
                                          const T *, T *, hipStream_t);                          \
    template hipError_t launch_adj_extrap<T>(int64_t, double, const T *, const T *, const T *,   \
                                             T *, T *, double *, int, hipStream_t, int *);

TVR_INST_ADJ(float)
TVR_INST_ADJ(double)

}  // namespace tvr

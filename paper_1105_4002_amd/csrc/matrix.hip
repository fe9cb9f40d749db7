// Stored transpose: A^T built once from the same ray tables and crossing
// formula as the on-the-fly gather, then applied as a bandwidth-bound
// sparse product.
//
// The paper takes A as given (the system matrix of Sec. II-A).  The gather
// backprojector spends most of its time re-deriving each ray/voxel length
// from the geometry (about 115 vector instructions per voxel and view); with
// 288 GB of HBM per GPU the voxel-major copy of a 256^3 scan (1.3e9
// non-zeros, 12 GB in FP32) is cheaper to stream (2.4 ms against 3.7 ms).
// The forward projector keeps its on-the-fly walk: it reads no matrix at
// all and beats streaming a ray-major copy (1.9 ms; a ray-major product
// measured 3.6 ms on the 256^3 scan).
//
// Layout: sliced ELLPACK with 8 x 8 voxel tiles as slices (one wavefront;
// the mapping is mat_slot / mat_voxel); entry k of lane l of slice s sits at
// off[s] + 64 k + l, so every step of a wavefront loads 64 consecutive
// values and indices.  A tile's voxels project onto a compact detector
// patch in every view, which keeps a step's gathers of r within a few cache
// lines (measured on the 256^3 scan: 2.27 ms against 2.77 ms for slices of
// 64 consecutive voxels along x).  A slice is as wide as its longest lane;
// shorter lanes are padded with zero weights on a ray index they already
// read, so the product loop is branch free; lanes of an edge tile past the
// volume have width 0.  The entries of a voxel follow the gather's order
// (views, then detector columns, then rows): a_ij = (t_exit - t_enter) |D_i|
// from the gather's enumeration, rounded once to T.  The product
// accumulates in double.
#include "gather.hpp"
#include "ray3d.hpp"
#include "reduce.hpp"
#include "tvreg_internal.hpp"

namespace tvr {

namespace {

constexpr int MB = 256;      // threads per block of the sparse products
constexpr int CT_TX = 16;    // build: voxel columns per block along x, y
constexpr int CT_TY = 16;
constexpr int CT_CZ = 8;     // build: voxels per thread along z

__device__ __forceinline__ double ray_dnorm(const GeomDev &g, int v, int row, int col)
{
    return g.cone ? g.dnorm[(size_t)row * g.cols + col] : g.dnorm[v];
}

// ---------------------------------------------------------------- counting

template <bool CONE>
__global__ __launch_bounds__(CT_TX *CT_TY) void count_voxels_kernel(GeomDev g,
                                                                   int32_t *__restrict__ cnt)
{
    const int ix = blockIdx.x * CT_TX + (threadIdx.x % CT_TX);
    const int iy = blockIdx.y * CT_TY + (threadIdx.x / CT_TX);
    const int iz0 = blockIdx.z * CT_CZ;
    if (ix >= g.nx || iy >= g.ny)
        return;
    const double X0 = -g.hx + (double)ix, X1 = X0 + 1.0;
    const double Y0 = -g.hy + (double)iy, Y1 = Y0 + 1.0;
    int n[CT_CZ];
#pragma unroll
    for (int k = 0; k < CT_CZ; ++k)
        n[k] = 0;
    for (int v = 0; v < g.nviews; ++v) {
        if (g.beam3d) {  // launch-uniform
            gather3d_visit<CT_CZ>(g, v, X0, X1, Y0, Y1, iz0,
                                  [&](int k, int, int, double) { n[k]++; });
            continue;
        }
        const GlobalSrc<float, CONE> src{&g, g.col + (size_t)v * g.cols, nullptr, 0.0};
        gather_view_visit<CONE, CT_CZ>(g, src, g.cs[v].x, g.cs[v].y, X0, X1, Y0, Y1, iz0, 0,
                                       g.cols - 1, 0, g.rows - 1,
                                       [&](int k, int, int, double) { n[k]++; });
    }
    const size_t plane = (size_t)g.nx * g.ny;
#pragma unroll
    for (int k = 0; k < CT_CZ; ++k)
        if (iz0 + k < g.nz)
            cnt[(size_t)(iz0 + k) * plane + (size_t)iy * g.nx + ix] = n[k];
}

// one wavefront per slice
__global__ __launch_bounds__(MB) void slice_width_kernel(int nx, int ny, int64_t sv,
                                                         const int32_t *__restrict__ cnt,
                                                         int32_t *__restrict__ w)
{
    const int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x;
    const int64_t s = i >> 6;
    int x, y, z, c = 0;
    if (s < sv && mat_voxel(nx, ny, s, (int)(i & 63), x, y, z))
        c = cnt[((size_t)z * ny + y) * nx + x];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        c = max(c, __shfl_xor(c, off, 64));
    if ((threadIdx.x & 63) == 0 && s < sv)
        w[s] = c;
}

// ------------------------------------------------------------------ filling

template <typename T, bool CONE>
__global__ __launch_bounds__(CT_TX *CT_TY) void fill_voxels_kernel(GeomDev g, T *__restrict__ val,
                                                                  int32_t *__restrict__ idx)
{
    const int ix = blockIdx.x * CT_TX + (threadIdx.x % CT_TX);
    const int iy = blockIdx.y * CT_TY + (threadIdx.x / CT_TX);
    const int iz0 = blockIdx.z * CT_CZ;
    if (ix >= g.nx || iy >= g.ny)
        return;
    const double X0 = -g.hx + (double)ix, X1 = X0 + 1.0;
    const double Y0 = -g.hy + (double)iy, Y1 = Y0 + 1.0;
    const size_t plane = (size_t)g.nx * g.ny;
    int64_t pos[CT_CZ], end[CT_CZ];
    int32_t last[CT_CZ];
#pragma unroll
    for (int k = 0; k < CT_CZ; ++k) {
        int64_t s;
        int l;
        mat_slot(g.nx, g.ny, ix, iy, iz0 + k < g.nz ? iz0 + k : 0, s, l);
        pos[k] = g.mat.off_v[s] + l;
        end[k] = pos[k] + 64 * (int64_t)g.mat.w_v[s];
        last[k] = 0;
    }
    for (int v = 0; v < g.nviews; ++v) {
        const int64_t vbase = (int64_t)v * g.rows * g.cols;
        auto put = [&](int k, int row, int col, double len) {
            if (pos[k] >= end[k])
                return;  // never past the lane's slots (the count pass bounds it)
            const int32_t i = (int32_t)(vbase + (int64_t)row * g.cols + col);
            val[pos[k]] = (T)(len * ray_dnorm(g, v, row, col));
            idx[pos[k]] = i;
            last[k] = i;
            pos[k] += 64;
        };
        if (g.beam3d) {  // launch-uniform
            gather3d_visit<CT_CZ>(g, v, X0, X1, Y0, Y1, iz0, put);
            continue;
        }
        const GlobalSrc<float, CONE> src{&g, g.col + (size_t)v * g.cols, nullptr, 0.0};
        gather_view_visit<CONE, CT_CZ>(g, src, g.cs[v].x, g.cs[v].y, X0, X1, Y0, Y1, iz0, 0,
                                       g.cols - 1, 0, g.rows - 1, put);
    }
#pragma unroll
    for (int k = 0; k < CT_CZ; ++k) {
        if (iz0 + k < g.nz) {
            for (int64_t p = pos[k]; p < end[k]; p += 64) {  // padding
                val[p] = T(0);
                idx[p] = last[k];
            }
        }
    }
}

// ---------------------------------------------------------- sparse products

// x = A^T r, one thread per voxel (lane of a tile slice); block `blk` of the
// product
template <typename T>
__device__ __forceinline__ void spmv_voxels_block(const GeomDev &g, const T *__restrict__ r,
                                                  T *__restrict__ out, int blk)
{
    const int64_t j = (int64_t)blk * MB + threadIdx.x;
    const int64_t s = j >> 6;
    if (s >= g.mat.sv)
        return;
    int x, y, z;
    const bool in = mat_voxel(g.nx, g.ny, s, (int)(j & 63), x, y, z);
    const T *__restrict__ val = (const T *)g.mat.val_v + g.mat.off_v[s] + (j & 63);
    const int32_t *__restrict__ idx = g.mat.idx_v + g.mat.off_v[s] + (j & 63);
    const int w = in ? g.mat.w_v[s] : 0;  // lanes past the volume hold no entries
    double acc = 0.0;
    // the matrix is read once per product: non-temporal loads keep it from
    // evicting r, which every voxel gathers from
#pragma unroll 8
    for (int k = 0; k < w; ++k) {
        const T a = __builtin_nontemporal_load(val + 64 * k);
        const int32_t i = __builtin_nontemporal_load(idx + 64 * k);
        acc = fma((double)a, (double)r[i], acc);
    }
    if (in)
        out[((size_t)z * g.ny + y) * g.nx + x] = (T)acc;
}

template <typename T>
__global__ __launch_bounds__(MB) void spmv_voxels_kernel(GeomDev g, const T *__restrict__ r,
                                                         T *__restrict__ out)
{
    spmv_voxels_block<T>(g, r, out, blockIdx.x);
}

// Batched: G = A^T RY for every problem with a stored transpose whose
// gradient is due this round.
template <typename T>
__global__ __launch_bounds__(MB) void spmv_grouped(BatchProblem<T> *probs, const int *offs, int n)
{
    const int p = find_problem(offs, n, blockIdx.x);
    const BatchProblem<T> &P = probs[p];
    if (P.state != B_RUNNING || !P.need_grad)
        return;
    spmv_voxels_block<T>(P.g, P.RY, P.G, blockIdx.x - offs[p]);
}

int blocks_for(int64_t n) { return (int)((n + MB - 1) / MB); }

}  // namespace

int matrix_product_blocks(const GeomDev &g) { return blocks_for(64 * mat_slices(g.nx, g.ny, g.nz)); }

template <typename T>
hipError_t launch_spmv_grouped(BatchProblem<T> *probs, const int *offs, int n, int blocks,
                               hipStream_t st)
{
    hipLaunchKernelGGL((spmv_grouped<T>), dim3(blocks), dim3(MB), 0, st, probs, offs, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_backproject_matrix(const GeomDev &g, const T *r, T *out, hipStream_t st)
{
    hipLaunchKernelGGL((spmv_voxels_kernel<T>), dim3(matrix_product_blocks(g)), dim3(MB), 0, st, g,
                       r, out);
    return hipGetLastError();
}

hipError_t launch_matrix_count(const GeomDev &g, int32_t *cnt_v, hipStream_t st)
{
    const dim3 gv((g.nx + CT_TX - 1) / CT_TX, (g.ny + CT_TY - 1) / CT_TY,
                  (g.nz + CT_CZ - 1) / CT_CZ);
    if (g.cone)
        hipLaunchKernelGGL((count_voxels_kernel<true>), gv, dim3(CT_TX * CT_TY), 0, st, g, cnt_v);
    else
        hipLaunchKernelGGL((count_voxels_kernel<false>), gv, dim3(CT_TX * CT_TY), 0, st, g,
                           cnt_v);
    return hipGetLastError();
}

hipError_t launch_slice_widths(const GeomDev &g, const int32_t *cnt, int32_t *w, hipStream_t st)
{
    const int64_t sv = mat_slices(g.nx, g.ny, g.nz);
    hipLaunchKernelGGL(slice_width_kernel, dim3(blocks_for(64 * sv)), dim3(MB), 0, st, g.nx, g.ny,
                       sv, cnt, w);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_matrix_fill(const GeomDev &g, T *val_v, int32_t *idx_v, hipStream_t st)
{
    const dim3 gv((g.nx + CT_TX - 1) / CT_TX, (g.ny + CT_TY - 1) / CT_TY,
                  (g.nz + CT_CZ - 1) / CT_CZ);
    if (g.cone)
        hipLaunchKernelGGL((fill_voxels_kernel<T, true>), gv, dim3(CT_TX * CT_TY), 0, st, g,
                           val_v, idx_v);
    else
        hipLaunchKernelGGL((fill_voxels_kernel<T, false>), gv, dim3(CT_TX * CT_TY), 0, st, g,
                           val_v, idx_v);
    return hipGetLastError();
}

#define TVR_INST_MAT(T)                                                                          \
    template hipError_t launch_backproject_matrix<T>(const GeomDev &, const T *, T *,            \
                                                     hipStream_t);                               \
    template hipError_t launch_matrix_fill<T>(const GeomDev &, T *, int32_t *, hipStream_t);     \
    template hipError_t launch_spmv_grouped<T>(BatchProblem<T> *, const int *, int, int,        \
                                               hipStream_t);

TVR_INST_MAT(float)
TVR_INST_MAT(double)

}  // namespace tvr

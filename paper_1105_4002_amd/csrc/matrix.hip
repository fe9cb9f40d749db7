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
    if (ix >= g.mat.mx || iy >= g.mat.my)
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
    const size_t plane = (size_t)g.mat.mx * g.mat.my;
#pragma unroll
    for (int k = 0; k < CT_CZ; ++k)
        if (iz0 + k < g.mat.mz)
            cnt[(size_t)(iz0 + k) * plane + (size_t)iy * g.mat.mx + ix] = n[k];
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
    const MatDev &M = g.mat;
    if (ix >= M.mx || iy >= M.my)
        return;
    const double X0 = -g.hx + (double)ix, X1 = X0 + 1.0;
    const double Y0 = -g.hy + (double)iy, Y1 = Y0 + 1.0;
    const bool keyed = M.rot > 1 || M.mir;
    int64_t pos[CT_CZ], end[CT_CZ];
    int32_t last[CT_CZ];
#pragma unroll
    for (int k = 0; k < CT_CZ; ++k) {
        // voxels past the stored cell (inside the volume when the cell is
        // the lower half in z) get no slots: put() then skips their entries
        const bool kept = iz0 + k < M.mz;
        int64_t s;
        int l;
        mat_slot(M.mx, M.my, ix, iy, kept ? iz0 + k : 0, s, l);
        pos[k] = M.off_v[s] + l;
        end[k] = kept ? pos[k] + 64 * (int64_t)M.w_v[s] : pos[k];
        last[k] = 0;
    }
    for (int v = 0; v < g.nviews; ++v) {
        const int64_t vbase = (int64_t)v * g.rows * g.cols;
        auto put = [&](int k, int row, int col, double len) {
            if (pos[k] >= end[k])
                return;  // never past the lane's slots (the count pass bounds it)
            const int32_t i = keyed ? (int32_t)(((uint32_t)v << (M.kc + M.kr)) |
                                                ((uint32_t)row << M.kc) | (uint32_t)col)
                                    : (int32_t)(vbase + (int64_t)row * g.cols + col);
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
        if (iz0 + k < M.mz) {
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

// An entry of r: with BUF `off` is a byte offset read through a buffer
// resource (32-bit, no 64-bit address arithmetic), else an element index.
template <typename T, bool BUF>
__device__ __forceinline__ double load_r(const T *__restrict__ r, __amdgpu_buffer_rsrc_t rs,
                                         unsigned off)
{
    if (BUF) {
        if (sizeof(T) == 4)
            return (double)__builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
    }
    return (double)r[off];
}

// The same product from a symmetric layout: one thread per voxel of the
// stored cell, each entry (a, key) applied to all ROT (x 2 with MIR) images
// of the voxel: image q of the turn reads view v + q V / ROT, the mirrored
// image reads row rows - 1 - row.  Each image sums its rays in the stored
// order (views from its own first one, cyclically), in double.  The offset
// into r is advanced by V / ROT views per image and wrapped at the end of r;
// it counts bytes with BUF (r under 2^31 bytes, read through a buffer
// resource), elements otherwise (fewer than 2^31), so it fits 32 bits.
template <typename T, int ROT, bool MIR, bool BUF>
__device__ __forceinline__ void spmv_sym_block(const GeomDev &g, const T *__restrict__ r,
                                               T *__restrict__ out, int blk)
{
    const MatDev &M = g.mat;
    const int64_t j = (int64_t)blk * MB + threadIdx.x;
    const int64_t s = j >> 6;
    if (s >= M.sv)
        return;
    int x, y, z;
    const bool in = mat_voxel(M.mx, M.my, s, (int)(j & 63), x, y, z);
    const T *__restrict__ val = (const T *)M.val_v + M.off_v[s] + (j & 63);
    const int32_t *__restrict__ idx = M.idx_v + M.off_v[s] + (j & 63);
    const int w = in ? M.w_v[s] : 0;
    constexpr int NI = ROT * (MIR ? 2 : 1);
    constexpr unsigned ES = BUF ? sizeof(T) : 1u;  // offset units
    const unsigned C = (unsigned)g.cols, R1 = (unsigned)g.rows - 1u;
    const unsigned view_b = (unsigned)g.rows * C * ES;              // bytes of one view
    const unsigned all_b = view_b * (unsigned)g.nviews;             // bytes of r
    const unsigned step_b = view_b * (unsigned)(g.nviews / ROT);    // one image further
    const int shv = M.kc + M.kr;
    const uint32_t mc = (1u << M.kc) - 1u, mr = (1u << M.kr) - 1u;
    // (without BUF the resource is built but never read)
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)r, (short)0, BUF ? (int)all_b : 0, BUF_WORD3);
    double acc[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q)
        acc[q] = 0.0;
#pragma unroll 4
    for (int k = 0; k < w; ++k) {
        const double a = (double)__builtin_nontemporal_load(val + 64 * k);
        const uint32_t key = (uint32_t)__builtin_nontemporal_load(idx + 64 * k);
        const unsigned col = key & mc, row = (key >> M.kc) & mr;
        const unsigned lo = (row * C + col) * ES;
        const unsigned hi = ((R1 - row) * C + col) * ES;
        unsigned base = (key >> shv) * view_b;
#pragma unroll
        for (int q = 0; q < ROT; ++q) {
            acc[q * (MIR ? 2 : 1)] =
                fma(a, load_r<T, BUF>(r, rs, base + lo), acc[q * (MIR ? 2 : 1)]);
            if (MIR)
                acc[2 * q + 1] = fma(a, load_r<T, BUF>(r, rs, base + hi), acc[2 * q + 1]);
            base += step_b;
            base -= base >= all_b ? all_b : 0u;
        }
    }
    if (!in)
        return;
    int xi = x, yi = y;
#pragma unroll
    for (int q = 0; q < ROT; ++q) {
        out[((size_t)z * g.ny + yi) * g.nx + xi] = (T)acc[q * (MIR ? 2 : 1)];
        if (MIR)
            out[((size_t)(g.nz - 1 - z) * g.ny + yi) * g.nx + xi] = (T)acc[2 * q + 1];
        if (ROT == 4) {  // a quarter turn: (i, j) -> (nx - 1 - j, i)
            const int t = xi;
            xi = g.nx - 1 - yi;
            yi = t;
        } else {         // a half turn: (i, j) -> (nx - 1 - i, ny - 1 - j)
            xi = g.nx - 1 - xi;
            yi = g.ny - 1 - yi;
        }
    }
}

// whether r fits a buffer resource (byte offsets below 2^31)
__host__ __device__ __forceinline__ bool sym_buffer_ok(const GeomDev &g, size_t elem)
{
    return elem * (size_t)g.nviews * g.rows * g.cols < (size_t(1) << 31);
}

template <typename T, bool BUF>
__device__ __forceinline__ void spmv_block_buf(const GeomDev &g, const T *__restrict__ r,
                                               T *__restrict__ out, int blk)
{
    if (g.mat.mir) {
        if (g.mat.rot == 4)
            spmv_sym_block<T, 4, true, BUF>(g, r, out, blk);
        else if (g.mat.rot == 2)
            spmv_sym_block<T, 2, true, BUF>(g, r, out, blk);
        else
            spmv_sym_block<T, 1, true, BUF>(g, r, out, blk);
    } else if (g.mat.rot == 4) {
        spmv_sym_block<T, 4, false, BUF>(g, r, out, blk);
    } else {
        spmv_sym_block<T, 2, false, BUF>(g, r, out, blk);
    }
}

template <typename T>
__device__ __forceinline__ void spmv_block(const GeomDev &g, const T *__restrict__ r,
                                           T *__restrict__ out, int blk)
{
    // the layout is uniform over a launch (one problem per block in batches)
    if (g.mat.rot <= 1 && !g.mat.mir)
        spmv_voxels_block<T>(g, r, out, blk);
    else if (sym_buffer_ok(g, sizeof(T)))
        spmv_block_buf<T, true>(g, r, out, blk);
    else
        spmv_block_buf<T, false>(g, r, out, blk);
}

template <typename T>
__global__ __launch_bounds__(MB) void spmv_voxels_kernel(GeomDev g, const T *__restrict__ r,
                                                         T *__restrict__ out)
{
    spmv_voxels_block<T>(g, r, out, blockIdx.x);
}

template <typename T, int ROT, bool MIR, bool BUF>
__global__ __launch_bounds__(MB) void spmv_sym_kernel(GeomDev g, const T *__restrict__ r,
                                                      T *__restrict__ out)
{
    spmv_sym_block<T, ROT, MIR, BUF>(g, r, out, blockIdx.x);
}

template <typename T, bool BUF>
void launch_sym(const GeomDev &g, const T *r, T *out, hipStream_t st)
{
    const dim3 gr(matrix_product_blocks(g));
    if (g.mat.mir) {
        if (g.mat.rot == 4)
            hipLaunchKernelGGL((spmv_sym_kernel<T, 4, true, BUF>), gr, dim3(MB), 0, st, g, r, out);
        else if (g.mat.rot == 2)
            hipLaunchKernelGGL((spmv_sym_kernel<T, 2, true, BUF>), gr, dim3(MB), 0, st, g, r, out);
        else
            hipLaunchKernelGGL((spmv_sym_kernel<T, 1, true, BUF>), gr, dim3(MB), 0, st, g, r, out);
    } else if (g.mat.rot == 4) {
        hipLaunchKernelGGL((spmv_sym_kernel<T, 4, false, BUF>), gr, dim3(MB), 0, st, g, r, out);
    } else {
        hipLaunchKernelGGL((spmv_sym_kernel<T, 2, false, BUF>), gr, dim3(MB), 0, st, g, r, out);
    }
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
    spmv_block<T>(P.g, P.RY, P.G, blockIdx.x - offs[p]);
}

int blocks_for(int64_t n) { return (int)((n + MB - 1) / MB); }

}  // namespace

int matrix_product_blocks(const GeomDev &g) { return blocks_for(64 * g.mat.sv); }

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
    if (g.mat.rot <= 1 && !g.mat.mir)
        hipLaunchKernelGGL((spmv_voxels_kernel<T>), dim3(matrix_product_blocks(g)), dim3(MB), 0,
                           st, g, r, out);
    else if (sym_buffer_ok(g, sizeof(T)))
        launch_sym<T, true>(g, r, out, st);
    else
        launch_sym<T, false>(g, r, out, st);
    return hipGetLastError();
}

hipError_t launch_matrix_count(const GeomDev &g, int32_t *cnt_v, hipStream_t st)
{
    const dim3 gv((g.mat.mx + CT_TX - 1) / CT_TX, (g.mat.my + CT_TY - 1) / CT_TY,
                  (g.mat.mz + CT_CZ - 1) / CT_CZ);
    if (g.cone)
        hipLaunchKernelGGL((count_voxels_kernel<true>), gv, dim3(CT_TX * CT_TY), 0, st, g, cnt_v);
    else
        hipLaunchKernelGGL((count_voxels_kernel<false>), gv, dim3(CT_TX * CT_TY), 0, st, g,
                           cnt_v);
    return hipGetLastError();
}

hipError_t launch_slice_widths(const GeomDev &g, const int32_t *cnt, int32_t *w, hipStream_t st)
{
    const int64_t sv = mat_slices(g.mat.mx, g.mat.my, g.mat.mz);
    hipLaunchKernelGGL(slice_width_kernel, dim3(blocks_for(64 * sv)), dim3(MB), 0, st, g.mat.mx,
                       g.mat.my, sv, cnt, w);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_matrix_fill(const GeomDev &g, T *val_v, int32_t *idx_v, hipStream_t st)
{
    const dim3 gv((g.mat.mx + CT_TX - 1) / CT_TX, (g.mat.my + CT_TY - 1) / CT_TY,
                  (g.mat.mz + CT_CZ - 1) / CT_CZ);
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

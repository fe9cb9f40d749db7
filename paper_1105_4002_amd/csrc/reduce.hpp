// Deterministic block-level FP64 reduction: wavefront (64-lane) shuffle tree,
// then the per-wave sums added in wave order by thread 0.  Every thread of
// the block must call it.
#pragma once

#include <hip/hip_runtime.h>

namespace tvr {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ int block_linear_id()
{
    return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}

__device__ __forceinline__ int thread_linear_id()
{
    return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
}

// Reduces v[0..NQ) over the block; thread 0 writes partials[slot[q] * pstride + bid].
template <int NQ>
__device__ __forceinline__ void block_reduce_store(double (&v)[NQ], double *partials,
                                                   int pstride, const int (&slot)[NQ], int bid)
{
    __shared__ double sh[NQ][16];
    const int tid = thread_linear_id();
    const int lane = tid & 63, wid = tid >> 6;
    const int nthreads = blockDim.x * blockDim.y * blockDim.z;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0)
            sh[q][wid] = s;
    }
    __syncthreads();
    if (tid == 0) {
        const int nw = (nthreads + 63) >> 6;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w)
                s += sh[q][w];
            partials[(size_t)slot[q] * pstride + bid] = s;
        }
    }
}

template <int NQ>
__device__ __forceinline__ void block_reduce_store(double (&v)[NQ], double *partials,
                                                   int pstride, const int (&slot)[NQ])
{
    block_reduce_store<NQ>(v, partials, pstride, slot, block_linear_id());
}

// Problem owning block b of a grouped launch: offs[p] is the first block of
// problem p (offs[0] = 0, increasing).
__device__ __forceinline__ int find_problem(const int *offs, int n, int b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

}  // namespace tvr

// Launch shapes and precision-dependent math shared by the voxel-space
// kernels (TV stencil, trial step, adjoint stencils, elementwise passes).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tvr {

constexpr int VB = 256;    // threads per block for 1-D kernels
constexpr int VX = 64;     // voxel kernels: block of 64 x 4 columns ...
constexpr int VY = 4;
constexpr int VZ = 16;     // ... each marching up 16 voxels
constexpr int EW_MAX_BLOCKS = 4096;

__host__ __device__ __forceinline__ int elementwise_blocks_dev(int64_t n)
{
    int64_t b = (n + VB - 1) / VB;
    if (b > EW_MAX_BLOCKS)
        b = EW_MAX_BLOCKS;
    return (int)(b < 1 ? 1 : b);
}

// Math in the stencil's precision.
template <typename C>
struct SM;

template <>
struct SM<float> {
    // 1 / max(tau, |v|) from |v|^2 (rsq(0) = +inf selects 1/tau)
    static __device__ __forceinline__ float inv_clamped(float d2, float tau, float itau)
    {
        return fminf(__builtin_amdgcn_rsqf(d2), itau);
    }
    static __device__ __forceinline__ float norm(float d2)
    {
        return d2 > 0.f ? d2 * __builtin_amdgcn_rsqf(d2) : 0.f;
    }
    static __device__ __forceinline__ float inv(float x) { return __builtin_amdgcn_rcpf(x); }
};

template <>
struct SM<double> {
    static __device__ __forceinline__ double inv_clamped(double d2, double tau, double)
    {
        return 1.0 / fmax(sqrt(d2), tau);
    }
    static __device__ __forceinline__ double norm(double d2) { return sqrt(d2); }
    static __device__ __forceinline__ double inv(double x) { return 1.0 / x; }
};

}  // namespace tvr

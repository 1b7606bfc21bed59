// Gaussian matrix drawn on the device (the optional G of the projection when
// the caller passes none).  Entry e (row-major) of the l x q matrix takes
// outputs 2e and 2e+1 of the counter-based stream (seed, tag | 2^63) as
// uniforms u1 = ((z >> 11) + 1) 2^-53 in (0, 1] and u2 = (z >> 11) 2^-53 in
// [0, 1), and the Box-Muller transform g = sqrt(-2 ln u1) cos(2 pi u2) gives
// an N(0, 1) value (computed in FP64, then rounded to the output type).
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace ids {

template <class T>
__device__ __forceinline__ void put(T* out, int64_t e, double g);
template <>
__device__ __forceinline__ void put<double>(double* out, int64_t e, double g) { out[e] = g; }
template <>
__device__ __forceinline__ void put<float>(float* out, int64_t e, double g) { out[e] = (float)g; }
template <>
__device__ __forceinline__ void put<uint16_t>(uint16_t* out, int64_t e, double g) {
    // FP64 -> FP32 -> BF16, each round to nearest even
    uint32_t u = __float_as_uint((float)g);
    u += 0x7fffu + ((u >> 16) & 1u);
    out[e] = (uint16_t)(u >> 16);
}

template <class T>
__global__ __launch_bounds__(256) void gauss_kernel(uint64_t key, int64_t count, T* out) {
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) {
        const uint64_t z1 = mix64(key + (uint64_t)(2 * e + 1) * GAMMA);
        const uint64_t z2 = mix64(key + (uint64_t)(2 * e + 2) * GAMMA);
        const double u1 = (double)((z1 >> 11) + 1) * 0x1p-53;
        const double u2 = (double)(z2 >> 11) * 0x1p-53;
        put<T>(out, e, sqrt(-2.0 * log(u1)) * cos(two_pi * u2));
    }
}

ids_status gaussian_fill(uint64_t seed, uint64_t tag, int64_t l, int64_t q, int32_t dtype, void* out, hipStream_t st) {
    const int64_t count = l * q;
    const uint64_t key = stream_key(seed, tag | (1ull << 63));
    const unsigned grid = (unsigned)std::min<int64_t>(4096, (count + 255) / 256);
    if (dtype == IDS_F64)
        hipLaunchKernelGGL(gauss_kernel<double>, dim3(grid), dim3(256), 0, st, key, count, (double*)out);
    else if (dtype == IDS_F32)
        hipLaunchKernelGGL(gauss_kernel<float>, dim3(grid), dim3(256), 0, st, key, count, (float*)out);
    else
        hipLaunchKernelGGL(gauss_kernel<uint16_t>, dim3(grid), dim3(256), 0, st, key, count, (uint16_t*)out);
    return check_launch("gaussian draw");
}

}  // namespace ids

// Finiteness scan of a finished sketch (IDS_CHECK_FINITE): one workgroup
// reads the l x n column-major Y once and writes IDS_OK or IDS_ENONFINITE to
// a device status word.  Streaming read (ids_stream_read): the practical HBM
// read ceiling that the sketch kernels are measured against.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace ids {

constexpr int FC_THREADS = 1024;

template <class T>
__global__ __launch_bounds__(FC_THREADS) void finite_check_kernel(const T* __restrict__ Y, int64_t l, int64_t n,
                                                                  int64_t ldy, int32_t* status) {
    bool bad = false;
    const int64_t total = l * n;
    for (int64_t e = threadIdx.x; e < total; e += FC_THREADS) {
        const int64_t j = e / l, i = e - j * l;
        bad = bad || !__builtin_isfinite((double)Y[j * ldy + i]);
    }
    bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) *status = bad ? IDS_ENONFINITE : IDS_OK;
}

ids_status check_finite(int32_t dtype, const void* Y, int64_t l, int64_t n, int64_t ldy, int32_t* status,
                        hipStream_t st) {
    if (dtype == IDS_F64)
        hipLaunchKernelGGL(finite_check_kernel<double>, dim3(1), dim3(FC_THREADS), 0, st, (const double*)Y, l, n,
                           ldy, status);
    else
        hipLaunchKernelGGL(finite_check_kernel<float>, dim3(1), dim3(FC_THREADS), 0, st, (const float*)Y, l, n,
                           ldy, status);
    return check_launch("finiteness check");
}

// Every 16-byte chunk of the buffer read once with non-temporal loads (as the
// dense CountSketch reads A): the buffer is cut into 32 KB blocks (8 rounds of
// 256 threads x 16 bytes), workgroup g takes blocks g, g + grid, ..., and a
// thread issues its 8 loads of a block before using any, so each wave streams
// 8 contiguous 4 KB runs at a time.  The XOR of all words goes to *sum so the
// loads are not dead.
constexpr int SR_THREADS = 256;
constexpr int SR_UNROLL = 8;
__global__ __launch_bounds__(SR_THREADS) void stream_read_kernel(const uint4* __restrict__ p, int64_t n16,
                                                                 uint32_t* sum) {
    typedef unsigned int u4v __attribute__((ext_vector_type(4)));
    constexpr int64_t BLK = (int64_t)SR_UNROLL * SR_THREADS;
    uint32_t x = 0;
    const int64_t full = n16 / BLK;
    for (int64_t q = blockIdx.x; q < full; q += gridDim.x) {
        const uint4* b = p + q * BLK + threadIdx.x;
        u4v v[SR_UNROLL];
#pragma unroll
        for (int u = 0; u < SR_UNROLL; ++u) v[u] = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(b + u * SR_THREADS));
#pragma unroll
        for (int u = 0; u < SR_UNROLL; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    if (blockIdx.x == 0)
        for (int64_t i = full * BLK + threadIdx.x; i < n16; i += SR_THREADS) {
            const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p + i));
            x ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    for (int o = 32; o > 0; o >>= 1) x ^= (uint32_t)__shfl_xor((int)x, o, 64);
    if ((threadIdx.x & 63) == 0) atomicXor(sum, x);
}

__global__ void zero_u32_kernel(uint32_t* p) { *p = 0u; }

ids_status stream_read(const void* p, size_t bytes, uint32_t* sum, hipStream_t st) {
    const int64_t n16 = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, sum);
    // 2 workgroups per CU: a sweep of 512..8192 workgroups (256 CUs) measured
    // 6.9, 6.5, 6.1, 5.2 and 3.6 TB/s -- fewer concurrent streams keep more
    // DRAM pages open
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
        ncu = 256;
    const int64_t blocks = n16 / ((int64_t)SR_UNROLL * SR_THREADS);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(2 * (int64_t)ncu, blocks));
    hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(SR_THREADS), 0, st, (const uint4*)p, n16, sum);
    return check_launch("stream read");
}

}  // namespace ids

// Finiteness scan of a finished sketch (IDS_CHECK_FINITE): one workgroup
// reads the l x n column-major Y once and writes IDS_OK or IDS_ENONFINITE to
// a device status word.
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

}  // namespace ids

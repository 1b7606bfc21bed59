// Interpolation matrix P = [I, R11^{-1} R12] Pi^T for large k (R11 far larger
// than LDS) by right-looking block back-substitution over 16-row blocks on
// the FP64 matrix cores, in place in P (row t of P = step t):
//   init      P[:, j] = R[0:k, j] for the non-pivot columns, e_pos for the
//             pivot columns (rows >= k_eff zero);
//   for i = nb - 1 .. 0:
//     diag(i)    T_i = R_ii^{-1} B_i for every 16-column tile (each workgroup
//                inverts the 16 x 16 diagonal block in LDS by back-substitution,
//                one thread per column, then v_mfma_f64_16x16x4f64);
//     update(i)  B_l -= R_li T_i for every row block l < i and column tile.
// R11 entries come from R11c (row t = the top rows of the column chosen at
// step t, so R[r][c] = R11c[c k + r]); past k_eff, R11 is the identity and
// the right-hand sides are zero.  Pivot columns are never written after init.
// In both products the FP64 MFMA result layout (register r: row 4 r + lane / 16,
// column lane % 16) is the B operand layout of K slice r.
#include "common.hpp"
#include "kernels.hpp"

namespace ids {

typedef double v4f64 __attribute__((ext_vector_type(4)));
constexpr int SB_WAVES = 4;  // column tiles per workgroup

__global__ __launch_bounds__(256) void sblk_init_kernel(int64_t n, int64_t k, const double* __restrict__ Rt,
                                                        const int32_t* __restrict__ pos,
                                                        const int64_t* __restrict__ keffp, double* P) {
    const int64_t keff = *keffp;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * k) return;
    const int64_t r = e / n, j = e - r * n;
    const int32_t pj = pos[j];
    P[e] = pj >= 0 ? (r == pj ? 1.0 : 0.0) : (r < keff ? Rt[j * k + r] : 0.0);
}

// R[r][c] of the padded R11 (identity past k_eff)
__device__ __forceinline__ double r11(const double* R11c, int64_t k, int64_t keff, int r, int c) {
    if (r >= keff || c >= keff) return r == c ? 1.0 : 0.0;
    return r <= c ? R11c[(int64_t)c * k + r] : 0.0;
}

__global__ __launch_bounds__(64 * SB_WAVES) void sblk_diag_kernel(int64_t n, int64_t k, int i,
                                                                  const double* __restrict__ R11c,
                                                                  const int32_t* __restrict__ pos,
                                                                  const int64_t* __restrict__ keffp, double* P) {
    __shared__ double D[16 * 16];   // R_ii, column-major (element (m, kk) at kk * 16 + m)
    __shared__ double Dinv[16 * 16];
    const int64_t keff = *keffp;
    if (16 * i >= keff) return;  // rows past k_eff stay zero
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    {
        const int m = tid & 15, kk = tid >> 4;
        D[kk * 16 + m] = r11(R11c, k, keff, 16 * i + m, 16 * i + kk);
    }
    __syncthreads();
    if (tid < 16) {  // column tid of the inverse: R_ii x = e_tid
        double x[16];
#pragma unroll
        for (int r = 15; r >= 0; --r) {
            double s = (r == tid) ? 1.0 : 0.0;
#pragma unroll
            for (int c = r + 1; c < 16; ++c) s = fma(-D[c * 16 + r], x[c], s);
            x[r] = s / D[r * 16 + r];
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) Dinv[tid * 16 + r] = x[r];
    }
    __syncthreads();
    const int64_t c0 = ((int64_t)blockIdx.x * SB_WAVES + w) * 16;
    if (c0 >= n) return;
    const int64_t j = c0 + (lane & 15);
    const bool live = j < n && pos[j] < 0;
    const int rq = lane >> 4;
    v4f64 b;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = 16 * i + 4 * r + rq;  // rows past k (the last block's padding) read as 0
        b[r] = (j < n && row < k) ? P[row * n + j] : 0.0;
    }
    v4f64 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) x = __builtin_amdgcn_mfma_f64_16x16x4f64(Dinv[64 * q + lane], b[q], x, 0, 0, 0);
    if (live) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = 16 * i + 4 * r + rq;
            if (row < k) P[row * n + j] = row < keff ? x[r] : 0.0;
        }
    }
}

// grid: x = column tiles / SB_WAVES, y = row block l < i
__global__ __launch_bounds__(64 * SB_WAVES) void sblk_update_kernel(int64_t n, int64_t k, int i,
                                                                    const double* __restrict__ R11c,
                                                                    const int32_t* __restrict__ pos,
                                                                    const int64_t* __restrict__ keffp, double* P) {
    const int64_t keff = *keffp;
    if (16 * i >= keff) return;
    const int l = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t c0 = ((int64_t)blockIdx.x * SB_WAVES + w) * 16;
    if (c0 >= n) return;
    const int64_t j = c0 + (lane & 15);
    const bool live = j < n && pos[j] < 0;
    const int rq = lane >> 4;
    v4f64 t, b;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t ri = 16 * i + 4 * r + rq, rl = 16 * l + 4 * r + rq;  // rl < 16 i <= k
        t[r] = (j < n && ri < k) ? P[ri * n + j] : 0.0;
        b[r] = (j < n) ? P[rl * n + j] : 0.0;
    }
    // A operand of K slice q: -R[16 l + lane % 16][16 i + 4 q + lane / 16]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double a = -r11(R11c, k, keff, 16 * l + (lane & 15), 16 * i + 4 * q + rq);
        b = __builtin_amdgcn_mfma_f64_16x16x4f64(a, t[q], b, 0, 0, 0);
    }
    if (live) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t row = 16 * l + 4 * r + rq;
            if (row < keff) P[row * n + j] = b[r];
        }
    }
}

ids_status solve_blocked(int64_t n, int64_t k, const double* Rt, const double* R11c, const int32_t* pos,
                         const int64_t* keff, double* P, hipStream_t st) {
    const int64_t nk = n * k;
    hipLaunchKernelGGL(sblk_init_kernel, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, st, n, k, Rt, pos, keff, P);
    const int nb = (int)((k + 15) / 16);
    const unsigned gx = (unsigned)(((n + 15) / 16 + SB_WAVES - 1) / SB_WAVES);
    for (int i = nb - 1; i >= 0; --i) {
        hipLaunchKernelGGL(sblk_diag_kernel, dim3(gx), dim3(64 * SB_WAVES), 0, st, n, k, i, R11c, pos, keff, P);
        if (i > 0)
            hipLaunchKernelGGL(sblk_update_kernel, dim3(gx, (unsigned)i), dim3(64 * SB_WAVES), 0, st, n, k, i, R11c,
                               pos, keff, P);
    }
    return check_launch("interpolation matrix (blocked)");
}

}  // namespace ids

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
#include <algorithm>

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

// k <= 128: the whole solve in one kernel.  Every workgroup stages the
// blocks R_il (l >= i) of the padded R11 in LDS -- column-major 16 x 16, the
// off-diagonal ones negated -- and replaces each diagonal block by its
// inverse (back-substitution, one thread per column); its waves then take
// tiles of 16 consecutive columns of P:
//   T_i = R_ii^{-1} (B_i - sum_{l > i} R_il T_l),  i = nb - 1 .. 0,
// with the tile's nb blocks in registers, every product on
// v_mfma_f64_16x16x4f64; a pivot column's lane writes e_pos instead, so each
// store writes a whole 128-byte row segment of P.
constexpr int SM_NBMAX = 8;  // 16-row blocks (k <= 128)
__device__ __forceinline__ int sm_tri(int i, int l) { return l * (l + 1) / 2 + i; }  // block (i <= l)

__global__ __launch_bounds__(256, 2) void smfma_solve_kernel(int n, int k, const double* __restrict__ Rt,
                                                             const double* __restrict__ R11c,
                                                             const int32_t* __restrict__ pos,
                                                             const int64_t* __restrict__ keffp, double* P) {
    extern __shared__ __attribute__((aligned(16))) double blk[];  // nb (nb + 1) / 2 blocks of 256
    const int keff = (int)max((int64_t)0, min(*keffp, (int64_t)k));  // a timed-out factorisation reports -1
    const int nb = (keff + 15) / 16;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nblk = nb * (nb + 1) / 2;
    {
        // thread tid holds element (tid & 15, tid >> 4) of every block; the
        // loads of 8 blocks are issued before any is stored
        const int m = tid & 15, kk = tid >> 4;
        for (int b0 = 0; b0 < nblk; b0 += 8) {
            double v[8];
            int il[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = min(b0 + u, nblk - 1);
                int l = 0;
                while ((l + 1) * (l + 2) / 2 <= b) ++l;
                const int i = b - l * (l + 1) / 2;
                il[u] = (i == l);
                v[u] = r11(R11c, k, keff, 16 * i + m, 16 * l + kk);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (b0 + u < nblk) blk[256 * (b0 + u) + kk * 16 + m] = il[u] ? v[u] : -v[u];
        }
    }
    __syncthreads();
    {
        // diagonal blocks -> inverses: thread (di, dc) solves R_ii x = e_dc
        const int di = tid >> 4, dc = tid & 15;
        double x[16];
        if (di < nb) {
            const double* D = blk + 256 * sm_tri(di, di);
#pragma unroll
            for (int r = 15; r >= 0; --r) {
                double s = (r == dc) ? 1.0 : 0.0;
#pragma unroll
                for (int c = r + 1; c < 16; ++c) s = fma(-D[c * 16 + r], x[c], s);
                x[r] = s / D[r * 16 + r];
            }
        }
        __syncthreads();
        if (di < nb) {
            double* Dw = blk + 256 * sm_tri(di, di);
#pragma unroll
            for (int r = 0; r < 16; ++r) Dw[dc * 16 + r] = x[r];
        }
    }
    __syncthreads();
    const int col = lane & 15, rq = lane >> 4;
    for (int t0 = ((int)blockIdx.x * 4 + w) * 16; t0 < n; t0 += (int)gridDim.x * 64) {
        const int jj = t0 + col;
        const int j = min(jj, n - 1);
        const int pj = pos[j];
        v4f64 acc[SM_NBMAX];
        // right-hand sides R[0:keff, j] (clamped loads, all in flight, then
        // masked); pivot columns load nothing
#pragma unroll
        for (int i = 0; i < SM_NBMAX; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[i][r] = (pj < 0) ? Rt[(int64_t)j * k + min(16 * i + 4 * r + rq, max(keff - 1, 0))] : 0.0;
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < SM_NBMAX; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][r] = (16 * i + 4 * r + rq < keff) ? acc[i][r] : 0.0;
#pragma unroll
        for (int i = SM_NBMAX - 1; i >= 0; --i) {
            if (i >= nb) continue;
#pragma unroll
            for (int l = i + 1; l < SM_NBMAX; ++l) {
                if (l >= nb) continue;
                const double* A = blk + 256 * sm_tri(i, l);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[64 * q + lane], acc[l][q], acc[i], 0, 0, 0);
            }
            const double* Di = blk + 256 * sm_tri(i, i);
            v4f64 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 4; ++q) x = __builtin_amdgcn_mfma_f64_16x16x4f64(Di[64 * q + lane], acc[i][q], x, 0, 0, 0);
            acc[i] = x;
        }
        if (jj < n) {
#pragma unroll
            for (int i = 0; i < SM_NBMAX; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * i + 4 * r + rq;
                    if (row < k)
                        P[(int64_t)row * n + j] = (pj >= 0) ? (row == pj ? 1.0 : 0.0) : (row < keff ? acc[i][r] : 0.0);
                }
        }
    }
}

ids_status solve_mfma_small(int64_t n, int64_t k, const double* Rt, const double* R11c, const int32_t* pos,
                            const int64_t* keff, double* P, hipStream_t st) {
    if (k > 16 * SM_NBMAX) {
        set_error("interpolation matrix: the one-kernel matrix-core solve takes k <= 128");
        return IDS_EINVAL;
    }
    const int nb = (int)((k + 15) / 16);
    const size_t lds = sizeof(double) * 256 * (size_t)(nb * (nb + 1) / 2);
    const int64_t tiles = (n + 15) / 16;
    const unsigned gx = (unsigned)std::min<int64_t>(1024, (tiles + 3) / 4);
    if (n >= INT32_MAX) {
        set_error("interpolation matrix: n must be < 2^31");
        return IDS_EINVAL;
    }
    hipLaunchKernelGGL(smfma_solve_kernel, dim3(gx), dim3(256), lds, st, (int)n, (int)k, Rt, R11c, pos, keff, P);
    return check_launch("interpolation matrix (matrix cores, k <= 128)");
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

// Second sketch stage Y = G Y1 (Gaussian projection of the CountSketch,
// Section 1.2.1) on the matrix cores: v_mfma_f64_16x16x4f64 (FP64) and
// v_mfma_f32_16x16x4f32 (FP32).  64x64 output tile per 256-thread workgroup,
// each wave a 32x32 quadrant of 2x2 16x16 MFMA blocks; K staged through LDS in
// slices of 64 (FP32) or 32 (FP64), the next slice prefetched into registers.  The output is written column-major (column j of Y
// contiguous), the layout the column-pivoted QR reads.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace ids {

typedef double v4f64 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    using Acc = v4f64;
    // result r of a lane is row 4 * r + lane / 16
    __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
    __device__ static Acc run(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<float> {
    using Acc = v4f32;
    // result r of a lane is row 4 * (lane / 16) + r
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static Acc run(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

constexpr int PBM = 64, PBN = 64;
template <typename T>
struct Pbk {
    static constexpr int K = sizeof(T) == 4 ? 64 : 32;  // K slice staged per barrier
};

// MFMA 16x16x4 operand layout (lane = 0..63):
//   A operand: A[lane % 16][lane / 16]      (16 x 4)
//   B operand: B[lane / 16][lane % 16]      (4 x 16)
//   result r : C[Mfma<T>::row(lane, r)][lane % 16]; the FP32 and FP64
//              instructions order the four result rows of a lane differently.
// The next K slice is loaded into registers while the current one is
// multiplied from LDS, so one barrier pair covers PBK = 64 (FP32) or 32 (FP64)
// columns of G.
// BCOL: Y1 column-major (entry (k, j) at Y1[j * ld1 + k]; the staging threads
// then walk k fastest so the loads stay coalesced), else row-major
// (Y1[k * ld1 + j]).
// Split K: workgroup (x, y, z) takes K range [z kchunk, min(q, (z+1) kchunk))
// and writes its partial product to Y + z * zstride (zstride = 0, kchunk = q:
// one pass straight into Y).
template <typename T, bool BCOL>
__global__ __launch_bounds__(256) void project_kernel(int64_t l, int64_t q, int64_t n, const T* __restrict__ G,
                                                      const T* __restrict__ Y1, int64_t ld1, T* __restrict__ Y,
                                                      int64_t ldy, int64_t kchunk, int64_t zstride) {
    constexpr int PBK = Pbk<T>::K;
    constexpr int NGA = PBM * PBK / 256, NBA = PBK * PBN / 256;  // staged elements per thread
    __shared__ T Gs[PBM][PBK + 1];
    __shared__ T Bs[PBK][PBN + 1];
    using M = Mfma<T>;
    using Acc = typename M::Acc;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const int64_t row0 = (int64_t)blockIdx.y * PBM;
    const int64_t col0 = (int64_t)blockIdx.x * PBN;
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = min(q, kb + kchunk);
    Y += (int64_t)blockIdx.z * zstride;
    Acc acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = Acc{0, 0, 0, 0};

    T gv[NGA], bv[NBA];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int e = 0; e < NGA; ++e) {
            const int idx = tid + e * 256;
            const int r = idx / PBK, c = idx % PBK;
            const int64_t gr = row0 + r, gc = k0 + c;
            gv[e] = (gr < l && gc < ke) ? G[gr * q + gc] : (T)0;
        }
#pragma unroll
        for (int e = 0; e < NBA; ++e) {
            const int idx = tid + e * 256;
            const int r = BCOL ? idx % PBK : idx / PBN, c = BCOL ? idx / PBK : idx % PBN;
            const int64_t gr = k0 + r, gc = col0 + c;
            bv[e] = (gr < ke && gc < n) ? (BCOL ? Y1[gc * ld1 + gr] : Y1[gr * ld1 + gc]) : (T)0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int e = 0; e < NGA; ++e) {
            const int idx = tid + e * 256;
            Gs[idx / PBK][idx % PBK] = gv[e];
        }
#pragma unroll
        for (int e = 0; e < NBA; ++e) {
            const int idx = tid + e * 256;
            if (BCOL)
                Bs[idx % PBK][idx / PBK] = bv[e];
            else
                Bs[idx / PBN][idx % PBN] = bv[e];
        }
    };
    load(kb);
    store();
    __syncthreads();
    for (int64_t k0 = kb; k0 < ke; k0 += PBK) {
        const bool more = k0 + PBK < ke;
        if (more) load(k0 + PBK);
#pragma unroll
        for (int kk = 0; kk < PBK; kk += 4) {
            T av[2], bw[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = Gs[wm * 32 + a * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bw[b] = Bs[kk + (lane >> 4)][wn * 32 + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = M::run(av[a], bw[b], acc[a][b]);
        }
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t gr = row0 + wm * 32 + a * 16 + M::row(lane, r);
                int64_t gc = col0 + wn * 32 + b * 16 + (lane & 15);
                if (gr < l && gc < n) Y[gc * ldy + gr] = acc[a][b][r];
            }
}

// partials[z] (l x n, column-major, leading dimension l) summed in z order
template <typename T>
__global__ void project_reduce_kernel(int64_t l, int64_t n, int32_t S, const T* __restrict__ part,
                                      T* __restrict__ Y, int64_t ldy) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= l * n) return;
    const int64_t c = e / l, r = e - c * l;
    T s = part[e];
    for (int z = 1; z < S; ++z) s += part[(int64_t)z * l * n + e];
    Y[c * ldy + r] = s;
}

ids_status project(int32_t dtype, int64_t l, int64_t q, int64_t n, const void* G, const void* Y1, int64_t ld1,
                   void* Y, int64_t ldy, hipStream_t st, bool y1_colmajor) {
    dim3 grid((unsigned)((n + PBN - 1) / PBN), (unsigned)((l + PBM - 1) / PBM));
    if (dtype == IDS_F64) {
        if (y1_colmajor)
            hipLaunchKernelGGL((project_kernel<double, true>), grid, dim3(256), 0, st, l, q, n, (const double*)G,
                               (const double*)Y1, ld1, (double*)Y, ldy, q, (int64_t)0);
        else
            hipLaunchKernelGGL((project_kernel<double, false>), grid, dim3(256), 0, st, l, q, n, (const double*)G,
                               (const double*)Y1, ld1, (double*)Y, ldy, q, (int64_t)0);
    } else if (dtype == IDS_F32 && !y1_colmajor) {
        hipLaunchKernelGGL((project_kernel<float, false>), grid, dim3(256), 0, st, l, q, n, (const float*)G,
                           (const float*)Y1, ld1, (float*)Y, ldy, q, (int64_t)0);
    } else {
        set_error("projection supports IDS_F64 and IDS_F32 (row-major sketch)");
        return IDS_EDTYPE;
    }
    return check_launch("projection");
}

int project_splits(int64_t l, int64_t q, int64_t n, int64_t target_wgs) {
    const int64_t tiles = ((n + PBN - 1) / PBN) * ((l + PBM - 1) / PBM);
    int64_t S = (target_wgs + tiles - 1) / tiles;
    S = std::min<int64_t>(S, std::max<int64_t>(1, q / (4 * Pbk<double>::K)));  // >= 4 K slices each
    return (int)std::max<int64_t>(1, std::min<int64_t>(S, 256));
}

template <typename T>
static ids_status split_run(int64_t l, int64_t q, int64_t n, const T* G, const T* Y1, int64_t ld1, bool y1_colmajor,
                            T* Y, int64_t ldy, int S, T* part, hipStream_t st) {
    constexpr int K = Pbk<T>::K;
    const int64_t kchunk = ((q + S - 1) / S + K - 1) / K * K;
    const int Sz = (int)((q + kchunk - 1) / kchunk);
    dim3 grid((unsigned)((n + PBN - 1) / PBN), (unsigned)((l + PBM - 1) / PBM), (unsigned)Sz);
    if (y1_colmajor)
        hipLaunchKernelGGL((project_kernel<T, true>), grid, dim3(256), 0, st, l, q, n, G, Y1, ld1, part, l, kchunk,
                           l * n);
    else
        hipLaunchKernelGGL((project_kernel<T, false>), grid, dim3(256), 0, st, l, q, n, G, Y1, ld1, part, l, kchunk,
                           l * n);
    hipLaunchKernelGGL(project_reduce_kernel<T>, dim3((unsigned)((l * n + 255) / 256)), dim3(256), 0, st, l, n, Sz,
                       part, Y, ldy);
    return check_launch("projection (split K)");
}

ids_status project_split(int32_t dtype, int64_t l, int64_t q, int64_t n, const void* G, const void* Y1, int64_t ld1,
                         bool y1_colmajor, void* Y, int64_t ldy, int S, void* part, hipStream_t st) {
    if (S <= 1) return project(dtype, l, q, n, G, Y1, ld1, Y, ldy, st, y1_colmajor);
    if (dtype == IDS_F64)
        return split_run<double>(l, q, n, (const double*)G, (const double*)Y1, ld1, y1_colmajor, (double*)Y, ldy, S,
                                 (double*)part, st);
    if (dtype == IDS_F32 && !y1_colmajor)
        return split_run<float>(l, q, n, (const float*)G, (const float*)Y1, ld1, false, (float*)Y, ldy, S,
                                (float*)part, st);
    set_error("projection supports IDS_F64 and IDS_F32 (row-major sketch)");
    return IDS_EDTYPE;
}

}  // namespace ids

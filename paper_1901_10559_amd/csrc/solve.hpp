// Column-oriented (axpy) back-substitution shared by the single-problem and
// batched interpolation-matrix kernels (Algorithm 1, last step: R11 x = b per
// column, x = R11^{-1} R12[:, j]).
//
// GQ lanes per column; lane q holds b_c, c = GQ s + q (s < TRSM_AX_KS), which
// becomes x_c once solved.  Step r: the owner lane forms x_r = b_r / R11[r][r]
// (reciprocal staged in LDS), x_r reaches the GQ lanes of the column by a DPP
// quad permutation, and every row c < r takes b_c -= R11[c][r] x_r with
// independent FMAs; the serial chain per step is one multiply, one lane
// exchange and one FMA.  R11 is staged transposed: row r holds column r of
// R11, as GQ lane segments of TRSM_AX_SQ doubles (segment q, slot s =
// R11[GQ s + q][r], zero on and below the diagonal and past the slots), so a
// lane reads its slots two at a time; the two padding slots put the GQ
// segments of a row in different LDS banks.
#pragma once
#include "common.hpp"

namespace ids {

constexpr int TRSM_AX_KS = 32;
constexpr int TRSM_AX_SQ = TRSM_AX_KS + 2;
// doubles per staged row of R11 for GQ lanes per column
template <int GQ>
constexpr int trsm_ax_ldk() { return GQ * TRSM_AX_SQ; }
// Stages the transposed R11 for axpy_solve: row r < keff of LDK doubles,
// segment q, slot sl = R11[GQ sl + q][r] where GQ sl + q < r, else 0.  Wave w
// takes rows w, w + nw, ...; a lane covers the row positions u = lane + 64 i
// (u < LDK), whose source entries it works out once, and UR rows' loads are
// issued together.  ld(r, c) reads R11[c][r]; it must be valid for r < keff
// and 0 <= c < cmax.
template <int GQ, int UR, class Ld>
__device__ __forceinline__ void stage_r11t(double* R11T, int keff, int cmax, int nthreads, Ld ld) {
    constexpr int LDK = trsm_ax_ldk<GQ>(), NI = (LDK + 63) / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = nthreads >> 6;
    int cu[NI];  // source entry of position u, -1 for a padding slot or u >= LDK
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int u = lane + 64 * i, q = u / TRSM_AX_SQ, sl = u - q * TRSM_AX_SQ;
        cu[i] = (u < LDK && sl < TRSM_AX_KS) ? GQ * sl + q : -1;
    }
    for (int r0 = w; r0 < keff; r0 += nw * UR) {
        double v[UR][NI];
#pragma unroll
        for (int ur = 0; ur < UR; ++ur) {
            const int r = min(r0 + ur * nw, keff - 1);
#pragma unroll
            for (int i = 0; i < NI; ++i) v[ur][i] = ld(r, min(max(cu[i], 0), cmax - 1));
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int ur = 0; ur < UR; ++ur) {
            const int r = r0 + ur * nw;
            if (r >= keff) break;
#pragma unroll
            for (int i = 0; i < NI; ++i) {
                const int u = lane + 64 * i;
                if (u < LDK) R11T[r * LDK + u] = (cu[i] >= 0 && cu[i] < r) ? v[ur][i] : 0.0;
            }
        }
    }
}

template <int GQ>
__device__ __forceinline__ double quad_bcast(double v, int qo) {
    if (GQ == 1) return v;
    if (GQ == 2) return (qo == 0) ? dpp_f64<0xA0, 0xf>(v) : dpp_f64<0xF5, 0xf>(v);  // [0,0,2,2] / [1,1,3,3]
    switch (qo) {                                                                  // [qo,qo,qo,qo]
        case 0: return dpp_f64<0x00, 0xf>(v);
        case 1: return dpp_f64<0x55, 0xf>(v);
        case 2: return dpp_f64<0xAA, 0xf>(v);
        default: return dpp_f64<0xFF, 0xf>(v);
    }
}

// b (this lane's rows of the right-hand side) -> x in place.  R11T: keff rows
// of trsm_ax_ldk<GQ>() doubles (16-byte aligned); rd: keff reciprocal
// diagonals.  The GQ lanes of a column must be active together.
template <int GQ>
__device__ __forceinline__ void axpy_solve(double (&b)[TRSM_AX_KS], const double* R11T, const double* rd, int keff,
                                           int q) {
    constexpr int KS = TRSM_AX_KS, SQ = TRSM_AX_SQ, LDK = trsm_ax_ldk<GQ>();
    // slot so and owner qo are compile-time indices: both loops are unrolled
#pragma unroll
    for (int so = KS - 1; so >= 0; --so) {
        if (GQ * so >= keff) continue;
#pragma unroll
        for (int qo = GQ - 1; qo >= 0; --qo) {
            const int r = GQ * so + qo;
            if (r >= keff) continue;
            const double xr = quad_bcast<GQ>(b[so] * rd[r], qo);
            const double* row = R11T + r * LDK + q * SQ;
#pragma unroll
            for (int sl = 0; sl + 1 < so; sl += 2) {
                const double2 v = *reinterpret_cast<const double2*>(row + sl);
                b[sl] = fma(-v.x, xr, b[sl]);
                b[sl + 1] = fma(-v.y, xr, b[sl + 1]);
            }
            if (so & 1) b[so - 1] = fma(-row[so - 1], xr, b[so - 1]);
            b[so] = (q == qo) ? xr : fma(-row[so], xr, b[so]);
        }
    }
}

// count elements e -> LDS through registers, U independent loads in flight per
// thread.  ld must be valid for every e < count and free of branches around
// its load (select after loading instead); slots past count load element
// count - 1 and are not stored, so no load sits behind a branch and the U
// loads are issued together.
template <int U, class Ld, class St>
__device__ __forceinline__ void copy_batched(int count, int nthreads, Ld ld, St st) {
    for (int e0 = threadIdx.x; e0 < count; e0 += U * nthreads) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ld(min(e0 + u * nthreads, count - 1));
        asm volatile("" ::: "memory");
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + u * nthreads;
            if (e < count) st(e, v[u]);
        }
    }
}

}  // namespace ids

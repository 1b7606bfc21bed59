// TensorSketch of the implicit matrix M = (Khatri-Rao of the factors) diag(lambda)
// (TensorSketch definition and the FFT formula for T A, Section 1.3;
// Algorithm 3).  Column r of T M is lambda_r times the circular convolution of
// the per-mode CountSketches c_n = S^(n) a^(n)_r, evaluated as
// IFFT( prod_n FFT(c_n) ).
//
// One 256-thread workgroup sketches two columns (r, r+1) at once:
//   * per mode: the two real CountSketches are packed as c(r) + i c(r+1) into
//     an LDS buffer, transformed by a radix-16
//     Stockham FFT in LDS, and split into the two half spectra
//     (Z[k] + conj Z[-k]) / 2 and (Z[k] - conj Z[-k]) / 2i, which are
//     multiplied into two running products (k = 0..J/2);
//   * the products are recombined as Q = P(r) + i P(r+1) (Hermitian extension)
//     and inverse transformed once: Re -> column r, Im -> column r+1.
// LDS: the padded complex work buffer (J * 17/16); the two half-spectrum
// products stay in registers (each thread owns up to 9 frequencies), so two
// workgroups share a CU.
//
// Mode CountSketch: thread t owns the contiguous bucket range
// [t J / 256, (t+1) J / 256), hence the contiguous stretch of the mode's plan
// (rows grouped by bucket, ascending row index inside a bucket).  It loads the
// stretch's row codes and factor entries TS_CB at a time (independent loads),
// recomputes each row's bucket from the hash, and adds the entries into a
// running bucket sum that it writes out when the bucket changes.  Every bucket
// is summed by one thread, from 0, in ascending row order: the result does not
// depend on scheduling.  CSC factors (sparse columns) take the per-column
// path below instead: the nonzeros only, no plan.
#include "common.hpp"
#include "kernels.hpp"

namespace ids {

__device__ __forceinline__ int padi(int i) { return i + (i >> 4); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

// cos / sin of 2 pi k / 16, k = 0..15 (correctly rounded decimal literals)
__device__ __constant__ double C16[16] = {
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
__device__ __constant__ double S16[16] = {
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674,
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977};

constexpr int bitrev(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i)
        if (x & (1 << i)) r |= 1 << (bits - 1 - i);
    return r;
}
constexpr int log2c(int R) { return R <= 1 ? 0 : 1 + log2c(R / 2); }

// in-register forward DFT of length R (power of two <= 16), natural order in/out
template <int R>
__device__ __forceinline__ void dft(double2* v) {
    constexpr int B = log2c(R);
    double2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[bitrev(i, B)] = v[i];
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const int q = k * (16 / len);
                // w = exp(-2 pi i k / len)
                const double2 w = make_double2(C16[q], -S16[q]);
                const double2 u = t[i + k];
                const double2 x = (k == 0) ? t[i + k + len / 2] : cmul(w, t[i + k + len / 2]);
                t[i + k] = cadd(u, x);
                t[i + k + len / 2] = csub(u, x);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
}

// one Stockham pass of radix R over J points held (padded) in LDS, in place.
template <int R>
__device__ __forceinline__ void stockham_pass(double2* buf, int J, int Ns, const double2* __restrict__ tw) {
    const int nj = J / R;
    const int j = threadIdx.x;
    double2 v[R];
    const bool act = j < nj;
    if (act) {
        const int k = j % Ns;
        const int tstep = k * (J / (Ns * R));  // twiddle index step: exp(-2 pi i r k / (Ns R))
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double2 x = buf[padi(j + r * nj)];
            if (r > 0 && Ns > 1) x = cmul(x, tw[r * tstep]);
            v[r] = x;
        }
        dft<R>(v);
    }
    __syncthreads();
    if (act) {
        const int k = j % Ns;
        const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[padi(idxD + r * Ns)] = v[r];
    }
    __syncthreads();
}

// forward FFT of J = 2^p points (16 <= J <= 4096) in LDS
__device__ void fft_lds(double2* buf, int J, const double2* __restrict__ tw) {
    int Ns = 1;
    while (Ns * 16 <= J) {
        stockham_pass<16>(buf, J, Ns, tw);
        Ns *= 16;
    }
    const int rem = J / Ns;
    if (rem == 8) stockham_pass<8>(buf, J, Ns, tw);
    else if (rem == 4) stockham_pass<4>(buf, J, Ns, tw);
    else if (rem == 2) stockham_pass<2>(buf, J, Ns, tw);
}

struct TsArgs {
    int32_t N;
    int64_t R;
    int32_t J;
    const double* fac[8];
    int64_t ld[8];
    const int32_t* off[8];
    const int32_t* rows[8];
    const double* lambda;
    const double2* tw;
    double* Y;  // J x R column-major
    uint64_t key[8];  // hash key of each mode's plan
    // CSC factors (colptr == nullptr: dense): column r's nonzeros are
    // rowind / val [colptr[r], colptr[r + 1]), rows ascending
    const int64_t* colptr[8];
    const int32_t* rowind[8];
    const double* val[8];
};

// Mode CountSketch of one CSC column into component `comp` (0: re, 1: im) of
// the packed LDS buffer, by one wave: the column's nonzeros in batches of 64
// (lane q holds entry p0 + q, rows ascending), each entry's bucket and sign
// from the hash.  Entries of a batch that share a bucket are ranked by lane
// (peer mask from one ballot per bucket bit, rank = peers below), and rank 0,
// 1, ... add in turn, so every bucket takes its entries in ascending row
// order -- the order of the dense path and of the textbook sum.
__device__ __forceinline__ void cs_sparse_column(double* bufd, int comp, int J, uint64_t key, const int64_t* colptr,
                                                 const int32_t* rowind, const double* val, int64_t r) {
    const int lane = threadIdx.x & 63;
    const int64_t q0 = colptr[r], q1 = colptr[r + 1];
    const int nbits = 32 - __clz(J - 1);  // J is a power of two
    for (int64_t p0 = q0; p0 < q1; p0 += 64) {
        const int64_t p = p0 + lane;
        const bool live = p < q1;
        uint32_t b = 0;
        double v = 0.0;
        if (live) {
            const int64_t i = rowind[p];
            bool ng;
            hash_row(key, i, (uint32_t)J, b, ng);
            v = ng ? -val[p] : val[p];
        }
        // lanes holding the same bucket: AND over the bucket bits
        uint64_t peers = __ballot(live);
        for (int t = 0; t < nbits; ++t) {
            const uint64_t m = __ballot(live && ((b >> t) & 1u));
            peers &= ((b >> t) & 1u) ? m : ~m;
        }
        const int rank = __popcll(peers & ((1ull << lane) - 1ull));
        int maxrank = live ? rank : 0;
        for (int o = 32; o > 0; o >>= 1) maxrank = max(maxrank, __shfl_xor(maxrank, o, 64));
        for (int k = 0; k <= maxrank; ++k) {
            if (live && rank == k) {
                double* d = bufd + 2 * padi((int)b) + comp;
                *d = *d + v;
            }
            // the wave's LDS operations complete in program order, so the next
            // round reads what this one wrote
            __builtin_amdgcn_wave_barrier();
        }
    }
}

constexpr int TS_CB = 8;  // plan positions loaded together

// frequencies k = tid + 256 q (q < TS_NK) of the half spectrum 0..J/2 are owned
// by thread tid, which keeps their running products in registers
constexpr int TS_NK = 9;  // ceil((4096 / 2 + 1) / 256)

__global__ __launch_bounds__(256) void tensorsketch_kernel(TsArgs a) {
    extern __shared__ double2 smem[];
    const int J = a.J;
    double2* buf = smem;  // padi(J) entries
    const int64_t r0 = (int64_t)blockIdx.x * 2;
    const bool two = r0 + 1 < a.R;
    const int tid = threadIdx.x;
    double2 P1[TS_NK], P2[TS_NK];

    for (int md = 0; md < a.N; ++md) {
        const double* f0 = a.fac[md] + r0 * a.ld[md];
        const double* f1 = two ? f0 + a.ld[md] : f0;
        const int32_t* off = a.off[md];
        const int32_t* rows = a.rows[md];
        // mode-n CountSketch of columns r0, r0+1 packed as re + i im
        if (a.colptr[md]) {
            // CSC factor: zero the buffer, then waves 0 and 1 add the nonzeros
            // of columns r0 and r0 + 1 into the real and imaginary parts
            for (int b = tid; b < J; b += 256) buf[padi(b)] = make_double2(0.0, 0.0);
            __syncthreads();
            const int w = tid >> 6;
            if (w == 0 || (w == 1 && two))
                cs_sparse_column((double*)buf, w, J, a.key[md], a.colptr[md], a.rowind[md], a.val[md], r0 + w);
        } else {
            const int bA = (int)(((int64_t)tid * J) >> 8), bB = (int)(((int64_t)(tid + 1) * J) >> 8);
            const int pA = off[bA], pB = off[bB];
            const uint64_t key = a.key[md];
            double s0 = 0.0, s1 = 0.0;
            int bcur = bA;
            for (int pb = pA; pb < pB; pb += TS_CB) {
                int32_t code[TS_CB];
#pragma unroll
                for (int u = 0; u < TS_CB; ++u) code[u] = (pb + u < pB) ? rows[pb + u] : 0;
                double x0[TS_CB], x1[TS_CB];
#pragma unroll
                for (int u = 0; u < TS_CB; ++u) {
                    const int64_t i = code[u] >= 0 ? code[u] : -(int64_t)code[u] - 1;
                    x0[u] = (pb + u < pB) ? f0[i] : 0.0;
                    x1[u] = (pb + u < pB) ? f1[i] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < TS_CB; ++u) {
                    if (pb + u < pB) {
                        const int64_t i = code[u] >= 0 ? code[u] : -(int64_t)code[u] - 1;
                        uint32_t bk;
                        bool ng;
                        hash_row(key, i, (uint32_t)J, bk, ng);
                        while (bcur < (int)bk) {
                            buf[padi(bcur)] = make_double2(s0, two ? s1 : 0.0);
                            s0 = s1 = 0.0;
                            ++bcur;
                        }
                        if (code[u] < 0) {
                            s0 -= x0[u];
                            s1 -= x1[u];
                        } else {
                            s0 += x0[u];
                            s1 += x1[u];
                        }
                    }
                }
            }
            for (; bcur < bB; ++bcur) {
                buf[padi(bcur)] = make_double2(s0, two ? s1 : 0.0);
                s0 = s1 = 0.0;
            }
        }
        __syncthreads();
        fft_lds(buf, J, a.tw);
        // split the packed spectrum, multiply into the products
#pragma unroll
        for (int q = 0; q < TS_NK; ++q) {
            const int k = tid + 256 * q;
            if (k > J / 2) continue;
            const double2 z = buf[padi(k)];
            const double2 zc = conj2(buf[padi((J - k) & (J - 1))]);
            const double2 A = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y + zc.y));
            // (z - zc) / (2i) = -i (z - zc) / 2
            const double2 d = csub(z, zc);
            const double2 B = make_double2(0.5 * d.y, -0.5 * d.x);
            if (md == 0) {
                P1[q] = A;
                P2[q] = B;
            } else {
                P1[q] = cmul(P1[q], A);
                P2[q] = cmul(P2[q], B);
            }
        }
        __syncthreads();
    }
    // Q = P1 + i P2 over the full circle (Hermitian extension); inverse FFT via
    // conj(FFT(conj(Q))) / J
#pragma unroll
    for (int q = 0; q < TS_NK; ++q) {
        const int k = tid + 256 * q;
        if (k > J / 2) continue;
        const double2 p1 = P1[q], p2 = P2[q];
        buf[padi(k)] = conj2(make_double2(p1.x - p2.y, p1.y + p2.x));
        if (k > 0 && k < J / 2) {
            const double2 c1 = conj2(p1), c2 = conj2(p2);
            buf[padi(J - k)] = conj2(make_double2(c1.x - c2.y, c1.y + c2.x));
        }
    }
    __syncthreads();
    fft_lds(buf, J, a.tw);
    const double inv = 1.0 / (double)J;
    const double l0 = a.lambda[r0] * inv;
    const double l1 = two ? a.lambda[r0 + 1] * inv : 0.0;
    for (int b = tid; b < J; b += 256) {
        const double2 w = buf[padi(b)];
        a.Y[r0 * J + b] = w.x * l0;
        if (two) a.Y[(r0 + 1) * J + b] = -w.y * l1;
    }
}

__global__ void twiddle_kernel(int J, double2* tw) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= J) return;
    double s, c;
    sincospi(2.0 * (double)q / (double)J, &s, &c);
    tw[q] = make_double2(c, -s);  // exp(-2 pi i q / J)
}

ids_status twiddles(int64_t Jlen, double2* tw, hipStream_t st) {
    hipLaunchKernelGGL(twiddle_kernel, dim3((unsigned)((Jlen + 255) / 256)), dim3(256), 0, st, (int)Jlen, tw);
    return check_launch("twiddles");
}

size_t ts_lds_bytes(int64_t J) { return sizeof(double2) * (size_t)(J + J / 16); }

ids_status tensorsketch(int32_t N, const int64_t* dims, int64_t R, const double* const* factors, const int64_t* ld,
                        const double* lambda, int64_t Jlen, const PlanBufs* plans, const uint64_t* keys,
                        const double2* tw, double* Y, hipStream_t st, const int64_t* const* colptr,
                        const int32_t* const* rowind, const double* const* val) {
    (void)dims;
    TsArgs a;
    a.N = N;
    a.R = R;
    a.J = (int32_t)Jlen;
    for (int n = 0; n < N; ++n) {
        const bool csc = colptr != nullptr;
        a.fac[n] = csc ? nullptr : factors[n];
        a.ld[n] = csc ? 0 : ld[n];
        a.off[n] = csc ? nullptr : plans[n].off;
        a.rows[n] = csc ? nullptr : plans[n].rows;
        a.key[n] = keys[n];
        a.colptr[n] = csc ? colptr[n] : nullptr;
        a.rowind[n] = csc ? rowind[n] : nullptr;
        a.val[n] = csc ? val[n] : nullptr;
    }
    a.lambda = lambda;
    a.tw = tw;
    a.Y = Y;
    const size_t lds = ts_lds_bytes(Jlen);
    hipLaunchKernelGGL(tensorsketch_kernel, dim3((unsigned)((R + 1) / 2)), dim3(256), lds, st, a);
    return check_launch("tensorsketch");
}

}  // namespace ids

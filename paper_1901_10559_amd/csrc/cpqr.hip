// Algorithm 1 on a sketch Y (l x n): rank-k column-pivoted QR, then
// P = [I, R11^{-1} R12] Pi^T in the original column order.
//
// cpqr_kernel is a persistent cooperative kernel.  Each wave owns CPW columns
// of Y held in registers for the whole factorisation (row i of a column lives
// in lane i % 64, register slot i / 64).  One step t:
//   1. every wave recomputes the trailing squared norms sum_{i>=t} y_ij^2 of its
//      live columns in FP64 (no downdating, so no cancellation guard needed);
//   2. the workgroup's best (largest norm, ties to the smallest column index)
//      is published with a copy of that column to a per-workgroup slot;
//   3. one device-wide barrier;
//   4. every workgroup reads all candidates, picks the same winner, copies the
//      winner's column to LDS and forms the Householder reflector
//      (v_t = 1, beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta);
//   5. the reflector is applied to every live column; row t of a column then
//      holds R[t][j].
// After k steps each column's top k rows are R[0:k, j] (original order).
// trsm_p_kernel then solves R11 x = R[0:k, j] per column by back-substitution
// and writes P.
#include "common.hpp"
#include "kernels.hpp"

namespace ids {

struct SelArgs {
    const void* Y;
    int32_t ydt;
    int64_t l, n, rs, cs, k;
    int64_t* J;
    int64_t* keff;
    double* Rt;        // n x k (column j's top rows contiguous)
    int32_t* pos;      // n: step at which the column was chosen, -1 otherwise
    double* slot;      // 2 x nb x lpad
    double* cand_nu;   // 2 x nb
    int64_t* cand_j;   // 2 x nb
    uint32_t* bar;     // [0] barrier counter, [1] timeout flag
    int32_t nb, lpad;
};

__device__ __forceinline__ bool better(double nu1, int64_t j1, double nu2, int64_t j2) {
    return nu1 > nu2 || (nu1 == nu2 && j1 < j2);
}

__device__ __forceinline__ double load_y(const SelArgs& a, int64_t off) {
    return a.ydt == IDS_F64 ? ((const double*)a.Y)[off] : (double)((const float*)a.Y)[off];
}

constexpr uint32_t SPIN_LIMIT = 1u << 21;

// Device-wide barrier for a cooperative launch (all workgroups co-resident).
// The spin has a cap so every wave always exits; on timeout a flag is raised.
__device__ void grid_sync(uint32_t* bar, uint32_t target) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <int RPL, int CPW, int NW>
__global__ __launch_bounds__(NW * 64) void cpqr_kernel(SelArgs a) {
    extern __shared__ double xb[];  // winner column, lpad doubles
    __shared__ double s_nu[NW];
    __shared__ int64_t s_j[NW];
    __shared__ int s_c[NW];
    __shared__ double s_wnu;
    __shared__ int64_t s_wj;

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t colbase = ((int64_t)blockIdx.x * NW + w) * CPW;
    const int64_t l = a.l, n = a.n;

    double y[CPW][RPL];
    bool alive[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int64_t j = colbase + c;
        alive[c] = j < n;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int64_t i = lane + 64 * r;
            y[c][r] = (alive[c] && i < l) ? load_y(a, i * a.rs + j * a.cs) : 0.0;
        }
        if (alive[c] && lane == 0) a.pos[j] = -1;
    }

    int64_t keff = a.k;
    for (int64_t t = 0; t < a.k; ++t) {
        const int par = (int)(t & 1);
        // ---- 1. trailing norms and the wave's best column
        double bnu = -1.0;
        int64_t bj = INT64_MAX;
        int bc = -1;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            if (!alive[c]) continue;
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t i = lane + 64 * r;
                if (i >= t) s = fma(y[c][r], y[c][r], s);
            }
            s = wave_sum(s);
            const int64_t j = colbase + c;
            if (better(s, j, bnu, bj)) {
                bnu = s;
                bj = j;
                bc = c;
            }
        }
        if (lane == 0) {
            s_nu[w] = bnu;
            s_j[w] = bj;
            s_c[w] = bc;
        }
        __syncthreads();
        // ---- 2. workgroup best -> candidate slot
        int bw = 0;
        {
            double wn = s_nu[0];
            int64_t wj = s_j[0];
            for (int q = 1; q < NW; ++q)
                if (better(s_nu[q], s_j[q], wn, wj)) {
                    wn = s_nu[q];
                    wj = s_j[q];
                    bw = q;
                }
            if (threadIdx.x == 0) {
                a.cand_nu[par * a.nb + blockIdx.x] = wn;
                a.cand_j[par * a.nb + blockIdx.x] = (wj == INT64_MAX) ? -1 : wj;
            }
        }
        if (w == bw && bc >= 0) {
            double* sl = a.slot + ((size_t)par * a.nb + blockIdx.x) * a.lpad;
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                if (c != bc) continue;
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    const int64_t i = lane + 64 * r;
                    if (i < l) sl[i] = y[c][r];
                }
            }
        }
        if (w == bw || threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        // ---- 3. device-wide barrier
        grid_sync(a.bar, (uint32_t)(a.nb * (t + 1)));
        // ---- 4. winner (identical in every workgroup)
        {
            double wn = -1.0;
            int64_t wj = INT64_MAX;
            for (int q = threadIdx.x; q < a.nb; q += NW * 64) {
                double nu = a.cand_nu[par * a.nb + q];
                int64_t j = a.cand_j[par * a.nb + q];
                if (j >= 0 && better(nu, j, wn, wj)) {
                    wn = nu;
                    wj = j;
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                double on = __shfl_xor(wn, o, 64);
                int64_t oj = __shfl_xor(wj, o, 64);
                if (better(on, oj, wn, wj)) {
                    wn = on;
                    wj = oj;
                }
            }
            if (lane == 0) {
                s_nu[w] = wn;
                s_j[w] = wj;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double bn = s_nu[0];
                int64_t bjj = s_j[0];
                for (int q = 1; q < NW; ++q)
                    if (better(s_nu[q], s_j[q], bn, bjj)) {
                        bn = s_nu[q];
                        bjj = s_j[q];
                    }
                s_wnu = bn;
                s_wj = bjj;
            }
            __syncthreads();
        }
        const double wnu = s_wnu;
        const int64_t wj = s_wj;
        if (wj == INT64_MAX || !(wnu > 0.0)) {
            keff = t;
            break;
        }
        const int wblk = (int)(wj / ((int64_t)NW * CPW));
        const double* wsl = a.slot + ((size_t)par * a.nb + wblk) * a.lpad;
        for (int64_t i = threadIdx.x; i < l; i += NW * 64) xb[i] = (i >= t) ? wsl[i] : 0.0;
        __syncthreads();
        // ---- Householder reflector (computed redundantly by every wave)
        double sig2 = 0.0;
        for (int64_t i = t + 1 + lane; i < l; i += 64) sig2 = fma(xb[i], xb[i], sig2);
        sig2 = wave_sum(sig2);
        const double alpha = xb[t];
        double tau, beta, scal;
        if (sig2 == 0.0) {
            tau = 0.0;
            beta = alpha;
            scal = 0.0;
        } else {
            const double nrm = sqrt(alpha * alpha + sig2);
            beta = (alpha >= 0.0) ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        // ---- 5. apply H = I - tau v v^T to the live columns
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            if (!alive[c]) continue;
            double d = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t i = lane + 64 * r;
                if (i >= t && i < l) {
                    const double v = (i == t) ? 1.0 : xb[i] * scal;
                    d = fma(v, y[c][r], d);
                }
            }
            d = wave_sum(d) * tau;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int64_t i = lane + 64 * r;
                if (i >= t && i < l) {
                    const double v = (i == t) ? 1.0 : xb[i] * scal;
                    y[c][r] = fma(-d, v, y[c][r]);
                }
            }
            const int64_t j = colbase + c;
            if (j == wj) {
                alive[c] = false;
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (lane + 64 * r == t) y[c][r] = beta;
                if (lane == 0) a.pos[j] = (int32_t)t;
            }
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) a.J[t] = wj;
        __syncthreads();  // xb is rewritten next step
    }

    // top keff rows of every column = R[0:keff, j]
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int64_t j = colbase + c;
        if (j >= n) continue;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int64_t i = lane + 64 * r;
            if (i < keff) a.Rt[j * a.k + i] = y[c][r];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const bool timed_out = __hip_atomic_load(a.bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        *a.keff = timed_out ? -1 : keff;
        for (int64_t t = keff; t < a.k; ++t) a.J[t] = -1;
    }
}

__global__ void zero_u32_kernel(uint32_t* p, int count) {
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0u;
}

// P[:, j]: e_t for a chosen column, R11^{-1} R[0:keff, j] otherwise.
constexpr int TRSM_THREADS = 256;
template <bool R11_LDS>
__global__ __launch_bounds__(TRSM_THREADS) void trsm_p_kernel(int64_t n, int64_t k, const double* __restrict__ Rt,
                                                              const int64_t* __restrict__ J,
                                                              const int32_t* __restrict__ pos,
                                                              const int64_t* __restrict__ keffp, double* P) {
    extern __shared__ double R11s[];
    const int64_t keff = *keffp;
    if (keff < 0) return;
    if (R11_LDS) {
        for (int64_t e = threadIdx.x; e < keff * keff; e += TRSM_THREADS) {
            const int64_t r = e / keff, c = e % keff;
            R11s[e] = (r <= c) ? Rt[J[c] * k + r] : 0.0;
        }
        __syncthreads();
    }
    const int64_t j = (int64_t)blockIdx.x * TRSM_THREADS + threadIdx.x;
    if (j >= n) return;
    const int32_t pj = pos[j];
    if (pj >= 0) {
        for (int64_t r = 0; r < k; ++r) P[r * n + j] = (r == pj) ? 1.0 : 0.0;
        return;
    }
    for (int64_t r = keff - 1; r >= 0; --r) {
        double s = Rt[j * k + r];
        for (int64_t c = r + 1; c < keff; ++c) {
            const double rc = R11_LDS ? R11s[r * keff + c] : Rt[J[c] * k + r];
            s = fma(-rc, P[c * n + j], s);
        }
        const double d = R11_LDS ? R11s[r * keff + r] : Rt[J[r] * k + r];
        P[r * n + j] = s / d;
    }
    for (int64_t r = keff; r < k; ++r) P[r * n + j] = 0.0;
}

__global__ __launch_bounds__(256) void lambda_hat_kernel(int64_t k, int64_t n, const double* __restrict__ P,
                                                         const int64_t* __restrict__ J,
                                                         const int64_t* __restrict__ keffp,
                                                         const double* __restrict__ lam, double* lhat) {
    __shared__ double red[4];
    const int64_t t = blockIdx.x;
    const int64_t keff = *keffp;
    if (t >= keff) {
        if (threadIdx.x == 0) lhat[t] = 0.0;
        return;
    }
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 256) s += P[t * n + r];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) lhat[t] = lam[J[t]] * ((red[0] + red[1]) + (red[2] + red[3]));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Inst {
    int rpl, cpw, nw;
    const void* fn;
};

template <int RPL, int CPW, int NW>
static const void* fnptr() {
    return (const void*)&cpqr_kernel<RPL, CPW, NW>;
}

static bool pick(int64_t l, Inst& in) {
    // rows per lane (power of two), columns per wave, waves per workgroup
    if (l <= 64) in = {1, 16, 8, fnptr<1, 16, 8>()};
    else if (l <= 128) in = {2, 8, 8, fnptr<2, 8, 8>()};
    else if (l <= 256) in = {4, 4, 8, fnptr<4, 4, 8>()};
    else if (l <= 512) in = {8, 2, 8, fnptr<8, 2, 8>()};
    else if (l <= 1024) in = {16, 1, 8, fnptr<16, 1, 8>()};
    else if (l <= 2048) in = {32, 1, 8, fnptr<32, 1, 8>()};
    else if (l <= 4096) in = {64, 1, 8, fnptr<64, 1, 8>()};
    else return false;
    return true;
}

ids_status select_plan(int64_t l, int64_t n, int64_t k, SelectPlan& sp) {
    Inst in;
    if (!pick(l, in)) {
        set_error("id_select: l must be <= 4096");
        return IDS_EINVAL;
    }
    sp.l = l;
    sp.n = n;
    sp.k = k;
    sp.rpl = in.rpl;
    sp.cpw = in.cpw;
    sp.nw = in.nw;
    const int64_t per = (int64_t)in.cpw * in.nw;
    sp.nb = (int)((n + per - 1) / per);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return IDS_EHIP;
    }
    int ncu = 0, per_cu = 0;
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t lds = sizeof(double) * (size_t)((l + 63) / 64 * 64);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, in.fn, in.nw * 64, lds) != hipSuccess) per_cu = 1;
    if ((int64_t)sp.nb > (int64_t)ncu * per_cu) {
        set_error("id_select: n too large for the register-resident CPQR (n = " + std::to_string(n) +
                  ", l = " + std::to_string(l) + ", max columns " + std::to_string((int64_t)ncu * per_cu * per) +
                  ")");
        return IDS_EINVAL;
    }
    return IDS_OK;
}

static size_t lpad_of(int64_t l) { return (size_t)((l + 63) / 64 * 64); }

size_t select_bytes(const SelectPlan& sp) {
    return align256(sizeof(double) * 2 * sp.nb * lpad_of(sp.l)) + align256(sizeof(double) * 2 * sp.nb) +
           align256(sizeof(int64_t) * 2 * sp.nb) + align256(sizeof(uint32_t) * 2) +
           align256(sizeof(double) * (size_t)sp.n * sp.k) + align256(sizeof(int32_t) * (size_t)sp.n);
}

ids_status select_run(const SelectPlan& sp, const void* Y, int32_t ydt, int64_t rs, int64_t cs, int64_t* J,
                      double* P, int64_t* keff, char* ws, hipStream_t st) {
    SelArgs a;
    a.Y = Y;
    a.ydt = ydt;
    a.l = sp.l;
    a.n = sp.n;
    a.rs = rs;
    a.cs = cs;
    a.k = sp.k;
    a.J = J;
    a.keff = keff;
    a.nb = sp.nb;
    a.lpad = (int32_t)lpad_of(sp.l);
    char* p = ws;
    a.slot = (double*)p;
    p += align256(sizeof(double) * 2 * sp.nb * lpad_of(sp.l));
    a.cand_nu = (double*)p;
    p += align256(sizeof(double) * 2 * sp.nb);
    a.cand_j = (int64_t*)p;
    p += align256(sizeof(int64_t) * 2 * sp.nb);
    a.bar = (uint32_t*)p;
    p += align256(sizeof(uint32_t) * 2);
    a.Rt = (double*)p;
    p += align256(sizeof(double) * (size_t)sp.n * sp.k);
    a.pos = (int32_t*)p;

    Inst in;
    pick(sp.l, in);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, st, a.bar, 2);
    void* args[] = {&a};
    const size_t lds = sizeof(double) * lpad_of(sp.l);
    {
        ProfScope ps(PK_CPQR, st);
        hipError_t e = hipLaunchCooperativeKernel(in.fn, dim3(sp.nb), dim3(in.nw * 64), args, (unsigned)lds, st);
        if (e != hipSuccess) {
            set_error(std::string("cpqr cooperative launch: ") + hipGetErrorString(e));
            return IDS_EHIP;
        }
    }
    ProfScope ps(PK_TRSM, st);
    const size_t r11 = sizeof(double) * (size_t)sp.k * sp.k;
    const unsigned g = (unsigned)((sp.n + TRSM_THREADS - 1) / TRSM_THREADS);
    if (r11 <= lds_limit())
        hipLaunchKernelGGL(trsm_p_kernel<true>, dim3(g), dim3(TRSM_THREADS), r11, st, sp.n, sp.k,
                           (const double*)a.Rt, (const int64_t*)J, (const int32_t*)a.pos, (const int64_t*)keff, P);
    else
        hipLaunchKernelGGL(trsm_p_kernel<false>, dim3(g), dim3(TRSM_THREADS), 0, st, sp.n, sp.k,
                           (const double*)a.Rt, (const int64_t*)J, (const int32_t*)a.pos, (const int64_t*)keff, P);
    return check_launch("cpqr / interpolation matrix");
}

ids_status lambda_hat(int64_t k, int64_t n, const double* P, const int64_t* J, const int64_t* keff,
                      const double* lambda, double* lhat, hipStream_t st) {
    hipLaunchKernelGGL(lambda_hat_kernel, dim3((unsigned)k), dim3(256), 0, st, k, n, P, J, keff, lambda, lhat);
    return check_launch("lambda_hat");
}

}  // namespace ids

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
    double* slot;      // 2 x nb x S: [0] = norm^2, [1] = column index bits, [2..2+l) = column
    uint32_t* bar;     // [0] barrier counter, [1] timeout flag
    int32_t nb, S;
};

__device__ __forceinline__ bool better(double nu1, int64_t j1, double nu2, int64_t j2) {
    return nu1 > nu2 || (nu1 == nu2 && j1 < j2);
}

__device__ __forceinline__ double load_y(const SelArgs& a, int64_t off) {
    return a.ydt == IDS_F64 ? ((const double*)a.Y)[off] : (double)((const float*)a.Y)[off];
}

// wave sums of CPW values at once (independent DPP chains overlap); the
// result is broadcast from one lane, so every lane holds the same bits.
template <int CPW>
__device__ __forceinline__ void wave_sum_many(double (&v)[CPW]) {
    wave_sum_dpp<CPW>(v);
}

constexpr uint32_t SPIN_LIMIT = 1u << 21;

// Cross-workgroup data (candidate slots, the barrier counter) is only ever
// accessed with agent-scope atomic loads and stores, which are coherent across
// the whole device per location without L2 write-back or invalidation.  The
// order "slot data before counter increment" is enforced by waiting for the
// wave's outstanding memory operations (s_waitcnt 0) before the increment; the
// order "counter observed before slot data read" by the control dependency on
// the polled value.
__device__ __forceinline__ void slot_store(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double slot_load(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-wide barrier for a cooperative launch (all workgroups co-resident).
// Callers that stored slot data must have executed s_waitcnt 0 first.  The
// spin is capped so every wave always exits; on timeout a flag is raised.
__device__ void grid_sync(uint32_t* bar, uint32_t target) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_s_waitcnt(0);
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > SPIN_LIMIT) {
                __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    __syncthreads();
}

// argmax over the wave of (nu, j): largest nu, then smallest j; j < 2^31.
// DPP max / min trees fold into lane 63, which is broadcast.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_keep_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_keep_i32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ void wave_argmax(double& nu, int& j) {
    double m = nu;
    m = fmax(m, dpp_keep_f64<0xB1, 0xf>(m));
    m = fmax(m, dpp_keep_f64<0x4E, 0xf>(m));
    m = fmax(m, dpp_keep_f64<0x141, 0xf>(m));
    m = fmax(m, dpp_keep_f64<0x140, 0xf>(m));
    m = fmax(m, dpp_keep_f64<0x142, 0xa>(m));
    m = fmax(m, dpp_keep_f64<0x143, 0xc>(m));
    m = lane63_f64(m);
    int q = (nu == m) ? j : INT32_MAX;
    q = min(q, dpp_keep_i32<0xB1, 0xf>(q));
    q = min(q, dpp_keep_i32<0x4E, 0xf>(q));
    q = min(q, dpp_keep_i32<0x141, 0xf>(q));
    q = min(q, dpp_keep_i32<0x140, 0xf>(q));
    q = min(q, dpp_keep_i32<0x142, 0xa>(q));
    q = min(q, dpp_keep_i32<0x143, 0xc>(q));
    nu = m;
    j = __builtin_amdgcn_readlane(q, 63);
}

// ALL = true: every workgroup copies all candidate slots to LDS with one bulk
// load (one round trip after the barrier); otherwise it reads the headers, then
// the winner's column.
template <int RPL, int CPW, int NW, bool ALL>
__global__ __launch_bounds__(NW * 64) void cpqr_kernel(SelArgs a) {
    extern __shared__ double sm[];
    __shared__ double s_nu[NW];
    __shared__ int64_t s_j[NW];
    __shared__ double s_wnu;
    __shared__ int64_t s_wj;
    constexpr int NT = NW * 64;

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int64_t colbase = ((int64_t)blockIdx.x * NW + w) * CPW;
    const int64_t l = a.l, n = a.n;
    const int S = a.S;

    double y[CPW][RPL];
    bool alive[CPW];
    // branch-free load: indices clamped into range, out-of-range entries zeroed
    if (a.ydt == IDS_F64) {
        const double* Yp = (const double*)a.Y;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int64_t jc = min(colbase + c, n - 1);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                const double v = Yp[(int64_t)min(i, (int)l - 1) * a.rs + jc * a.cs];
                y[c][r] = (colbase + c < n && i < l) ? v : 0.0;
            }
        }
    } else {
        const float* Yp = (const float*)a.Y;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int64_t jc = min(colbase + c, n - 1);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                const double v = (double)Yp[(int64_t)min(i, (int)l - 1) * a.rs + jc * a.cs];
                y[c][r] = (colbase + c < n && i < l) ? v : 0.0;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int64_t j = colbase + c;
        alive[c] = j < n;
        if (alive[c] && lane == 0) a.pos[j] = -1;
    }
    // trailing squared norms for step 0
    double nu[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RPL; ++r) s = fma(y[c][r], y[c][r], s);
        nu[c] = s;
    }
    wave_sum_many<CPW>(nu);

    int64_t keff = a.k;
    for (int64_t t = 0; t < a.k; ++t) {
        const int par = (int)(t & 1);
        double* slots = a.slot + (size_t)par * a.nb * S;
        // ---- 1. the wave's best live column (largest norm, smallest index)
        double bnu = -1.0;
        int64_t bj = INT64_MAX;
        int bc = -1;
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            const int64_t j = colbase + c;
            if (alive[c] && better(nu[c], j, bnu, bj)) {
                bnu = nu[c];
                bj = j;
                bc = c;
            }
        }
        if (lane == 0) {
            s_nu[w] = bnu;
            s_j[w] = bj;
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
                double* sl = slots + (size_t)blockIdx.x * S;
                slot_store(sl, wn);
                slot_store(sl + 1, __longlong_as_double((wj == INT64_MAX) ? -1LL : (long long)wj));
            }
        }
        if (w == bw && bc >= 0) {
            double* sl = slots + (size_t)blockIdx.x * S + 2;
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                if (c != bc) continue;
#pragma unroll
                for (int r = 0; r < RPL; ++r) {
                    const int64_t i = lane + 64 * r;
                    if (i < l) slot_store(sl + i, y[c][r]);
                }
            }
            __builtin_amdgcn_s_waitcnt(0);
        }
        // ---- 3. device-wide barrier
        grid_sync(a.bar, (uint32_t)(a.nb * (t + 1)));
        // ---- 4. winner (identical in every workgroup)
        if (ALL) {
            // all candidate slots -> LDS, 8 loads in flight per thread
            const int tot = a.nb * S;
            for (int e0 = 0; e0 < tot; e0 += NT * 8) {
                double tmp[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT + (int)threadIdx.x;
                    tmp[u] = (e < tot) ? slot_load(slots + e) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT + (int)threadIdx.x;
                    if (e < tot) sm[e] = tmp[u];
                }
            }
            __syncthreads();
        }
        {
            double wn = -1.0;
            int wjj = INT32_MAX;
            for (int q = threadIdx.x; q < a.nb; q += NT) {
                double nuq;
                int64_t jq;
                if (ALL) {
                    nuq = sm[(size_t)q * S];
                    jq = (int64_t)__double_as_longlong(sm[(size_t)q * S + 1]);
                } else {
                    nuq = slot_load(slots + (size_t)q * S);
                    jq = (int64_t)__double_as_longlong(slot_load(slots + (size_t)q * S + 1));
                }
                if (jq >= 0 && better(nuq, jq, wn, wjj)) {
                    wn = nuq;
                    wjj = (int)jq;
                }
            }
            wave_argmax(wn, wjj);
            if (lane == 0) {
                s_nu[w] = wn;
                s_j[w] = (wjj == INT32_MAX) ? INT64_MAX : (int64_t)wjj;
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
        const double* xb;
        if (ALL) {
            xb = sm + (size_t)wblk * S + 2;
        } else {
            const double* wsl = slots + (size_t)wblk * S + 2;
            for (int i0 = 0; i0 < (int)l; i0 += NT * 8) {
                double tmp[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + u * NT + (int)threadIdx.x;
                    tmp[u] = (i < l) ? slot_load(wsl + i) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + u * NT + (int)threadIdx.x;
                    if (i < l) sm[i] = tmp[u];
                }
            }
            __syncthreads();
            xb = sm;
        }
        // ---- Householder reflector of the winner's rows t..l-1 (every wave
        //      computes it redundantly from the same LDS data: same bits)
        double sig2 = 0.0;
        for (int64_t i = t + 1 + lane; i < l; i += 64) sig2 = fma(xb[i], xb[i], sig2);
        sig2 = wave_sum_dpp1(sig2);
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
        // reflector entry of row i: 0 above t, 1 at t, x_i * scal below
        const int ti = (int)t, li = (int)l;
        auto vof = [&](int i) -> double {
            return (i < ti || i >= li) ? 0.0 : (i == ti ? 1.0 : xb[i] * scal);
        };
        constexpr bool VREG = RPL <= 8;  // tall sketches re-read v from LDS
        double v[VREG ? RPL : 1];
        if (VREG) {
#pragma unroll
            for (int r = 0; r < RPL; ++r) v[VREG ? r : 0] = vof(lane + 64 * r);
        }
        // ---- 5. apply H = I - tau v v^T to the live columns, then the new
        //      trailing norms (rows > t), all columns' reductions interleaved
        // (tall sketches: v is re-read from LDS in chunks of 8 rows, with a
        //  compiler barrier per chunk so only a few entries are live at once)
        double d[CPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                s = fma(VREG ? v[VREG ? r : 0] : vof(lane + 64 * r), y[c][r], s);
                if (!VREG && (r & 7) == 7) asm volatile("" ::: "memory");
            }
            d[c] = s;
        }
        wave_sum_many<CPW>(d);
        if (!VREG) asm volatile("" ::: "memory");
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            if (!alive[c]) continue;
            const double dt = d[c] * tau;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                y[c][r] = fma(-dt, VREG ? v[VREG ? r : 0] : vof(lane + 64 * r), y[c][r]);
                if (!VREG && (r & 7) == 7) asm volatile("" ::: "memory");
            }
            const int64_t j = colbase + c;
            if (j == wj) {
                alive[c] = false;
#pragma unroll
                for (int r = 0; r < RPL; ++r)
                    if (lane + 64 * r == ti) y[c][r] = beta;
                if (lane == 0) a.pos[j] = (int32_t)t;
            }
        }
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                s = fma(i > ti ? y[c][r] : 0.0, y[c][r], s);
            }
            nu[c] = s;
        }
        wave_sum_many<CPW>(nu);
        if (blockIdx.x == 0 && threadIdx.x == 0) a.J[t] = wj;
        __syncthreads();  // LDS is rewritten next step
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

// ---------------------------------------------------------------------------
// Short sketches (l <= 256): lane-column layout.  A group of G lanes holds one
// column (lane part p holds rows [p*R, p*R + R)), so a wave holds 64/G
// columns and the dot products and norms of a column are lane-local sums
// combined over only log2(G) lane exchanges.  Same step structure, slot
// protocol and arithmetic definitions as cpqr_kernel.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ double tree_sum(double (&s)[N]) {
#pragma unroll
    for (int h = N / 2; h > 0; h >>= 1)
#pragma unroll
        for (int q = 0; q < h; ++q) s[q] += s[q + h];
    return s[0];
}

template <int G>
__device__ __forceinline__ double part_sum(double v) {
#pragma unroll
    for (int o = 64 / G; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int G, int R, int NW, bool ALL>
__global__ __launch_bounds__(NW * 64) void cpqr_lc_kernel(SelArgs a) {
    extern __shared__ double sm[];
    __shared__ double s_nu[NW];
    __shared__ int64_t s_j[NW];
    __shared__ double s_wnu;
    __shared__ int64_t s_wj;
    constexpr int NT = NW * 64;
    constexpr int CPWV = 64 / G;  // columns per wave

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int cl = lane % CPWV;   // column within the wave
    const int p = lane / CPWV;    // row part
    const int64_t j = ((int64_t)blockIdx.x * NW + w) * CPWV + cl;
    const int64_t l = a.l, n = a.n;
    const int S = a.S;
    const int64_t row0 = (int64_t)p * R;

    double y[R];
    bool alive = j < n;
    {
        const int64_t jc = min(j, n - 1);
        if (a.ydt == IDS_F64) {
            const double* Yp = (const double*)a.Y;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = (int)row0 + r;
                const double v = Yp[(int64_t)min(i, (int)l - 1) * a.rs + jc * a.cs];
                y[r] = (alive && i < l) ? v : 0.0;
            }
        } else {
            const float* Yp = (const float*)a.Y;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = (int)row0 + r;
                const double v = (double)Yp[(int64_t)min(i, (int)l - 1) * a.rs + jc * a.cs];
                y[r] = (alive && i < l) ? v : 0.0;
            }
        }
    }
    if (alive && p == 0) a.pos[j] = -1;
    // sums over a lane's rows use NACC interleaved accumulators (fixed order)
    constexpr int NACC = R >= 8 ? 8 : R;
    double nu;
    {
        double s[NACC];
#pragma unroll
        for (int q = 0; q < NACC; ++q) s[q] = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) s[r % NACC] = fma(y[r], y[r], s[r % NACC]);
        nu = part_sum<G>(tree_sum<NACC>(s));
    }

    int64_t keff = a.k;
    for (int64_t t = 0; t < a.k; ++t) {
        const int par = (int)(t & 1);
        double* slots = a.slot + (size_t)par * a.nb * S;
        // ---- 1. wave best, 2. workgroup best -> slot
        double wn = alive ? nu : -1.0;
        int wjj = alive ? (int)j : INT32_MAX;
        wave_argmax(wn, wjj);
        if (lane == 0) {
            s_nu[w] = wn;
            s_j[w] = (wjj == INT32_MAX) ? INT64_MAX : (int64_t)wjj;
        }
        __syncthreads();
        {
            double bn = s_nu[0];
            int64_t bj = s_j[0];
            for (int q = 1; q < NW; ++q)
                if (better(s_nu[q], s_j[q], bn, bj)) {
                    bn = s_nu[q];
                    bj = s_j[q];
                }
            if (threadIdx.x == 0) {
                double* sl = slots + (size_t)blockIdx.x * S;
                slot_store(sl, bn);
                slot_store(sl + 1, __longlong_as_double((bj == INT64_MAX) ? -1LL : (long long)bj));
            }
            if (alive && j == bj) {
                double* sl = slots + (size_t)blockIdx.x * S + 2;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int64_t i = row0 + r;
                    if (i < l) slot_store(sl + i, y[r]);
                }
                __builtin_amdgcn_s_waitcnt(0);
            }
        }
        // ---- 3. device-wide barrier
        grid_sync(a.bar, (uint32_t)(a.nb * (t + 1)));
        // ---- 4. winner
        if (ALL) {
            const int tot = a.nb * S;
            for (int e0 = 0; e0 < tot; e0 += NT * 8) {
                double tmp[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT + (int)threadIdx.x;
                    tmp[u] = (e < tot) ? slot_load(slots + e) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT + (int)threadIdx.x;
                    if (e < tot) sm[e] = tmp[u];
                }
            }
            __syncthreads();
        }
        {
            double bn = -1.0;
            int bjj = INT32_MAX;
            for (int q = threadIdx.x; q < a.nb; q += NT) {
                double nuq;
                int64_t jq;
                if (ALL) {
                    nuq = sm[(size_t)q * S];
                    jq = (int64_t)__double_as_longlong(sm[(size_t)q * S + 1]);
                } else {
                    nuq = slot_load(slots + (size_t)q * S);
                    jq = (int64_t)__double_as_longlong(slot_load(slots + (size_t)q * S + 1));
                }
                if (jq >= 0 && better(nuq, jq, bn, bjj)) {
                    bn = nuq;
                    bjj = (int)jq;
                }
            }
            wave_argmax(bn, bjj);
            if (lane == 0) {
                s_nu[w] = bn;
                s_j[w] = (bjj == INT32_MAX) ? INT64_MAX : (int64_t)bjj;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double b2 = s_nu[0];
                int64_t j2 = s_j[0];
                for (int q = 1; q < NW; ++q)
                    if (better(s_nu[q], s_j[q], b2, j2)) {
                        b2 = s_nu[q];
                        j2 = s_j[q];
                    }
                s_wnu = b2;
                s_wj = j2;
            }
            __syncthreads();
        }
        const double wnu = s_wnu;
        const int64_t wj = s_wj;
        if (wj == INT64_MAX || !(wnu > 0.0)) {
            keff = t;
            break;
        }
        const int wblk = (int)(wj / ((int64_t)NW * CPWV));
        const double* xb;
        if (ALL) {
            xb = sm + (size_t)wblk * S + 2;
        } else {
            const double* wsl = slots + (size_t)wblk * S + 2;
            for (int i = threadIdx.x; i < (int)l; i += NT) sm[i] = slot_load(wsl + i);
            __syncthreads();
            xb = sm;
        }
        // ---- Householder reflector (every wave, same bits)
        double sig2 = 0.0;
        for (int64_t i = t + 1 + lane; i < l; i += 64) sig2 = fma(xb[i], xb[i], sig2);
        sig2 = wave_sum_dpp1(sig2);
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
        // ---- 5. apply to the live column held by this lane group
        double dsum;
        {
            double s[NACC];
#pragma unroll
            for (int q = 0; q < NACC; ++q) s[q] = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t i = row0 + r;
                const double v = (i < t || i >= l) ? 0.0 : (i == t ? 1.0 : xb[i] * scal);
                s[r % NACC] = fma(v, y[r], s[r % NACC]);
            }
            dsum = part_sum<G>(tree_sum<NACC>(s));
        }
        asm volatile("" ::: "memory");
        if (alive) {
            const double dt = dsum * tau;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t i = row0 + r;
                const double v = (i < t || i >= l) ? 0.0 : (i == t ? 1.0 : xb[i] * scal);
                y[r] = fma(-dt, v, y[r]);
            }
            if (j == wj) {
                alive = false;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (row0 + r == t) y[r] = beta;
                if (p == 0) a.pos[j] = (int32_t)t;
            }
        }
        {
            double s[NACC];
#pragma unroll
            for (int q = 0; q < NACC; ++q) s[q] = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int64_t i = row0 + r;
                if (i > t) s[r % NACC] = fma(y[r], y[r], s[r % NACC]);
            }
            nu = part_sum<G>(tree_sum<NACC>(s));
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) a.J[t] = wj;
        __syncthreads();
    }

    if (j < n) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = row0 + r;
            if (i < keff) a.Rt[j * a.k + i] = y[r];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const bool timed_out = __hip_atomic_load(a.bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        *a.keff = timed_out ? -1 : keff;
        for (int64_t t = keff; t < a.k; ++t) a.J[t] = -1;
    }
}

// ---------------------------------------------------------------------------
// Short sketches, grouped-lane layout: column c of a wave lives in the G
// consecutive lanes 8..: lane = G*c + p holds rows [p*R, p*R + R) of it.  Column
// sums are G-lane DPP trees (quad_perm, half-mirror, mirror: every lane of the
// group ends with the same bits); updates are branch-free; every wave resolves
// the workgroup and device argmax itself from LDS, so a step has three
// workgroup barriers plus the device-wide one.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    if (G >= 2) v += dpp_f64<0xB1, 0xf>(v);   // lanes i, i^1
    if (G >= 4) v += dpp_f64<0x4E, 0xf>(v);   // lanes i, i^2
    if (G >= 8) v += dpp_f64<0x141, 0xf>(v);  // half-row mirror (8 lanes)
    if (G >= 16) v += dpp_f64<0x140, 0xf>(v); // row mirror (16 lanes)
    return v;
}

template <int G, int R, int NW, bool ALL>
__global__ __launch_bounds__(NW * 64) void cpqr_gl_kernel(SelArgs a) {
    extern __shared__ double sm[];
    __shared__ double s_nu[NW];
    __shared__ int s_j[NW];
    constexpr int NT = NW * 64;
    constexpr int CPWV = 64 / G;  // columns per wave

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int p = lane % G;       // row part
    const int wcol0 = (blockIdx.x * NW + w) * CPWV;
    const int j = wcol0 + lane / G;
    const int n = (int)a.n, l = (int)a.l;
    const int S = a.S;
    const int row0 = p * R;

    double y[R];
    bool alive = j < n;
    {
        const int64_t jc = min(j, n - 1);
        if (a.ydt == IDS_F64) {
            const double* Yp = (const double*)a.Y;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = row0 + r;
                const double v = Yp[(int64_t)min(i, l - 1) * a.rs + jc * a.cs];
                y[r] = (alive && i < l) ? v : 0.0;
            }
        } else {
            const float* Yp = (const float*)a.Y;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = row0 + r;
                const double v = (double)Yp[(int64_t)min(i, l - 1) * a.rs + jc * a.cs];
                y[r] = (alive && i < l) ? v : 0.0;
            }
        }
    }
    if (alive && p == 0) a.pos[j] = -1;
    double nu;
    {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) s = fma(y[r], y[r], s);
        nu = group_sum<G>(s);
    }

    const int k = (int)a.k;
    int keff = k;
    for (int t = 0; t < k; ++t) {
        const int par = t & 1;
        double* slots = a.slot + (size_t)par * a.nb * S;
        // ---- wave best, then workgroup best (every wave computes it)
        {
            double wn = alive ? nu : -1.0;
            int wj = alive ? j : INT32_MAX;
            wave_argmax(wn, wj);
            if (lane == 0) {
                s_nu[w] = wn;
                s_j[w] = wj;
            }
        }
        __syncthreads();
        double bn = (lane < NW) ? s_nu[lane] : -1.0;
        int bj = (lane < NW) ? s_j[lane] : INT32_MAX;
        wave_argmax(bn, bj);
        if (threadIdx.x == 0) {
            double* sl = slots + (size_t)blockIdx.x * S;
            slot_store(sl, bn);
            slot_store(sl + 1, __longlong_as_double((bj == INT32_MAX) ? -1LL : (long long)bj));
        }
        if (j == bj) {  // the G lanes of the workgroup's best column publish it
            double* sl = slots + (size_t)blockIdx.x * S + 2 + row0;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (row0 + r < l) slot_store(sl + r, y[r]);
            __builtin_amdgcn_s_waitcnt(0);
        }
        // ---- device-wide barrier
        grid_sync(a.bar, (uint32_t)(a.nb * (t + 1)));
        // ---- every wave finds the winner
        if (ALL) {
            const int tot = a.nb * S;
            for (int e0 = 0; e0 < tot; e0 += NT * 8) {
                double tmp[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT + (int)threadIdx.x;
                    tmp[u] = (e < tot) ? slot_load(slots + e) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT + (int)threadIdx.x;
                    if (e < tot) sm[e] = tmp[u];
                }
            }
            __syncthreads();
        }
        double wnu = -1.0;
        int wj = INT32_MAX;
        for (int q = lane; q < a.nb; q += 64) {
            double nq;
            long long jq;
            if (ALL) {
                nq = sm[(size_t)q * S];
                jq = __double_as_longlong(sm[(size_t)q * S + 1]);
            } else {
                nq = slot_load(slots + (size_t)q * S);
                jq = __double_as_longlong(slot_load(slots + (size_t)q * S + 1));
            }
            if (jq >= 0 && (nq > wnu || (nq == wnu && (int)jq < wj))) {
                wnu = nq;
                wj = (int)jq;
            }
        }
        wave_argmax(wnu, wj);
        if (wj == INT32_MAX || !(wnu > 0.0)) {
            keff = t;
            break;
        }
        const int wblk = wj / (NW * CPWV);
        const double* xb;
        if (ALL) {
            xb = sm + (size_t)wblk * S + 2;
        } else {
            const double* wsl = slots + (size_t)wblk * S + 2;
            for (int i = threadIdx.x; i < l; i += NT) sm[i] = slot_load(wsl + i);
            __syncthreads();
            xb = sm;
        }
        // ---- Householder reflector (every wave, same bits)
        double sig2 = 0.0;
        for (int i = t + 1 + lane; i < l; i += 64) sig2 = fma(xb[i], xb[i], sig2);
        sig2 = wave_sum_dpp1(sig2);
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
        double v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = row0 + r;
            const double xi = xb[min(i, l - 1)];
            v[r] = (i < t || i >= l) ? 0.0 : (i == t ? 1.0 : xi * scal);
        }
        // ---- apply H (branch-free: dead columns get a zero multiplier)
        double d = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) d = fma(v[r], y[r], d);
        d = group_sum<G>(d);
        const double dt = alive ? d * tau : 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = fma(-dt, v[r], y[r]);
        if (j == wj) {
            alive = false;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (row0 + r == t) y[r] = beta;
            if (p == 0) a.pos[j] = t;
        }
        // ---- trailing norms for the next step (rows > t)
        {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double yr = (row0 + r > t) ? y[r] : 0.0;
                s = fma(yr, yr, s);
            }
            nu = group_sum<G>(s);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) a.J[t] = wj;
        __syncthreads();  // LDS is rewritten next step
    }

    if (j < n) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = row0 + r;
            if (i < keff) a.Rt[(int64_t)j * a.k + i] = y[r];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const bool timed_out = __hip_atomic_load(a.bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        *a.keff = timed_out ? -1 : keff;
        for (int t = keff; t < a.k; ++t) a.J[t] = -1;
    }
}

// ---------------------------------------------------------------------------
// Tall sketches (2048 < l <= 64 * (RREG + RLDS)): one column per wave; rows
// lane + 64 r, r < RREG, in registers and the remaining RLDS chunks of 64 rows
// in LDS (per wave), so a 4096-row FP64 column fits beside the winner's copy.
// Same step structure and arithmetic as cpqr_kernel.
// ---------------------------------------------------------------------------
template <int RREG, int RLDS, int NW>
__global__ __launch_bounds__(NW * 64) void cpqr_tall_kernel(SelArgs a) {
    extern __shared__ double sm[];
    constexpr int LP = 64 * (RREG + RLDS);           // rows covered (>= l)
    double* xb = sm;                                 // winner column, LP entries (zero past l)
    double* yl = sm + LP;                            // NW x RLDS x 64 rows held in LDS
    __shared__ double s_nu[NW];
    __shared__ int s_j[NW];
    constexpr int NT = NW * 64;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int j = blockIdx.x * NW + w;
    const int n = (int)a.n, l = (int)a.l, S = a.S;
    double* myl = yl + (size_t)w * RLDS * 64 + lane;  // chunk RREG + q of this lane at myl[64 q]

    // Row i = lane + 64 r.  Predicates on i are uniform per chunk r except for
    // the one chunk that contains the boundary, which keeps the masks scalar.
    double y[RREG];
    bool alive = j < n;
    {
        const int64_t jc = min(j, n - 1);
        auto ld = [&](int i) -> double {
            double v;
            if (a.ydt == IDS_F64)
                v = ((const double*)a.Y)[(int64_t)min(i, l - 1) * a.rs + jc * a.cs];
            else
                v = (double)((const float*)a.Y)[(int64_t)min(i, l - 1) * a.rs + jc * a.cs];
            return (alive && i < l) ? v : 0.0;
        };
#pragma unroll
        for (int r = 0; r < RREG; ++r) y[r] = ld(lane + 64 * r);
        for (int q = 0; q < RLDS; ++q) myl[64 * q] = ld(lane + 64 * (RREG + q));
    }
    if (alive && lane == 0) a.pos[j] = -1;
    // sum of squares over rows i >= from
    auto trailing = [&](int from) -> double {
        const int c0 = from >> 6, lo = from & 63;
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RREG; ++r) {
            if (r < c0) continue;
            const double yr = (r == c0 && lane < lo) ? 0.0 : y[r];
            s = fma(yr, yr, s);
        }
        for (int q = max(c0 - RREG, 0); q < RLDS; ++q) {
            const double yq = myl[64 * q];
            const double yr = (RREG + q == c0 && lane < lo) ? 0.0 : yq;
            s = fma(yr, yr, s);
        }
        return wave_sum_dpp1(s);
    };
    double nu = trailing(0);

    const int k = (int)a.k;
    int keff = k;
    for (int t = 0; t < k; ++t) {
        const int par = t & 1;
        double* slots = a.slot + (size_t)par * a.nb * S;
        if (lane == 0) {
            s_nu[w] = alive ? nu : -1.0;
            s_j[w] = alive ? j : INT32_MAX;
        }
        __syncthreads();
        double bn = (lane < NW) ? s_nu[lane] : -1.0;
        int bj = (lane < NW) ? s_j[lane] : INT32_MAX;
        wave_argmax(bn, bj);
        if (threadIdx.x == 0) {
            double* sl = slots + (size_t)blockIdx.x * S;
            slot_store(sl, bn);
            slot_store(sl + 1, __longlong_as_double((bj == INT32_MAX) ? -1LL : (long long)bj));
        }
        if (j == bj) {  // rows < l only: the slot holds S >= l + 2 entries
            double* sl = slots + (size_t)blockIdx.x * S + 2 + lane;
#pragma unroll
            for (int r = 0; r < RREG; ++r)
                if (lane + 64 * r < l) slot_store(sl + 64 * r, y[r]);
            for (int q = 0; q < RLDS; ++q)
                if (lane + 64 * (RREG + q) < l) slot_store(sl + 64 * (RREG + q), myl[64 * q]);
            __builtin_amdgcn_s_waitcnt(0);
        }
        grid_sync(a.bar, (uint32_t)(a.nb * (t + 1)));
        double wnu = -1.0;
        int wj = INT32_MAX;
        for (int q = lane; q < a.nb; q += 64) {
            const double nq = slot_load(slots + (size_t)q * S);
            const long long jq = __double_as_longlong(slot_load(slots + (size_t)q * S + 1));
            if (jq >= 0 && (nq > wnu || (nq == wnu && (int)jq < wj))) {
                wnu = nq;
                wj = (int)jq;
            }
        }
        wave_argmax(wnu, wj);
        if (wj == INT32_MAX || !(wnu > 0.0)) {
            keff = t;
            break;
        }
        {
            const double* wsl = slots + (size_t)(wj / NW) * S + 2;
            const int lp = LP;
            for (int i0 = 0; i0 < lp; i0 += NT * 8) {
                double tmp[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + u * NT + (int)threadIdx.x;
                    tmp[u] = (i < l) ? slot_load(wsl + i) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = i0 + u * NT + (int)threadIdx.x;
                    if (i < lp) xb[i] = tmp[u];
                }
            }
        }
        __syncthreads();
        double sig2 = 0.0;
        for (int i = t + 1 + lane; i < l; i += 64) sig2 = fma(xb[i], xb[i], sig2);
        sig2 = wave_sum_dpp1(sig2);
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
        const int c0 = t >> 6, lo = t & 63;
        // reflector entry of chunk r for this lane: 0 above t, 1 at t, x_i scal below
        auto vchunk = [&](int r) -> double {
            const double x = xb[lane + 64 * r] * scal;
            return (r == c0) ? (lane < lo ? 0.0 : (lane == lo ? 1.0 : x)) : x;
        };
        double d = 0.0;
#pragma unroll
        for (int r = 0; r < RREG; ++r)
            if (r >= c0) d = fma(vchunk(r), y[r], d);
        for (int q = max(c0 - RREG, 0); q < RLDS; ++q) d = fma(vchunk(RREG + q), myl[64 * q], d);
        d = wave_sum_dpp1(d);
        const double dt = alive ? d * tau : 0.0;
#pragma unroll
        for (int r = 0; r < RREG; ++r)
            if (r >= c0) y[r] = fma(-dt, vchunk(r), y[r]);
        for (int q = max(c0 - RREG, 0); q < RLDS; ++q) myl[64 * q] = fma(-dt, vchunk(RREG + q), myl[64 * q]);
        if (j == wj) {
            alive = false;
            if (c0 < RREG) {
#pragma unroll
                for (int r = 0; r < RREG; ++r)
                    if (r == c0 && lane == lo) y[r] = beta;
            } else if (lane == lo) {
                myl[64 * (c0 - RREG)] = beta;
            }
            if (lane == 0) a.pos[j] = t;
        }
        nu = trailing(t + 1);
        if (blockIdx.x == 0 && threadIdx.x == 0) a.J[t] = wj;
        __syncthreads();
    }
    if (j < n) {
        double* Rj = a.Rt + (int64_t)j * a.k;
#pragma unroll
        for (int r = 0; r < RREG; ++r)
            if (lane + 64 * r < keff) Rj[lane + 64 * r] = y[r];
        for (int q = 0; q < RLDS; ++q)
            if (lane + 64 * (RREG + q) < keff) Rj[lane + 64 * (RREG + q)] = myl[64 * q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const bool timed_out = __hip_atomic_load(a.bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        *a.keff = timed_out ? -1 : keff;
        for (int t = keff; t < a.k; ++t) a.J[t] = -1;
    }
}

__global__ void zero_u32_kernel(uint32_t* p, int count) {
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0u;
}

// P[:, j]: e_t for a chosen column, R11^{-1} R[0:keff, j] otherwise, by
// back-substitution (one thread per column, in the order of the textbook
// recurrence x_r = (b_r - sum_{c>r} R11[r][c] x_c) / R11[r][r]).  The solution
// vector of each thread lives in LDS (xs[c][thread]); R11 is staged in LDS
// when it fits.
constexpr int TRSM_THREADS = 64;
template <bool R11_LDS, bool X_LDS>
__global__ __launch_bounds__(TRSM_THREADS) void trsm_p_kernel(int64_t n, int64_t k, const double* __restrict__ Rt,
                                                              const int64_t* __restrict__ J,
                                                              const int32_t* __restrict__ pos,
                                                              const int64_t* __restrict__ keffp, double* P) {
    extern __shared__ double sm[];
    const int64_t keff = *keffp;
    if (keff < 0) return;
    double* R11s = sm;
    double* xs = sm + (R11_LDS ? k * k : 0);
    if (R11_LDS) {
        for (int64_t e = threadIdx.x; e < keff * keff; e += TRSM_THREADS) {
            const int64_t r = e / keff, c = e % keff;
            R11s[e] = (r <= c) ? Rt[J[c] * k + r] : 0.0;
        }
        __syncthreads();
    }
    const int tid = threadIdx.x;
    const int64_t j = (int64_t)blockIdx.x * TRSM_THREADS + tid;
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
            const double xc = X_LDS ? xs[c * TRSM_THREADS + tid] : P[c * n + j];
            s = fma(-rc, xc, s);
        }
        const double d = R11_LDS ? R11s[r * keff + r] : Rt[J[r] * k + r];
        const double x = s / d;
        if (X_LDS) xs[r * TRSM_THREADS + tid] = x;
        P[r * n + j] = x;
    }
    for (int64_t r = keff; r < k; ++r) P[r * n + j] = 0.0;
}

// Faster variant for k <= 16*KS: a group of 16 lanes solves one column.  Lane q
// of the group keeps x_c and b_c for c = 16*s + q in register slot s; at step r
// every lane forms its part of b_r - sum_{c>r} R11[r][c] x_c, the 16 parts are
// summed with DPP row operations, and x_r = (that sum) / R11[r][r].
template <int KS, bool R11_LDS>
__global__ __launch_bounds__(256) void trsm_group_kernel(int64_t n, int64_t k, const double* __restrict__ Rt,
                                                         const int64_t* __restrict__ J,
                                                         const int32_t* __restrict__ pos,
                                                         const int64_t* __restrict__ keffp, double* P) {
    extern __shared__ double R11s[];
    const int64_t keff = *keffp;
    if (keff < 0) return;
    if (R11_LDS) {
        for (int64_t e = threadIdx.x; e < keff * keff; e += 256) {
            const int64_t r = e / keff, c = e % keff;
            R11s[e] = (r <= c) ? Rt[J[c] * k + r] : 0.0;
        }
        __syncthreads();
    }
    const int q = threadIdx.x & 15;
    const int64_t j = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    if (j >= n) return;
    const int32_t pj = pos[j];
    if (pj >= 0) {
        for (int64_t r = q; r < k; r += 16) P[r * n + j] = (r == pj) ? 1.0 : 0.0;
        return;
    }
    double b[KS], x[KS];
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) {
        const int64_t c = 16 * sl + q;
        b[sl] = (c < keff) ? Rt[j * k + c] : 0.0;
        x[sl] = 0.0;
    }
    for (int64_t r = keff - 1; r >= 0; --r) {
        double part = 0.0;
#pragma unroll
        for (int sl = 0; sl < KS; ++sl) {
            const int64_t c = 16 * sl + q;
            if (c == r) part = b[sl];
            if (c > r && c < keff) {
                const double rc = R11_LDS ? R11s[r * keff + c] : Rt[J[c] * k + r];
                part = fma(-rc, x[sl], part);
            }
        }
        part += dpp_f64<0xB1, 0xf>(part);
        part += dpp_f64<0x4E, 0xf>(part);
        part += dpp_f64<0x141, 0xf>(part);
        part += dpp_f64<0x140, 0xf>(part);
        const double d = R11_LDS ? R11s[r * keff + r] : Rt[J[r] * k + r];
        const double xr = part / d;
        if (q == (int)(r & 15)) {
#pragma unroll
            for (int sl = 0; sl < KS; ++sl)
                if (sl == (int)(r >> 4)) x[sl] = xr;
        }
        if (q == 0) P[r * n + j] = xr;
    }
    for (int64_t r = keff + q; r < k; r += 16) P[r * n + j] = 0.0;
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
    const void* fn_all;
    const void* fn_one;
    size_t lds_extra = 0;  // tall kernel: LDS-held rows (bytes per workgroup)
};

template <int RPL, int CPW, int NW>
static Inst inst() {
    return {RPL, CPW, NW, (const void*)&cpqr_kernel<RPL, CPW, NW, true>,
            (const void*)&cpqr_kernel<RPL, CPW, NW, false>};
}

// lane-column kernels: G lanes per column, R rows per lane; reported as
// (rpl = -R, cpw = 64 / G) so the column count per workgroup is cpw * nw
template <int G, int R, int NW>
static Inst inst_lc() {
    return {-R, 64 / G, NW, (const void*)&cpqr_lc_kernel<G, R, NW, true>,
            (const void*)&cpqr_lc_kernel<G, R, NW, false>};
}
template <int G, int R, int NW>
static Inst inst_gl() {
    return {-R, 64 / G, NW, (const void*)&cpqr_gl_kernel<G, R, NW, true>,
            (const void*)&cpqr_gl_kernel<G, R, NW, false>};
}

static bool pick(int64_t l, Inst& in) {
    // grouped-lane kernels for short sketches, column-per-wave beyond 256 rows
    if (l <= 32) in = inst_gl<2, 16, 8>();
    else if (l <= 64) in = inst_gl<4, 16, 8>();
    else if (l <= 128) in = inst_gl<8, 16, 8>();
    else if (l <= 256) in = inst_gl<16, 16, 8>();
    else if (l <= 512) in = inst<8, 2, 8>();
    else if (l <= 1024) in = inst<16, 1, 8>();
    else if (l <= 2048) in = inst<32, 1, 8>();
    else if (l <= 4096) {
        // 40 chunks of 64 rows in registers, 24 in LDS (12 KB per wave)
        const void* f = (const void*)&cpqr_tall_kernel<40, 24, 8>;
        in = {64, 1, 8, f, f, sizeof(double) * 8 * 24 * 64};
    }
    else return false;
    return true;
}

static int slot_stride(int64_t l) { return (int)((l + 2 + 31) / 32 * 32); }
constexpr size_t ALL_SLOTS_LDS_MAX = 64 * 1024;

static size_t cpqr_lds(const SelectPlan& sp, bool& all) {
    const size_t S = (size_t)slot_stride(sp.l);
    if (sp.l > 2048) {  // tall kernel: winner column (4096 rows) + LDS-held rows
        all = false;
        return sizeof(double) * 64 * 64 + sizeof(double) * 8 * 24 * 64;
    }
    all = sizeof(double) * S * sp.nb <= ALL_SLOTS_LDS_MAX;
    return all ? sizeof(double) * S * sp.nb : sizeof(double) * S;
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
    bool all = false;
    const size_t lds = cpqr_lds(sp, all);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, all ? in.fn_all : in.fn_one, in.nw * 64, lds) !=
        hipSuccess)
        per_cu = 1;
    if ((int64_t)sp.nb > (int64_t)ncu * per_cu) {
        set_error("id_select: n too large for the register-resident CPQR (n = " + std::to_string(n) +
                  ", l = " + std::to_string(l) + ", max columns " + std::to_string((int64_t)ncu * per_cu * per) +
                  ")");
        return IDS_EINVAL;
    }
    return IDS_OK;
}

size_t select_bytes(const SelectPlan& sp) {
    return align256(sizeof(double) * 2 * sp.nb * (size_t)slot_stride(sp.l)) + align256(sizeof(uint32_t) * 2) +
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
    a.S = slot_stride(sp.l);
    char* p = ws;
    a.slot = (double*)p;
    p += align256(sizeof(double) * 2 * sp.nb * (size_t)a.S);
    a.bar = (uint32_t*)p;
    p += align256(sizeof(uint32_t) * 2);
    a.Rt = (double*)p;
    p += align256(sizeof(double) * (size_t)sp.n * sp.k);
    a.pos = (int32_t*)p;

    Inst in;
    pick(sp.l, in);
    bool all = false;
    const size_t lds = cpqr_lds(sp, all);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, st, a.bar, 2);
    void* args[] = {&a};
    {
        ProfScope ps(PK_CPQR, st);
        hipError_t e = hipLaunchCooperativeKernel(all ? in.fn_all : in.fn_one, dim3(sp.nb), dim3(in.nw * 64), args,
                                                  (unsigned)lds, st);
        if (e != hipSuccess) {
            set_error(std::string("cpqr cooperative launch: ") + hipGetErrorString(e));
            return IDS_EHIP;
        }
    }
    ProfScope ps(PK_TRSM, st);
    const size_t r11 = sizeof(double) * (size_t)sp.k * sp.k;
    const size_t xb = sizeof(double) * (size_t)sp.k * TRSM_THREADS;
    const unsigned g = (unsigned)((sp.n + TRSM_THREADS - 1) / TRSM_THREADS);
    const size_t lim = lds_limit();
    const double* Rt = a.Rt;
    const int32_t* pos = a.pos;
    const unsigned g16 = (unsigned)((sp.n + 15) / 16);
#define IDS_TRSM_GROUP(KS)                                                                                         \
    do {                                                                                                           \
        if (r11 <= lim)                                                                                            \
            hipLaunchKernelGGL((trsm_group_kernel<KS, true>), dim3(g16), dim3(256), r11, st, sp.n, sp.k, Rt,       \
                               (const int64_t*)J, pos, (const int64_t*)keff, P);                                   \
        else                                                                                                       \
            hipLaunchKernelGGL((trsm_group_kernel<KS, false>), dim3(g16), dim3(256), 0, st, sp.n, sp.k, Rt,        \
                               (const int64_t*)J, pos, (const int64_t*)keff, P);                                   \
    } while (0)
    if (sp.k <= 32)
        IDS_TRSM_GROUP(2);
    else if (sp.k <= 64)
        IDS_TRSM_GROUP(4);
    else if (sp.k <= 128)
        IDS_TRSM_GROUP(8);
    else if (sp.k <= 256)
        IDS_TRSM_GROUP(16);
#undef IDS_TRSM_GROUP
    else if (r11 + xb <= lim)
        hipLaunchKernelGGL((trsm_p_kernel<true, true>), dim3(g), dim3(TRSM_THREADS), r11 + xb, st, sp.n, sp.k, Rt,
                           (const int64_t*)J, pos, (const int64_t*)keff, P);
    else if (xb <= lim)
        hipLaunchKernelGGL((trsm_p_kernel<false, true>), dim3(g), dim3(TRSM_THREADS), xb, st, sp.n, sp.k, Rt,
                           (const int64_t*)J, pos, (const int64_t*)keff, P);
    else
        hipLaunchKernelGGL((trsm_p_kernel<false, false>), dim3(g), dim3(TRSM_THREADS), 0, st, sp.n, sp.k, Rt,
                           (const int64_t*)J, pos, (const int64_t*)keff, P);
    return check_launch("cpqr / interpolation matrix");
}

ids_status lambda_hat(int64_t k, int64_t n, const double* P, const int64_t* J, const int64_t* keff,
                      const double* lambda, double* lhat, hipStream_t st) {
    hipLaunchKernelGGL(lambda_hat_kernel, dim3((unsigned)k), dim3(256), 0, st, k, n, P, J, keff, lambda, lhat);
    return check_launch("lambda_hat");
}

}  // namespace ids

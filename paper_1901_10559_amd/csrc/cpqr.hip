// Algorithm 1 on a sketch Y (l x n): rank-k column-pivoted QR, then
// P = [I, R11^{-1} R12] Pi^T in the original column order.
//
// The factorisation is one persistent cooperative kernel.  The columns of Y
// are spread over the workgroups and stay in registers for all k steps.  One
// step t:
//   1. each workgroup finds its best live column (largest trailing squared
//      norm, ties to the smallest column index) and publishes (norm, index);
//   2. every workgroup reads all published candidates and picks the same
//      winner;
//   3. the winner's column reaches every workgroup, which forms the
//      Householder reflector of its rows t..l-1 (v_t = 1,
//      beta = -sign(alpha) ||x||, tau = (beta - alpha) / beta) and applies it
//      to its live columns; row t of a column then holds R[t][j];
//   4. the trailing squared norms (rows > t) are recomputed in FP64 (no
//      downdating, so no cancellation guard is needed).
// After k steps the top k rows of column j hold R[0:k, j].  The trsm kernels
// then solve R11 x = R[0:k, j] per column and write P.
//
// Exchange between workgroups: write-once mailboxes.  Step t owns its own
// region of the workspace, filled with the sentinel pattern MB_SENT (a
// signalling-NaN bit pattern) before the kernel starts.  Writers store each
// 8-byte value once with agent-scope atomic stores; readers reload a value
// until it differs from the sentinel.  A location only ever holds the
// sentinel or its final value and 8-byte accesses are single-copy atomic, so
// a value that is not the sentinel is the value: there is no barrier counter,
// fence or flag per step, and a reader waits only for the data it needs.
// Data whose bits equal MB_SENT are stored as the canonical quiet NaN.
// A step region starts with the headers, packed (publisher q at 2 q, 2 q + 1)
// so that the vote polls a few cache lines only.  Two ways to move the
// winner's column (chosen on the host by size):
//   MB_SPEC  every publisher also writes its best column speculatively into
//            its own column slot; after the vote everyone reads the winner's.
//            The slots form two sets used by alternate steps: once the vote
//            of step t is complete every workgroup has finished step t - 1,
//            so each workgroup resets its own slot of that set to the
//            sentinel for step t + 1, and waits for those stores to complete
//            before the barrier that precedes its next publication (the one
//            place where a location is written twice: sentinel, then value);
//   MB_OWNER headers only; after the vote the owner of the winner publishes
//            its column into the step's column box, which follows the
//            headers (many publishers or very long columns).
// The reflector norm is the winner's published trailing norm:
// ||x_{t..l-1}||^2 = nu_winner, so beta = -sign(alpha) sqrt(nu_winner) and no
// workgroup re-sums the column.  (nu_winner <= alpha^2 means the entries
// below the diagonal vanish to rounding: H = I, as when they are exactly 0.)
// Every wait is capped; on expiry a device flag is raised, every other wait
// gives up at once, and k_eff is reported as -1.
#include <algorithm>
#include <atomic>

#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"
#include "tune.hpp"

namespace ids {

enum { MB_SPEC = 0, MB_OWNER = 1 };

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

struct SelArgs {
    const void* Y;
    int32_t ydt;
    int64_t l, n, rs, cs, k;
    int64_t* J;
    int64_t* keff;
    double* Rt;       // n x k (column j's top rows contiguous)
    double* R11c;     // k x k: row t = top rows of the column chosen at step t
    int32_t* pos;     // n: step at which the column was chosen, -1 otherwise
    double* mb;       // k step regions of RS doubles each, sentinel-filled
    uint32_t* flag;   // [0] timeout flag, [1] non-finite norm seen
    int32_t* status;  // optional device status word (IDS_OK, IDS_ERANKDEF, ...)
    uint32_t spin_limit;  // polls before a wait gives up
    int32_t nh;       // publishers (headers per step)
    int32_t S;        // MB_SPEC: stride of the publishers' column slots
    int32_t H0;       // header q at 2 q, 2 q + 1 of a step region; MB_OWNER: column box at H0
    int64_t RS;       // doubles per step region
    double* ring;     // MB_SPEC: two sets of column slots (step t uses set t & 1)
    int64_t CS;       // MB_SPEC: doubles per set (nh slots of S)
};

constexpr uint64_t MB_SENT = 0xFFF4A5A5A5A5A5A5ull;
constexpr uint64_t MB_QNAN = 0x7FF8000000000000ull;
constexpr uint32_t SPIN_LIMIT = 1u << 20;  // default polls before a wait gives up

// MB_SPEC column slots of step t
__device__ __forceinline__ double* spec_slots(const SelArgs& a, int t) { return a.ring + (size_t)(t & 1) * a.CS; }

// back to the sentinel (a slot reused two steps later)
__device__ __forceinline__ void mb_clear(double* p) {
    __hip_atomic_store((uint64_t*)p, MB_SENT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void mb_put(double* p, double v) {
    uint64_t b = (uint64_t)__double_as_longlong(v);
    if (b == MB_SENT) b = MB_QNAN;
    __hip_atomic_store((uint64_t*)p, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t mb_load(const double* p) {
    return __hip_atomic_load((uint64_t*)const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double mb_val(uint64_t b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ double idx_bits(int j) { return __longlong_as_double((long long)j); }

// U values per lane from addr(u) (nullptr: unused, reads as 0).  Sentinel
// entries are reloaded until every lane of the wave has final values; the
// loop is wave-uniform.  On timeout the flag is raised and the remaining
// entries keep the sentinel (a NaN).  SLEEP: pause about 64 clocks between
// polls (less polling traffic on the lines being published; used where the
// awaited data is normally on its way already).
template <int U, bool SLEEP = false, class F>
__device__ __forceinline__ void mb_read(uint64_t (&v)[U], F addr, const SelArgs& a) {
    uint32_t* flag = a.flag;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const double* p = addr(u);
        v[u] = p ? mb_load(p) : 0ull;
    }
    for (uint32_t spin = 0;; ++spin) {
        if (SLEEP && spin) __builtin_amdgcn_s_sleep(1);
        bool pend = false;
#pragma unroll
        for (int u = 0; u < U; ++u) pend = pend || (v[u] == MB_SENT);
        if (!__any(pend)) return;
        if (spin >= a.spin_limit ||
            ((spin & 63) == 63 && __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            if (pend) __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (v[u] == MB_SENT) v[u] = mb_load(addr(u));
    }
}

// preset != 0 raises the timeout flag before the factorisation starts: every
// wait then gives up as soon as it finds data missing (a host-forced test of
// the give-up path; the kernels still run their bounded loops to the end)
__global__ void mb_fill_kernel(uint64_t* mb, int64_t count, uint32_t* flag, uint32_t preset) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        flag[0] = preset;
        flag[1] = 0u;
    }
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
        mb[e] = MB_SENT;
}

// argmax over the wave of (nu, j): largest nu, then smallest j; j < 2^31.
// DPP max / min trees fold into lane 63, which is broadcast.  With SKIP = s,
// aligned groups of 2^s lanes hold identical pairs and the first s steps
// (which only combine lanes inside such a group) are left out.
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
template <int SKIP = 0>
__device__ __forceinline__ void wave_argmax(double& nu, int& j) {
    double m = nu;
    if (SKIP < 1) m = fmax(m, dpp_keep_f64<0xB1, 0xf>(m));
    if (SKIP < 2) m = fmax(m, dpp_keep_f64<0x4E, 0xf>(m));
    if (SKIP < 3) m = fmax(m, dpp_keep_f64<0x141, 0xf>(m));
    if (SKIP < 4) m = fmax(m, dpp_keep_f64<0x140, 0xf>(m));
    m = fmax(m, dpp_keep_f64<0x142, 0xa>(m));
    m = fmax(m, dpp_keep_f64<0x143, 0xc>(m));
    m = lane63_f64(m);
    int q = (nu == m) ? j : INT32_MAX;
    if (SKIP < 1) q = min(q, dpp_keep_i32<0xB1, 0xf>(q));
    if (SKIP < 2) q = min(q, dpp_keep_i32<0x4E, 0xf>(q));
    if (SKIP < 3) q = min(q, dpp_keep_i32<0x141, 0xf>(q));
    if (SKIP < 4) q = min(q, dpp_keep_i32<0x140, 0xf>(q));
    q = min(q, dpp_keep_i32<0x142, 0xa>(q));
    q = min(q, dpp_keep_i32<0x143, 0xc>(q));
    nu = m;
    j = __builtin_amdgcn_readlane(q, 63);
}

// the same over lanes 0..NL-1 only (NL = 2, 4, 8, 16), broadcast from lane 0
template <int NL>
__device__ __forceinline__ void wave_argmax_lo(double& nu, int& j) {
    static_assert(NL == 2 || NL == 4 || NL == 8 || NL == 16, "NL must be 2, 4, 8 or 16");
    double m = nu;
    m = fmax(m, dpp_keep_f64<0xB1, 0xf>(m));
    if (NL >= 4) m = fmax(m, dpp_keep_f64<0x4E, 0xf>(m));
    if (NL >= 8) m = fmax(m, dpp_keep_f64<0x141, 0xf>(m));
    if (NL >= 16) m = fmax(m, dpp_keep_f64<0x140, 0xf>(m));
    m = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(m), 0),
                         __builtin_amdgcn_readlane(__double2loint(m), 0));
    int q = (nu == m) ? j : INT32_MAX;
    q = min(q, dpp_keep_i32<0xB1, 0xf>(q));
    if (NL >= 4) q = min(q, dpp_keep_i32<0x4E, 0xf>(q));
    if (NL >= 8) q = min(q, dpp_keep_i32<0x141, 0xf>(q));
    if (NL >= 16) q = min(q, dpp_keep_i32<0x140, 0xf>(q));
    nu = m;
    j = __builtin_amdgcn_readlane(q, 0);
}

// fold one published header into a running (norm, index) best
__device__ __forceinline__ void take(uint64_t nb_bits, uint64_t j_bits, double& bn, int& bj) {
    const double nq = mb_val(nb_bits);
    const long long jq = (long long)j_bits;
    if (jq >= 0 && jq < INT32_MAX && (nq > bn || (nq == bn && (int)jq < bj))) {
        bn = nq;
        bj = (int)jq;
    }
}

// The vote from headers: the nh headers (header q at reg + q * hs) are read
// by all threads of the workgroup (up to 4 each), reduced per wave, then over
// the waves through LDS; every wave returns the same winner.
constexpr int VOTE_PER_THREAD = 4;
template <int NW, bool SLEEP>
__device__ __forceinline__ void vote_hdr(const SelArgs& a, const double* reg, int hs, double* s_vn, int* s_vj,
                                         double& wnu, int& wj) {
    constexpr int NT = NW * 64;
    constexpr int UH = VOTE_PER_THREAD;
    uint64_t hv[2 * UH];
    mb_read<2 * UH, SLEEP>(
        hv,
        [&](int u) -> const double* {
            const int q = (int)threadIdx.x + NT * (u >> 1);
            return q < a.nh ? reg + (size_t)q * hs + (u & 1) : nullptr;
        },
        a);
    double bn = -1.0;
    int bj = INT32_MAX;
#pragma unroll
    for (int u = 0; u < UH; ++u)
        if ((int)threadIdx.x + NT * u < a.nh) take(hv[2 * u], hv[2 * u + 1], bn, bj);
    wave_argmax(bn, bj);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        s_vn[w] = bn;
        s_vj[w] = bj;
    }
    __syncthreads();
    wnu = (lane < NW) ? s_vn[lane] : -1.0;
    wj = (lane < NW) ? s_vj[lane] : INT32_MAX;
    wave_argmax_lo<NW>(wnu, wj);
}

// Vote and winner column in one wave (speculative slots, nh <= 64 HPL headers):
// lane q polls headers q + 64 h (h < HPL); every poll round also (re)loads
// the rows of the column of the best candidate seen so far, so when the last header arrives
// the winner's column is usually complete already (one round trip instead of
// two after the last publication).  Lane holds rows lane + 64 u, u < U.
// Returns with the winner in (wnu, wj) and its rows in xv (0 past l), all
// lanes agreeing; on timeout the flag is raised and the values may be NaN.
template <int U, int HPL>
__device__ __forceinline__ void vote_prefetch(const SelArgs& a, const double* reg, const double* slots,
                                              int cols_per_blk, int l, double& wnu, int& wj, uint64_t (&xv)[U]) {
    const int lane = threadIdx.x & 63;
    bool mine[HPL], have[HPL];
    const double* hd[HPL];
    uint64_t hn[HPL], hj[HPL];
#pragma unroll
    for (int h = 0; h < HPL; ++h) {
        const int q = lane + 64 * h;  // headers q = lane + 64 h of this lane
        mine[h] = q < a.nh;
        hd[h] = reg + 2 * (mine[h] ? q : 0);
        have[h] = !mine[h];
        hn[h] = hj[h] = 0;
    }
    int cand = -1;
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = MB_SENT;
    for (uint32_t spin = 0;; ++spin) {
        if (spin) __builtin_amdgcn_s_sleep(1);  // about 64 clocks between polls
#pragma unroll
        for (int h = 0; h < HPL; ++h)
            if (!have[h]) {
                hn[h] = mb_load(hd[h]);
                hj[h] = mb_load(hd[h] + 1);
            }
        if (cand >= 0) {
            const double* col = slots + (size_t)(cand / cols_per_blk) * a.S;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                if (xv[u] == MB_SENT) xv[u] = (i < l) ? mb_load(col + i) : 0ull;
            }
        }
        bool missing = false;
#pragma unroll
        for (int h = 0; h < HPL; ++h) {
            if (!have[h]) have[h] = (hn[h] != MB_SENT) && (hj[h] != MB_SENT);
            missing = missing || !have[h];
        }
        bool col_pend = false;
#pragma unroll
        for (int u = 0; u < U; ++u) col_pend = col_pend || (xv[u] == MB_SENT);
        const bool col_ok = cand >= 0 && !__any(col_pend);
        double bn = -1.0;
        int bj = INT32_MAX;
#pragma unroll
        for (int h = 0; h < HPL; ++h)
            if (mine[h] && have[h]) take(hn[h], hj[h], bn, bj);
        wave_argmax(bn, bj);
        const bool all = !__any(missing);
        if (all && (bj == INT32_MAX || (bj == cand && col_ok))) {
            wnu = bn;
            wj = bj;
            return;
        }
        if (bj != INT32_MAX && bj != cand) {
            cand = bj;
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = MB_SENT;
        }
        if (spin >= a.spin_limit ||
            ((spin & 63) == 63 && __hip_atomic_load(a.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            if (lane == 0) __hip_atomic_store(a.flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            wnu = bn;
            wj = bj;
            return;
        }
    }
}

// l published values at src -> LDS dst, zeros up to lpad (all threads), then a
// workgroup barrier.  Row i is stored at i + (i >> PSH): one pad slot per
// 2^PSH rows, so lane parts that read rows 2^PSH apart hit different banks.
template <int NT, int PSH, bool SLEEP>
__device__ __forceinline__ void fetch_col_lds(const SelArgs& a, const double* src, int l, int lpad, double* dst) {
    for (int i = l + (int)threadIdx.x; i < lpad; i += NT) dst[i + (i >> PSH)] = 0.0;
    for (int i0 = 0; i0 < l; i0 += NT * 8) {
        uint64_t v[8];
        mb_read<8, SLEEP>(
            v,
            [&](int u) -> const double* {
                const int i = i0 + u * NT + (int)threadIdx.x;
                return i < l ? src + i : nullptr;
            },
            a);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * NT + (int)threadIdx.x;
            if (i < l) dst[i + (i >> PSH)] = mb_val(v[u]);
        }
    }
    __syncthreads();
}

// Householder scalars of the winner x (rows t..l-1) from alpha = x_t and the
// published trailing norm nu2 = sum_{i>=t} x_i^2; v_i = x_i * scal below t.
__device__ __forceinline__ void reflector(double alpha, double nu2, double& tau, double& beta, double& scal) {
    if (!(nu2 > alpha * alpha)) {
        tau = 0.0;
        beta = alpha;
        scal = 0.0;
    } else {
        const double nrm = sqrt(nu2);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
    }
}

// A column whose initial norm is not finite (NaN or infinite entries, or a
// sum of squares that overflows) raises flag[1].  The store is complete before
// the workgroup barrier that precedes this workgroup's first publication, and
// workgroup 0 has read every first publication before it reaches finish(), so
// it sees the flag there.
__device__ __forceinline__ void flag_nonfinite(const SelArgs& a) {
    __hip_atomic_store(a.flag + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
}

// k_eff, unused J entries and the status word, written once by workgroup 0
__device__ __forceinline__ void finish(const SelArgs& a, int keff) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const bool timed_out = __hip_atomic_load(a.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        const bool nonfinite = __hip_atomic_load(a.flag + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
        *a.keff = timed_out ? -1 : keff;
        for (int64_t t = keff; t < a.k; ++t) a.J[t] = -1;
        if (a.status)
            *a.status = timed_out ? IDS_ETIMEOUT : nonfinite ? IDS_ENONFINITE : (keff < a.k ? IDS_ERANKDEF : IDS_OK);
    }
}

// ---------------------------------------------------------------------------
// Short sketches (l <= 256), grouped-lane layout: column c of a wave lives in
// the G consecutive lanes G*c .. G*c+G-1; lane part p holds rows
// [p*R, p*R + R).  Column sums are G-lane DPP trees (quad_perm, half-mirror,
// mirror: every lane of the group ends with the same bits); updates are
// branch-free.  The workgroup's best column is published once per step; the
// LDS buffers alternate with the step parity, so a step has three workgroup
// barriers (best, vote, winner column).
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    if (G >= 2) v += dpp_f64<0xB1, 0xf>(v);   // lanes i, i^1
    if (G >= 4) v += dpp_f64<0x4E, 0xf>(v);   // lanes i, i^2
    if (G >= 8) v += dpp_f64<0x141, 0xf>(v);  // half-row mirror (8 lanes)
    if (G >= 16) v += dpp_f64<0x140, 0xf>(v); // row mirror (16 lanes)
    return v;
}

template <int G, int R, int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void cpqr_gl_kernel(SelArgs a) {
    extern __shared__ double sm[];  // two winner-column buffers (step parity)
    __shared__ double s_nu[2][NW];
    __shared__ int s_j[2][NW];
    __shared__ double s_vn[2][NW];
    __shared__ int s_vj[2][NW];
    constexpr int NT = NW * 64;
    constexpr int CPWV = 64 / G;  // columns per wave

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int p = lane % G;       // row part
    const int j = (blockIdx.x * NW + w) * CPWV + lane / G;
    const int n = (int)a.n, l = (int)a.l;
    const int S = a.S;
    const int row0 = p * R;
    constexpr int LP = G * R;     // rows covered (>= l)
    constexpr int PSH = ilog2(R); // LDS row padding (R is a power of two)
    static_assert((1 << PSH) == R, "rows per lane must be a power of two");
    constexpr int LB = LP + LP / R;  // doubles per LDS buffer

    double y[R];
    bool alive = j < n;
    int tsel = -1;  // step at which this column was chosen
    {
        // every lane loads all R rows (addresses clamped into Y), then masks:
        // the barrier keeps the compiler from turning the mask into a branch
        // around each load, which would serialise the loads
        const int64_t jc = min(j, n - 1);
        if (a.ydt == IDS_F64) {
            const double* Yp = (const double*)a.Y;
#pragma unroll
            for (int r = 0; r < R; ++r) y[r] = Yp[(int64_t)min(row0 + r, l - 1) * a.rs + jc * a.cs];
        } else {
            const float* Yp = (const float*)a.Y;
#pragma unroll
            for (int r = 0; r < R; ++r) y[r] = (double)Yp[(int64_t)min(row0 + r, l - 1) * a.rs + jc * a.cs];
        }
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = (alive && row0 + r < l) ? y[r] : 0.0;
    }
    if (alive && p == 0) a.pos[j] = -1;
    double nu;
    {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) s = fma(y[r], y[r], s);
        nu = group_sum<G>(s);
    }
    if (alive && !__builtin_isfinite(nu)) flag_nonfinite(a);

    const int k = (int)a.k;
    int keff = k;
    for (int t = 0; t < k; ++t) {
        const int par = t & 1;
        double* reg = a.mb + (size_t)t * a.RS;
        // ---- workgroup best (every wave computes it), published once
        {
            double wn = alive ? nu : -1.0;
            int wjw = alive ? j : INT32_MAX;
            wave_argmax<ilog2(G)>(wn, wjw);  // the G lanes of a column agree
            if (lane == 0) {
                s_nu[par][w] = wn;
                s_j[par][w] = wjw;
            }
        }
        // the previous step's sentinel stores into this step's column slot are
        // complete (globally visible) before the barrier, hence before this
        // workgroup's header and column of this step
        if (MODE == MB_SPEC) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        double bn = (lane < NW) ? s_nu[par][lane] : -1.0;
        int bj = (lane < NW) ? s_j[par][lane] : INT32_MAX;
        wave_argmax_lo<NW>(bn, bj);
        double* hd = reg + 2 * blockIdx.x;
        double* slots = (MODE == MB_SPEC) ? spec_slots(a, t) : nullptr;
        double* sc = slots + (size_t)blockIdx.x * S;  // MB_SPEC: this workgroup's column slot
        if (threadIdx.x == 0) {
            mb_put(hd, bn);
            mb_put(hd + 1, idx_bits(bj == INT32_MAX ? -1 : bj));
        }
        const bool one_wave_vote = MODE == MB_SPEC && a.nh <= 256;  // uniform
        if (MODE == MB_SPEC && j == bj) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (row0 + r < l) mb_put(sc + row0 + r, y[r]);
        }
        // ---- vote, winner column -> LDS
        double wnu;
        int wj;
        double* xb = sm + par * LB;
        if (one_wave_vote) {
            constexpr int UP = (LP + 63) / 64;
            if (w == 0) {
                uint64_t xv[UP];
                double vn;
                int vj;
                if (a.nh <= 64)
                    vote_prefetch<UP, 1>(a, reg, slots, NW * CPWV, l, vn, vj, xv);
                else
                    vote_prefetch<UP, 4>(a, reg, slots, NW * CPWV, l, vn, vj, xv);
#pragma unroll
                for (int u = 0; u < UP; ++u) {
                    const int i = lane + 64 * u;
                    if (i < LP) xb[i + (i >> PSH)] = mb_val(xv[u]);
                }
                if (lane == 0) {
                    s_vn[par][0] = vn;
                    s_vj[par][0] = vj;
                }
            }
            __syncthreads();
            wnu = s_vn[par][0];
            wj = s_vj[par][0];
        } else {
            vote_hdr<NW, MODE == MB_SPEC>(a, reg, 2, s_vn[par], s_vj[par], wnu, wj);
        }
        if (wj == INT32_MAX || !(wnu > 0.0)) {
            keff = t;
            break;
        }
        if (MODE == MB_SPEC && t >= 1 && t + 1 < k) {
            // every workgroup has published step t, so none still reads the
            // column slots of step t - 1: this workgroup's slot there is
            // reset for step t + 1 (same slot set)
            double* nsc = spec_slots(a, t + 1) + (size_t)blockIdx.x * S;
            for (int i = threadIdx.x; i < l; i += NT) mb_clear(nsc + i);
        }
        if (one_wave_vote) {
            // the winner's rows are in LDS already
        } else if (MODE == MB_SPEC) {
            fetch_col_lds<NT, PSH, true>(a, slots + (size_t)(wj / (NW * CPWV)) * S, l, LP, xb);
        } else {
            double* cb = reg + a.H0;
            if (j == wj) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (row0 + r < l) mb_put(cb + row0 + r, y[r]);
            }
            fetch_col_lds<NT, PSH, false>(a, cb, l, LP, xb);
        }
        // ---- Householder reflector (every wave, same bits)
        double tau, beta, scal;
        reflector(xb[t + (t >> PSH)], wnu, tau, beta, scal);
        // reflector entry of row row0 + r: 0 above t, 1 at t, x_i scal below
        // (rows >= l read the LDS zero padding).  Short lane parts keep v in
        // registers; long ones re-read it from LDS in the update.
        auto vof = [&](int r) -> double {
            const int i = row0 + r;
            const double xi = xb[i + (i >> PSH)];
            return (i < t) ? 0.0 : (i == t ? 1.0 : xi * scal);
        };
        constexpr bool VREG = R <= 16;
        double v[VREG ? R : 1];
        if (VREG) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[VREG ? r : 0] = vof(r);
        }
        // ---- apply H (branch-free: dead columns get a zero multiplier)
        double d0 = 0.0, d1 = 0.0;
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            d0 = fma(VREG ? v[VREG ? r : 0] : vof(r), y[r], d0);
            if (r + 1 < R) d1 = fma(VREG ? v[VREG ? r + 1 : 0] : vof(r + 1), y[r + 1], d1);
        }
        const double d = group_sum<G>(d0 + d1);
        const double dt = alive ? d * tau : 0.0;
        if (!VREG) asm volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < R; ++r) y[r] = fma(-dt, VREG ? v[VREG ? r : 0] : vof(r), y[r]);
        if (j == wj) {
            alive = false;
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (row0 + r == t) y[r] = beta;
            if (p == 0) a.pos[j] = t;
            tsel = t;
        }
        // ---- trailing norms for the next step (rows > t)
        {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int r = 0; r < R; r += 2) {
                const double y0 = (row0 + r > t) ? y[r] : 0.0;
                s0 = fma(y0, y0, s0);
                if (r + 1 < R) {
                    const double y1 = (row0 + r + 1 > t) ? y[r + 1] : 0.0;
                    s1 = fma(y1, y1, s1);
                }
            }
            nu = group_sum<G>(s0 + s1);
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) a.J[t] = wj;
        // no barrier here: the LDS buffers alternate with the step parity
    }

    if (j < n) {
        double* rj = (tsel >= 0) ? a.R11c + (int64_t)tsel * a.k : nullptr;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = row0 + r;
            if (i < keff) {
                a.Rt[(int64_t)j * a.k + i] = y[r];
                if (rj) rj[i] = y[r];
            }
        }
    }
    finish(a, keff);
}

// ---------------------------------------------------------------------------
// Long sketches (256 < l <= 4096), row-band layout: a workgroup of 8 waves
// owns NC columns; wave w holds rows [64 RB w, 64 RB (w + 1)) of all of them,
// row 64 RB w + 64 r + lane in y[c][r].  Each wave reads only its rows of the
// winner's column, straight into registers.  With
// v^T y_c = y_c[t] + scal * sum_{i>t} x_i y_ci, one workgroup reduction gives
// all NC dot products, a second the new trailing norms.
// ---------------------------------------------------------------------------
// Sums over the workgroup of M per-lane values: the partials go to LDS
// (red[w][m][lane]), wave m mod NW adds entry m over the waves and then over
// its lanes, and every thread reads the M totals back.  The order is fixed,
// so every workgroup gets the same bits for the same data.
template <int M, int NW>
__device__ __forceinline__ void wg_sum_t(double (&v)[M], double* red, double* res) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int m = 0; m < M; ++m) red[(w * M + m) * 64 + lane] = v[m];
    __syncthreads();
#pragma unroll
    for (int mm = 0; mm < (M + NW - 1) / NW; ++mm) {
        const int m = w + NW * mm;
        if (m < M) {
            double s = red[m * 64 + lane];
#pragma unroll
            for (int q = 1; q < NW; ++q) s += red[(q * M + m) * 64 + lane];
            s = wave_sum_dpp1(s);
            if (lane == 0) res[m] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m) v[m] = res[m];
}

template <int NC, int RB>
__device__ __forceinline__ double ysel(const double (&y)[NC][RB], int c, int r) {
    double v = 0.0;
#pragma unroll
    for (int cc = 0; cc < NC; ++cc)
        if (cc == c) v = y[cc][r];
    return v;
}

constexpr int RB_NW = 8;
template <int NC>
constexpr size_t rb_lds_bytes() { return sizeof(double) * RB_NW * NC * 64; }

template <int NC, int RB, int MODE>
__global__ __launch_bounds__(512) void cpqr_rb_kernel(SelArgs a) {
    constexpr int NW = RB_NW;
    constexpr int BAND = 64 * RB;  // rows per wave
    extern __shared__ double red[];  // NW x NC x 64 partial sums
    __shared__ double res[NC];
    __shared__ double s_vn[2][NW];
    __shared__ int s_vj[2][NW];
    __shared__ double s_row[NC + 1];  // row t: y_c[t] (c < NC) and x_t (NC)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col0 = blockIdx.x * NC;
    const int n = (int)a.n, l = (int)a.l;
    const int rb0 = BAND * w + lane;  // row of y[c][r] is rb0 + 64 r

    double y[NC][RB];
    bool alive[NC];
    int tsel[NC];  // step at which column c was chosen (uniform)
    // every load is issued before any value is used (FP32 data waits in the
    // low word of y until then), so the loads overlap
    const bool f64 = a.ydt == IDS_F64;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        alive[c] = col0 + c < n;
        tsel[c] = -1;
    }
    if (f64) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int r = 0; r < RB; ++r)
                y[c][r] = ((const double*)a.Y)[(int64_t)min(rb0 + 64 * r, l - 1) * a.rs +
                                               (int64_t)min(col0 + c, n - 1) * a.cs];
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int r = 0; r < RB; ++r)
                y[c][r] = __hiloint2double(0, __float_as_int(((const float*)a.Y)[(int64_t)min(rb0 + 64 * r, l - 1) * a.rs +
                                                                                 (int64_t)min(col0 + c, n - 1) * a.cs]));
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const double v = f64 ? y[c][r] : (double)__int_as_float(__double2loint(y[c][r]));
            y[c][r] = (alive[c] && rb0 + 64 * r < l) ? v : 0.0;
        }
    if (w == 0 && lane < NC && col0 + lane < n) a.pos[col0 + lane] = -1;
    double nu[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < RB; ++r) s = fma(y[c][r], y[c][r], s);
        nu[c] = s;
    }
    wg_sum_t<NC, NW>(nu, red, res);
    if (threadIdx.x == 0) {
        bool bad = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) bad = bad || (alive[c] && !__builtin_isfinite(nu[c]));
        if (bad) flag_nonfinite(a);
    }

    const int k = (int)a.k;
    int keff = k;
    for (int t = 0; t < k; ++t) {
        const int par = t & 1;
        double* reg = a.mb + (size_t)t * a.RS;
        // ---- workgroup best (nu is identical in every thread)
        double bn = -1.0;
        int bc = -1;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (alive[c] && nu[c] > bn) {
                bn = nu[c];
                bc = c;
            }
        double* hd = reg + 2 * blockIdx.x;
        double* slots = (MODE == MB_SPEC) ? spec_slots(a, t) : nullptr;
        double* sc = slots + (size_t)blockIdx.x * a.S;  // MB_SPEC: this workgroup's column slot
        if (threadIdx.x == 0) {
            mb_put(hd, bn);
            mb_put(hd + 1, idx_bits(bc >= 0 ? col0 + bc : -1));
        }
        if (MODE == MB_SPEC && bc >= 0) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = rb0 + 64 * r;
                if (i < l) mb_put(sc + i, ysel(y, bc, r));
            }
        }
        double wnu;
        int wj;
        vote_hdr<NW, MODE == MB_SPEC>(a, reg, 2, s_vn[par], s_vj[par], wnu, wj);
        if (wj == INT32_MAX || !(wnu > 0.0)) {
            keff = t;
            break;
        }
        const int wblk = wj / NC;
        const double* src;
        if (MODE == MB_OWNER) {
            double* cb = reg + a.H0;
            if (wblk == (int)blockIdx.x) {
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int i = rb0 + 64 * r;
                    if (i < l) mb_put(cb + i, ysel(y, wj - col0, r));
                }
            }
            src = cb;
        } else {
            src = slots + (size_t)wblk * a.S;
        }
        double x[RB];
        {
            uint64_t xv[RB];
            mb_read<RB, MODE == MB_SPEC>(
                xv,
                [&](int r) -> const double* {
                    const int i = rb0 + 64 * r;
                    return i < l ? src + i : nullptr;
                },
                a);
#pragma unroll
            for (int r = 0; r < RB; ++r) x[r] = (rb0 + 64 * r < l) ? mb_val(xv[r]) : 0.0;
        }
        if (MODE == MB_SPEC && t >= 1 && t + 1 < k) {
            // every workgroup has published step t, so none still reads the
            // column slots of step t - 1: this workgroup's slot there is reset
            // for step t + 1 (each thread its own rows, as it writes them)
            double* nsc = spec_slots(a, t + 1) + (size_t)blockIdx.x * a.S;
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (rb0 + 64 * r < l) mb_clear(nsc + rb0 + 64 * r);
        }
        // ---- dot products with the rows below t
        double pa[NC];
        {
            double xm[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) xm[r] = (rb0 + 64 * r > t) ? x[r] : 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double s = 0.0;
#pragma unroll
                for (int r = 0; r < RB; ++r) s = fma(xm[r], y[c][r], s);
                pa[c] = s;
            }
        }
        if (w == t / BAND && lane == (t & 63)) {
            const int rt = (t % BAND) >> 6;
#pragma unroll
            for (int r = 0; r < RB; ++r)
                if (r == rt) {
                    s_row[NC] = x[r];
#pragma unroll
                    for (int c = 0; c < NC; ++c) s_row[c] = y[c][r];
                }
        }
        wg_sum_t<NC, NW>(pa, red, res);
        double tau, beta, scal;
        reflector(s_row[NC], wnu, tau, beta, scal);
        // ---- apply H to the live columns (dead ones get a zero multiplier)
        {
            double v[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int i = rb0 + 64 * r;
                v[r] = (i < t) ? 0.0 : (i == t ? 1.0 : x[r] * scal);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double dt = alive[c] ? (s_row[c] + scal * pa[c]) * tau : 0.0;
#pragma unroll
                for (int r = 0; r < RB; ++r) y[c][r] = fma(-dt, v[r], y[c][r]);
            }
        }
        if (wblk == (int)blockIdx.x) {
            const int cw = wj - col0;
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if (c == cw) {
                    alive[c] = false;
                    tsel[c] = t;
#pragma unroll
                    for (int r = 0; r < RB; ++r)
                        if (rb0 + 64 * r == t) y[c][r] = beta;
                }
            if (threadIdx.x == 0) a.pos[wj] = t;
        }
        // ---- trailing norms for the next step (rows > t)
        {
            double msk[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) msk[r] = (rb0 + 64 * r > t) ? 1.0 : 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                double s = 0.0;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const double q = y[c][r] * msk[r];
                    s = fma(q, q, s);
                }
                nu[c] = s;
            }
        }
        // the sentinel stores are complete (globally visible) before the
        // barriers below, hence before the next step's header
        if (MODE == MB_SPEC) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        wg_sum_t<NC, NW>(nu, red, res);
        if (blockIdx.x == 0 && threadIdx.x == 0) a.J[t] = wj;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if (col0 + c >= n) continue;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int i = rb0 + 64 * r;
            if (i < keff) {
                a.Rt[(int64_t)(col0 + c) * a.k + i] = y[c][r];
                if (tsel[c] >= 0) a.R11c[(int64_t)tsel[c] * a.k + i] = y[c][r];
            }
        }
    }
    finish(a, keff);
}

// R11 (keff x keff, row-major, zero below the diagonal) into LDS from the
// compact copy R11c (row t = top rows of the column chosen at step t, so
// R11[r][c] = R11c[c][r]).
__device__ __forceinline__ void stage_r11(double* R11s, const double* __restrict__ R11c, int64_t k, int keff,
                                          int nthreads) {
    copy_batched<16>(
        keff * keff, nthreads,
        [&](int e) {
            const int r = e / keff, c = e - r * keff;
            return R11c[(int64_t)c * k + r];
        },
        [&](int e, double v) {
            const int r = e / keff, c = e - r * keff;
            R11s[e] = (r <= c) ? v : 0.0;
        });
}

// Faster variant for k <= 16*KS with R11 in LDS: a group of 16 lanes solves one column.  Lane q
// of the group keeps x_c and b_c for c = 16*s + q in register slot s; at step r
// every lane forms its part of b_r - sum_{c>r} R11[r][c] x_c, the 16 parts are
// summed with DPP row operations, and x_r = (that sum) / R11[r][r].
template <int KS>
__global__ __launch_bounds__(256) void trsm_group_kernel(int64_t n, int64_t k, const double* __restrict__ Rt,
                                                         const double* __restrict__ R11c,
                                                         const int32_t* __restrict__ pos,
                                                         const int64_t* __restrict__ keffp, double* P) {
    extern __shared__ double R11s[];
    const int64_t keff = *keffp;
    if (keff < 0) return;
    stage_r11(R11s, R11c, k, (int)keff, 256);
    __syncthreads();
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
        // the row's reads issued together from clamped addresses (a read
        // behind the c > r test is compiled as a branch and a wait each)
        double rv[KS];
#pragma unroll
        for (int sl = 0; sl < KS; ++sl) rv[sl] = R11s[r * keff + min<int64_t>(16 * sl + q, keff - 1)];
        asm volatile("" ::: "memory");
        double part = 0.0;
#pragma unroll
        for (int sl = 0; sl < KS; ++sl) {
            const int64_t c = 16 * sl + q;
            const double f = fma(-rv[sl], x[sl], part);
            part = (c == r) ? b[sl] : ((c > r && c < keff) ? f : part);
        }
        part += dpp_f64<0xB1, 0xf>(part);
        part += dpp_f64<0x4E, 0xf>(part);
        part += dpp_f64<0x141, 0xf>(part);
        part += dpp_f64<0x140, 0xf>(part);
        const double d = R11s[r * keff + r];
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

// The same solve where R11 does not fit in LDS (k up to 16*KS): R11 is read
// from memory TRSM_TC steps at a time.  The workgroup (16 columns) stages the
// entries R11[r][c] of a block of TRSM_TC consecutive steps into LDS
// cooperatively (contiguous reads along r of the column-major R11), and the
// next block's loads are in flight while the current block's steps run, so a
// step waits on LDS instead of an L2 round trip.  A column's right-hand side
// and solution live in LDS too (x_c = 0 until solved), so a step is plain
// FMAs over all slots with no per-slot selects: each lane keeps four partial
// sums, the 16 lanes are summed with DPP, x_r = (b_r + sum) / R11[r][r] (the
// reciprocals of a block's diagonal formed at staging) and one lane stores
// x_r for the column's later steps.  One wave per SIMD is all this solve has
// (16 lanes per column), so instructions per step set its pace.
constexpr int TRSM_TC = 16;
template <int KS>
__global__ __launch_bounds__(256) void trsm_chunk_kernel(int64_t n, int64_t k, const double* __restrict__ Rt,
                                                         const double* __restrict__ R11c,
                                                         const int32_t* __restrict__ pos,
                                                         const int64_t* __restrict__ keffp, double* P) {
    constexpr int KP = 16 * KS;                       // staged entries per step
    constexpr int PER = (TRSM_TC * KP + 255) / 256;   // staged doubles per thread per block
    static_assert(TRSM_TC * KP % 256 == 0, "whole blocks per thread");
    __shared__ double stg[2][TRSM_TC * KP];           // [buffer][rr * KP + c] = R11[r1 - rr][c]
    __shared__ double rdg[2][TRSM_TC];                // [buffer][rr] = 1 / R11[r1 - rr][r1 - rr]
    __shared__ double xs[16][KP];                     // [column][c] = x_c, 0 until solved
    __shared__ double bs[16][KP];                     // [column][c] = b_c
    const int64_t keff64 = *keffp;
    if (keff64 < 0) return;  // the same for the whole workgroup
    const int keff = (int)keff64;
    const int tid = threadIdx.x, q = tid & 15, col = tid >> 4;
    const int64_t j = (int64_t)blockIdx.x * 16 + (tid >> 4);
    const bool inb = j < n;
    const int32_t pj = inb ? pos[j] : 0;
    const bool solve = inb && pj < 0;  // other lanes only help with the staging
    if (inb && pj >= 0)
        for (int64_t r = q; r < k; r += 16) P[r * n + j] = (r == pj) ? 1.0 : 0.0;
    {
        // loads from clamped addresses, all in flight together, then masked;
        // a column's b and x are used by its own 16 lanes only (one wave)
        const int64_t jr = (inb ? j : 0) * k;
        double bv[KS];
#pragma unroll
        for (int sl = 0; sl < KS; ++sl) bv[sl] = Rt[jr + min(16 * sl + q, max(keff - 1, 0))];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int sl = 0; sl < KS; ++sl) {
            const int c = 16 * sl + q;
            bs[col][c] = (solve && c < keff) ? bv[sl] : 0.0;
            xs[col][c] = 0.0;
        }
    }
    // block i holds steps r = r1 - rr, rr < TRSM_TC, r1 = keff - 1 - i TRSM_TC;
    // element e of a block: c = e / TRSM_TC, rr = e % TRSM_TC
    const int nblk = (keff + TRSM_TC - 1) / TRSM_TC;
    double v[PER], dg = 1.0;  // dg: thread rr < TRSM_TC also loads R11[r1 - rr][r1 - rr]
    auto load = [&](int i) {
        const int r1 = keff - 1 - i * TRSM_TC;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u, c = e / TRSM_TC, r = r1 - e % TRSM_TC;
            const bool ok = c < keff && r >= 0;
            v[u] = R11c[ok ? (int64_t)c * k + r : 0];
        }
        const int rd = r1 - tid;
        dg = R11c[(tid < TRSM_TC && rd >= 0) ? (int64_t)rd * (k + 1) : 0];
        asm volatile("" ::: "memory");
    };
    auto store = [&](int i) {
        double* S = stg[i & 1];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u, c = e / TRSM_TC, rr = e % TRSM_TC;
            S[rr * KP + c] = v[u];
        }
        if (tid < TRSM_TC) rdg[i & 1][tid] = 1.0 / dg;
    };
    load(0);
    store(0);
    __syncthreads();
    for (int i = 0; i < nblk; ++i) {
        if (i + 1 < nblk) load(i + 1);
        const double* S = stg[i & 1];
        const int r1 = keff - 1 - i * TRSM_TC;
        for (int rr = 0; rr < TRSM_TC; ++rr) {
            const int r = r1 - rr;
            if (r < 0) break;
            const double* row = S + rr * KP;  // row[c] = R11[r][c]
            const double* xc = xs[col];
            // all reads issued together, then the FMAs (unsolved x_c are 0)
            double rv[KS], xv[KS];
#pragma unroll
            for (int sl = 0; sl < KS; ++sl) {
                rv[sl] = row[16 * sl + q];
                xv[sl] = xc[16 * sl + q];
            }
            asm volatile("" ::: "memory");
            double ps[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int sl = 0; sl < KS; ++sl) ps[sl & 3] = fma(-rv[sl], xv[sl], ps[sl & 3]);
            double part = (ps[0] + ps[1]) + (ps[2] + ps[3]);
            part += dpp_f64<0xB1, 0xf>(part);
            part += dpp_f64<0x4E, 0xf>(part);
            part += dpp_f64<0x141, 0xf>(part);
            part += dpp_f64<0x140, 0xf>(part);
            const double xr = (bs[col][r] + part) * rdg[i & 1][rr];
            if (q == 0) {
                xs[col][r] = xr;
                if (solve) P[(int64_t)r * n + j] = xr;
            }
        }
        if (i + 1 < nblk) store(i + 1);
        __syncthreads();
    }
    if (solve)
        for (int64_t r = keff + q; r < k; r += 16) P[r * n + j] = 0.0;
}

// k <= 128: the axpy back-substitution, GQ = 1, 2, 4 lanes per column
template <int GQ>
__global__ __launch_bounds__(256) void trsm_axpy_kernel(int64_t n, int64_t k, const double* __restrict__ Rt,
                                                        const double* __restrict__ R11c,
                                                        const int32_t* __restrict__ pos,
                                                        const int64_t* __restrict__ keffp, double* P) {
    constexpr int KS = TRSM_AX_KS, LDK = trsm_ax_ldk<GQ>();
    extern __shared__ __attribute__((aligned(16))) double sm[];
    const int64_t keff64 = *keffp;
    if (keff64 < 0) return;
    const int keff = (int)keff64;
    double* R11T = sm;                    // keff x LDK
    double* rd = sm + (size_t)keff * LDK;  // keff reciprocal diagonals
    const int tid = threadIdx.x, lane = tid & 63;
    stage_r11t<GQ, 4>(R11T, keff, (int)k, 256, [&](int r, int c) { return R11c[(int64_t)r * k + c]; });
    copy_batched<1>(
        keff, 256, [&](int r) { return R11c[(int64_t)r * k + r]; }, [&](int r, double v) { rd[r] = 1.0 / v; });
    __syncthreads();
    const int q = lane % GQ;
    const int64_t j = (int64_t)blockIdx.x * (256 / GQ) + tid / GQ;
    if (j >= n) return;
    const int32_t pj = pos[j];
    if (pj >= 0) {
        for (int64_t c = q; c < k; c += GQ) P[c * n + j] = (c == pj) ? 1.0 : 0.0;
        return;
    }
    double b[KS];
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) {
        const int c = GQ * sl + q;
        b[sl] = (c < keff) ? Rt[j * k + c] : 0.0;
    }
    axpy_solve<GQ>(b, R11T, rd, keff, q);
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) {
        const int c = GQ * sl + q;
        if (c < k) P[(int64_t)c * n + j] = (c < keff) ? b[sl] : 0.0;
    }
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
    int cols;           // columns per workgroup
    int pubs;           // candidate publishers per workgroup
    int threads;        // threads per workgroup
    bool gl;            // grouped-lane kernel (winner column staged in LDS)
    int rows;           // grouped lanes: rows covered (G * R)
    int lane_rows;      // grouped lanes: rows per lane (R)
    size_t lds_fixed;   // dynamic LDS of a row-band kernel
    const void* fn[2];  // per mailbox mode
};

template <int G, int R, int NW>
static Inst inst_gl() {
    return {NW * (64 / G), 1, NW * 64, true, G * R, R, 0,
            {(const void*)&cpqr_gl_kernel<G, R, NW, MB_SPEC>, (const void*)&cpqr_gl_kernel<G, R, NW, MB_OWNER>}};
}
template <int NC, int RB>
static Inst inst_rb() {
    return {NC, 1, 64 * RB_NW, false, 0, 1, rb_lds_bytes<NC>(),
            {(const void*)&cpqr_rb_kernel<NC, RB, MB_SPEC>, (const void*)&cpqr_rb_kernel<NC, RB, MB_OWNER>}};
}

// kernel instance for l rows; variant 1 (a tuned knob) takes 4-wave
// workgroups instead of 8 for the grouped-lane kernels (twice the
// publishers, half the threads per vote)
static bool pick(int64_t l, int variant, Inst& in) {
    // grouped-lane kernels for short sketches, row bands beyond 256 rows
    if (l <= 32) in = variant ? inst_gl<2, 16, 4>() : inst_gl<2, 16, 8>();
    else if (l <= 64) in = variant ? inst_gl<4, 16, 4>() : inst_gl<4, 16, 8>();
    else if (l <= 128) in = variant ? inst_gl<8, 16, 4>() : inst_gl<8, 16, 8>();
    else if (l <= 256) in = variant ? inst_gl<16, 16, 4>() : inst_gl<16, 16, 8>();
    else if (l <= 512) in = inst_rb<16, 1>();
    else if (l <= 1024) in = inst_rb<16, 2>();
    else if (l <= 2048) in = inst_rb<8, 4>();
    else if (l <= 4096) in = inst_rb<8, 8>();
    else return false;
    return true;
}

static int gl_variant(int64_t l, int64_t n) {
    if (l > 256) return 0;
    const char* lb = l <= 32 ? "l32" : l <= 64 ? "l64" : l <= 128 ? "l128" : "l256";
    return (int)tune_get(std::string("select.gl.") + lb + "." + n_bucket(n), 0);
}

static int64_t round32(int64_t x) { return (x + 31) / 32 * 32; }
constexpr int SPEC_PUBS_MAX = 256;            // candidate columns stored per step
constexpr size_t SPEC_RING_MAX = 64u << 20;   // the two sets of column slots

// mailbox mode and geometry (sp.l, sp.k, sp.nh set)
static void mb_layout(SelectPlan& sp) {
    // headers packed at the start of each step region (one or a few cache
    // lines for the vote to poll), column slots after them
    sp.H0 = (int)round32(2 * (int64_t)sp.nh);
    sp.S = (int)round32(sp.l);
    const size_t ring = 2 * sizeof(double) * (size_t)sp.S * sp.nh;  // two sets of column slots
    sp.mode = (sp.nh <= SPEC_PUBS_MAX && ring <= SPEC_RING_MAX) ? MB_SPEC : MB_OWNER;
    sp.RS = (sp.mode == MB_OWNER) ? sp.H0 + round32(sp.l) : sp.H0;
    sp.CS = (sp.mode == MB_OWNER) ? 0 : (int64_t)sp.S * sp.nh;
}

static size_t cpqr_lds(const SelectPlan& sp, const Inst& in) {
    return in.gl ? 2 * sizeof(double) * (size_t)(in.rows + in.rows / in.lane_rows) : in.lds_fixed;
}

// the plan for one kernel variant; IDS_EINVAL if its workgroups cannot all be
// co-resident for this n
static ids_status select_plan_variant(int64_t l, int64_t n, int64_t k, int variant, SelectPlan& sp);

// the column-steps plan (columns in HBM, one kernel per pivot step)
static ids_status steps_plan(int64_t l, int64_t n, int64_t k, SelectPlan& sp) {
    if (l > 4096) {
        set_error("id_select: l must be <= 4096");
        return IDS_EINVAL;
    }
    sp = SelectPlan{};
    sp.l = l;
    sp.n = n;
    sp.k = k;
    sp.steps = 1;
    set_error("");
    return IDS_OK;
}

ids_status select_plan(int64_t l, int64_t n, int64_t k, SelectPlan& sp) {
    if (tune_get("select.steps", 0)) return steps_plan(l, n, k, sp);
    // the tuned variant; a grouped-lane shape too wide for it takes the other
    // variant if that one holds it (4-wave workgroups are co-resident in
    // larger numbers); a shape too wide for the register-resident
    // factorisation altogether takes the column-steps one
    const int v = gl_variant(l, n);
    ids_status s = select_plan_variant(l, n, k, v, sp);
    if (s == IDS_EINVAL && l <= 256) {
        SelectPlan alt;
        if (select_plan_variant(l, n, k, 1 - v, alt) == IDS_OK) {
            sp = alt;
            set_error("");
            return IDS_OK;
        }
    }
    if (s == IDS_EINVAL && l <= 4096) return steps_plan(l, n, k, sp);
    return s;
}

static ids_status select_plan_variant(int64_t l, int64_t n, int64_t k, int variant, SelectPlan& sp) {
    Inst in;
    sp.steps = 0;
    sp.variant = variant;
    if (!pick(l, sp.variant, in)) {
        set_error("id_select: l must be <= 4096");
        return IDS_EINVAL;
    }
    sp.l = l;
    sp.n = n;
    sp.k = k;
    sp.cols = in.cols;
    sp.threads = in.threads;
    sp.nb = (int)((n + in.cols - 1) / in.cols);
    sp.nh = sp.nb * in.pubs;
    mb_layout(sp);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        set_error("hipGetDevice failed");
        return IDS_EHIP;
    }
    int ncu = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        set_error("hipDeviceGetAttribute failed");
        return IDS_EHIP;
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, in.fn[sp.mode], in.threads, cpqr_lds(sp, in)) !=
        hipSuccess)
        per_cu = 1;
    const int64_t max_nb = std::min<int64_t>((int64_t)ncu * per_cu,
                                             (int64_t)VOTE_PER_THREAD * in.threads / in.pubs);
    if ((int64_t)sp.nb > max_nb) {
        set_error("id_select: n too large for the register-resident CPQR (n = " + std::to_string(n) +
                  ", l = " + std::to_string(l) + ", max columns " + std::to_string(max_nb * in.cols) + ")");
        return IDS_EINVAL;
    }
    return IDS_OK;
}

static size_t mb_doubles(const SelectPlan& sp) { return (size_t)sp.k * sp.RS + 2 * (size_t)sp.CS; }

size_t select_bytes(const SelectPlan& sp) {
    if (sp.steps)
        return steps_bytes(sp.l, sp.n, sp.k, nullptr) + align256(sizeof(double) * (size_t)sp.n * sp.k) +
               align256(sizeof(double) * (size_t)sp.k * sp.k) + align256(sizeof(int32_t) * (size_t)sp.n);
    return align256(sizeof(double) * mb_doubles(sp)) + align256(sizeof(uint32_t) * 2) +
           align256(sizeof(double) * (size_t)sp.n * sp.k) + align256(sizeof(double) * (size_t)sp.k * sp.k) +
           align256(sizeof(int32_t) * (size_t)sp.n);
}

// polls before a device-wide wait gives up (0: the exchange is treated as
// expired from the start -- a host-forced test of the give-up path)
static std::atomic<uint32_t> g_wait_limit{SPIN_LIMIT};

void set_wait_limit(int64_t polls) {
    g_wait_limit.store(polls < 0 ? SPIN_LIMIT : (uint32_t)std::min<int64_t>(polls, SPIN_LIMIT));
}

static ids_status solve_p(const SelectPlan& sp, const double* Rt, const double* R11c, const int32_t* pos,
                          int64_t* keff, double* P, hipStream_t st, bool prof);

ids_status select_run(const SelectPlan& sp, const void* Y, int32_t ydt, int64_t rs, int64_t cs, int64_t* J,
                      double* P, int64_t* keff, int32_t* status, char* ws, hipStream_t st, bool prof) {
    if (sp.steps) {
        char* p = ws + steps_bytes(sp.l, sp.n, sp.k, nullptr);
        double* Rt = (double*)p;
        p += align256(sizeof(double) * (size_t)sp.n * sp.k);
        double* R11c = (double*)p;
        p += align256(sizeof(double) * (size_t)sp.k * sp.k);
        int32_t* pos = (int32_t*)p;
        ids_status s;
        {
            ProfScope ps(prof ? PK_CPQR : -1, st);
            s = steps_factor(Y, ydt, sp.l, sp.n, rs, cs, sp.k, J, keff, status, Rt, R11c, pos, ws, st);
        }
        if (s) return s;
        return solve_p(sp, Rt, R11c, pos, keff, P, st, prof);
    }
    SelArgs a;
    a.status = status;
    a.spin_limit = g_wait_limit.load();
    a.Y = Y;
    a.ydt = ydt;
    a.l = sp.l;
    a.n = sp.n;
    a.rs = rs;
    a.cs = cs;
    a.k = sp.k;
    a.J = J;
    a.keff = keff;
    a.nh = sp.nh;
    a.S = sp.S;
    a.H0 = sp.H0;
    a.RS = sp.RS;
    a.CS = sp.CS;
    char* p = ws;
    a.mb = (double*)p;
    a.ring = a.mb + (size_t)sp.k * sp.RS;
    p += align256(sizeof(double) * mb_doubles(sp));
    a.flag = (uint32_t*)p;
    p += align256(sizeof(uint32_t) * 2);
    a.Rt = (double*)p;
    p += align256(sizeof(double) * (size_t)sp.n * sp.k);
    a.R11c = (double*)p;
    p += align256(sizeof(double) * (size_t)sp.k * sp.k);
    a.pos = (int32_t*)p;

    Inst in;
    pick(sp.l, sp.variant, in);
    const int64_t cnt = (int64_t)mb_doubles(sp);
    const unsigned fg = (unsigned)std::min<int64_t>((cnt + 255) / 256, 4096);
    hipLaunchKernelGGL(mb_fill_kernel, dim3(fg), dim3(256), 0, st, (uint64_t*)a.mb, cnt, a.flag,
                       a.spin_limit == 0 ? 1u : 0u);
    void* args[] = {&a};
    {
        ProfScope ps(prof ? PK_CPQR : -1, st);
        hipError_t e = hipLaunchCooperativeKernel(in.fn[sp.mode], dim3(sp.nb), dim3(in.threads), args,
                                                  (unsigned)cpqr_lds(sp, in), st);
        if (e != hipSuccess) {
            set_error(std::string("cpqr cooperative launch: ") + hipGetErrorString(e));
            return IDS_EHIP;
        }
    }
    return solve_p(sp, a.Rt, a.R11c, a.pos, keff, P, st, prof);
}

// P = [I, R11^{-1} R12] Pi^T from Rt, R11c and the pivot positions
static ids_status solve_p(const SelectPlan& sp, const double* Rt, const double* R11c, const int32_t* pos,
                          int64_t* keff, double* P, hipStream_t st, bool prof) {
    ProfScope ps(prof ? PK_TRSM : -1, st);
    const size_t r11 = sizeof(double) * (size_t)sp.k * sp.k;
    const size_t lim = lds_limit();
    const unsigned g16 = (unsigned)((sp.n + 15) / 16);
#define IDS_TRSM_AXPY(GQ)                                                                                          \
    hipLaunchKernelGGL((trsm_axpy_kernel<GQ>), dim3((unsigned)((sp.n + 256 / GQ - 1) / (256 / GQ))), dim3(256),     \
                       sizeof(double) * (size_t)sp.k * (trsm_ax_ldk<GQ>() + 1), st, sp.n, sp.k, Rt, R11c, pos,     \
                       (const int64_t*)keff, P)
#define IDS_TRSM_GROUP(KS)                                                                                         \
    do {                                                                                                           \
        if (r11 <= lim)                                                                                            \
            hipLaunchKernelGGL((trsm_group_kernel<KS>), dim3(g16), dim3(256), r11, st, sp.n, sp.k, Rt, R11c, pos,  \
                               (const int64_t*)keff, P);                                                           \
        else                                                                                                       \
            hipLaunchKernelGGL((trsm_chunk_kernel<KS>), dim3(g16), dim3(256), 0, st, sp.n, sp.k, Rt, R11c, pos,    \
                               (const int64_t*)keff, P);                                                           \
    } while (0)
    // lanes per column of the solve for k <= 128 (tuned knobs; GQ lanes hold
    // 32 slots each, so GQ = 1, 2, 4 serve k <= 32, 64, 128; 8 is the
    // 16-lane dot-product kernel)
    // k <= 128: the one-kernel block solve on the FP64 matrix cores (tuned
    // knob trsm.mfma), else the lane-per-column kernels below
    if (sp.k <= 128 && tune_get("trsm.mfma", 0)) return solve_mfma_small(sp.n, sp.k, Rt, R11c, pos, keff, P, st);
    const size_t ax = sizeof(double) * (size_t)sp.k * (trsm_ax_ldk<4>() + 1);
    const int64_t gq = sp.k <= 32 ? tune_get("trsm.k32", 1) : sp.k <= 64 ? tune_get("trsm.k64", 2)
                                                                            : tune_get("trsm.k128", 4);
    if (sp.k <= 32 && gq == 1)
        IDS_TRSM_AXPY(1);
    else if (sp.k <= 64 && gq <= 2)
        IDS_TRSM_AXPY(2);
    else if (sp.k <= 128 && gq <= 4 && ax <= lim)
        IDS_TRSM_AXPY(4);
    else if (sp.k <= 128)
        IDS_TRSM_GROUP(8);
    else if (sp.k <= 256)
        IDS_TRSM_GROUP(16);
#undef IDS_TRSM_GROUP
#undef IDS_TRSM_AXPY
    else
        return solve_blocked(sp.n, sp.k, Rt, R11c, pos, keff, P, st);  // k > 256
    return check_launch("cpqr / interpolation matrix");
}

ids_status lambda_hat(int64_t k, int64_t n, const double* P, const int64_t* J, const int64_t* keff,
                      const double* lambda, double* lhat, hipStream_t st) {
    hipLaunchKernelGGL(lambda_hat_kernel, dim3((unsigned)k), dim3(256), 0, st, k, n, P, J, keff, lambda, lhat);
    return check_launch("lambda_hat");
}

}  // namespace ids

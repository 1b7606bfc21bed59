// Algorithm 1 for sketches with more columns than the register-resident
// pivoted QR holds: the columns live in a working copy in HBM (FP64, column
// major) and each pivot step is one ordinary kernel, so no workgroup ever
// waits for another.  Kernel t (t = 0 .. k), one wave per column:
//   1. pivot of step t - 1: every workgroup reduces the same per-workgroup
//      partials of kernel t - 1 (largest trailing norm, ties to the smallest
//      column index -- an order-independent maximum, so all agree) and forms
//      the winner's Householder reflector (v = 1 at row t - 1 and the
//      winner's rows below scaled by 1 / (alpha - beta), beta =
//      -sign(alpha) ||x||, tau = (beta - alpha) / beta; ||x||^2 is the
//      winner's trailing norm, as in the register-resident kernels);
//   2. the winner's wave records its rows above t - 1 and beta as row t - 1 of
//      R11 (R11c) and its step; every live column gets the reflector applied
//      to its rows >= t - 1 (row t - 1 of R into Rt); columns chosen earlier
//      are not touched again;
//   3. trailing norms over rows >= t recomputed in FP64, each workgroup's best
//      (with its entry in row t, the next alpha) into the partials of parity
//      t, which kernel t + 1 reads while kernel t's own are no longer needed.
// A zero largest norm stops the factorisation (k_eff = t - 1, the smallest
// such step); the stopping kernel leaves no candidates, so later kernels stop
// after their reduction too.  Lane q of a column's wave owns rows q + 64 u in every
// kernel, so a lane only ever reads rows of its own column that it wrote
// itself; the winner's column, staged once per workgroup in LDS as the
// reflector, is not written in the kernel that reads it.  The interpolation matrix is then solved from Rt /
// R11c by the same kernels as the register-resident path.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace ids {

struct StepArgs {
    const void* Y;
    int32_t ydt;
    int64_t l, n, rs, cs, k, ldw;
    double* W;        // working copy, column j at W + j ldw
    double* bn;       // 2 x nwg: per workgroup best trailing norm^2 (by step parity)
    double* ba;       //          that column's entry in the next pivot row
    int32_t* bj;      //          and its index (INT32_MAX: none)
    int32_t* ist;     // [0] k_eff so far (k until a stop), [1] non-finite flag
    double* Rt;       // n x k: column j's top k rows of R
    double* R11c;     // k x k: row t = top rows of the column chosen at step t
    int32_t* pos;     // step at which a column was chosen, -1 otherwise
    int64_t* J;
    int64_t* keff;
    int32_t* status;
    int nwg;
};

// waves (columns) per workgroup for U rows per lane: the column stays in
// registers (2 U VGPRs) within the per-wave budget
static inline int steps_waves(int64_t l) { return l <= 1024 ? 16 : l <= 2048 ? 8 : 4; }

__device__ __forceinline__ bool st_better(double n1, int j1, double n0, int j0) {
    return j1 != INT32_MAX && (n1 > n0 || (n1 == n0 && j1 < j0));
}

template <int U, int NW>
__global__ __launch_bounds__(64 * NW) void steps_kernel(StepArgs a, int t) {
    __shared__ double s_n[NW], s_a[NW];
    __shared__ int s_j[NW];
    __shared__ double s_r[3];
    __shared__ int s_w;
    __shared__ double sv[64 * U];  // the reflector of step t - 1
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * NW + w;
    const int l = (int)a.l, k = (int)a.k;
    const int s = t - 1;  // the step whose pivot this kernel takes and applies
    double* col = a.W + j * a.ldw;
    double y[U];
    bool live = false;
    // the column's rows, issued before the pivot reduction so both latencies overlap
    if (j < a.n) {
        if (t == 0) {
            // working copy of column j (FP32 sketches widened to FP64)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                double x = 0.0;
                if (i < l)
                    x = a.ydt == IDS_F64 ? ((const double*)a.Y)[i * a.rs + j * a.cs]
                                         : (double)((const float*)a.Y)[i * a.rs + j * a.cs];
                y[u] = x;
                if (i < l) col[i] = x;
            }
            if (lane == 0) a.pos[j] = -1;
            live = true;
        } else {
            // loaded whatever the column's state (no wait on pos); a column
            // chosen earlier drops them
            const int32_t pj = a.pos[j];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                y[u] = (i >= s && i < l) ? col[i] : 0.0;
            }
            live = pj < 0;
        }
    }
    if (t > 0) {
        // ---- 1. the pivot of step s
        const int par = s & 1;
        double bn = -1.0, ba = 0.0;
        int bj = INT32_MAX;
        for (int q = threadIdx.x; q < a.nwg; q += 64 * NW) {
            const double nq = a.bn[par * a.nwg + q];
            const int jq = a.bj[par * a.nwg + q];
            const double aq = a.ba[par * a.nwg + q];
            if (st_better(nq, jq, bn, bj)) {
                bn = nq;
                bj = jq;
                ba = aq;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double n2 = __shfl_xor(bn, o, 64);
            const int j2 = __shfl_xor(bj, o, 64);
            const double a2 = __shfl_xor(ba, o, 64);
            if (st_better(n2, j2, bn, bj)) {
                bn = n2;
                bj = j2;
                ba = a2;
            }
        }
        if (lane == 0) {
            s_n[w] = bn;
            s_j[w] = bj;
            s_a[w] = ba;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = -1.0, alpha = 0.0;
            int jb = INT32_MAX;
            for (int q = 0; q < NW; ++q)
                if (st_better(s_n[q], s_j[q], b, jb)) {
                    b = s_n[q];
                    jb = s_j[q];
                    alpha = s_a[q];
                }
            s_w = (jb == INT32_MAX || !(b > 0.0)) ? -1 : jb;
            if (s_w >= 0) {
                double tau, beta, scal;
                if (!(b > alpha * alpha)) {  // entries below s vanish to rounding: H = I
                    tau = 0.0;
                    beta = alpha;
                    scal = 0.0;
                } else {
                    const double nrm = sqrt(b);
                    beta = (alpha >= 0.0) ? -nrm : nrm;
                    tau = (beta - alpha) / beta;
                    scal = 1.0 / (alpha - beta);
                }
                s_r[0] = tau;
                s_r[1] = beta;
                s_r[2] = scal;
                if (blockIdx.x == 0) a.J[s] = jb;
            } else {
                // no pivot left: k_eff = s (the first such step; every
                // workgroup stops here and leaves no candidate, so every
                // later kernel stops at once as well)
                if (blockIdx.x == 0) __hip_atomic_fetch_min(a.ist, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (t < k) {
                    a.bn[(t & 1) * a.nwg + blockIdx.x] = -1.0;
                    a.bj[(t & 1) * a.nwg + blockIdx.x] = INT32_MAX;
                }
            }
        }
        __syncthreads();
        const int jw = s_w;
        if (jw < 0) return;
        const double tau = s_r[0], beta = s_r[1], scal = s_r[2];
        {
            // the reflector, once per workgroup: v_s = 1, v_i = x_i / (alpha - beta)
            const double* xw = a.W + (int64_t)jw * a.ldw;
            for (int i = threadIdx.x; i < 64 * U; i += 64 * NW)
                sv[i] = (i > s && i < l) ? xw[i] * scal : (i == s ? 1.0 : 0.0);
        }
        __syncthreads();
        // ---- 2. record the winner / apply H_s to the live columns
        if (j == jw) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                if (i < s) a.R11c[(int64_t)s * k + i] = col[i];
            }
            if (lane == 0) {
                a.R11c[(int64_t)s * k + s] = beta;
                a.Rt[j * k + s] = beta;
                a.pos[j] = s;
            }
            live = false;
        } else if (j < a.n && live) {
            double d = 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u) d = fma(sv[lane + 64 * u], y[u], d);
            d = wave_sum_dpp1(d);
            const double dt = d * tau;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                if (i >= s && i < l) {
                    y[u] = fma(-dt, sv[i], y[u]);
                    col[i] = y[u];
                    if (i == s) a.Rt[j * k + s] = y[u];  // row s of R
                }
            }
        }
    }
    if (t >= k) return;  // the last kernel only applies reflector k - 1
    // ---- 3. trailing norms over rows >= t, each workgroup's best
    double nu = -1.0, at = 0.0;
    int cj = INT32_MAX;
    if (j < a.n && live) {
        double q = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = lane + 64 * u;
            if (i >= t && i < l) q = fma(y[u], y[u], q);
            if (i == t) at = y[u];
        }
        nu = wave_sum_dpp1(q);
        at = __shfl(at, t & 63, 64);
        cj = (int)j;
        if (t == 0 && !__builtin_isfinite(nu) && lane == 0)
            __hip_atomic_store(a.ist + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // s_n / s_j / s_a are free again: the pivot reduction finished at the
    // barrier above
    if (lane == 0) {
        s_n[w] = nu;
        s_j[w] = cj;
        s_a[w] = at;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = -1.0, ab = 0.0;
        int jb = INT32_MAX;
        for (int q = 0; q < NW; ++q)
            if (st_better(s_n[q], s_j[q], b, jb)) {
                b = s_n[q];
                jb = s_j[q];
                ab = s_a[q];
            }
        const int par = t & 1;
        a.bn[par * a.nwg + blockIdx.x] = b;
        a.bj[par * a.nwg + blockIdx.x] = jb;
        a.ba[par * a.nwg + blockIdx.x] = ab;
    }
}

__global__ void steps_init_kernel(StepArgs a) {
    a.ist[0] = (int32_t)a.k;
    a.ist[1] = 0;
}

__global__ void steps_finish_kernel(StepArgs a) {
    const int kst = a.ist[0];
    *a.keff = kst;
    for (int64_t t = kst; t < a.k; ++t) a.J[t] = -1;
    if (a.status) *a.status = a.ist[1] ? IDS_ENONFINITE : (kst < a.k ? IDS_ERANKDEF : IDS_OK);
}

int64_t steps_workgroups(int64_t l, int64_t n) {
    const int nw = steps_waves(l);
    return (n + nw - 1) / nw;
}

size_t steps_bytes(int64_t l, int64_t n, int64_t k, int64_t* ldw) {
    const int64_t lw = (l + 7) / 8 * 8;
    const int64_t nwg = steps_workgroups(l, n);
    if (ldw) *ldw = lw;
    return align256(sizeof(double) * (size_t)lw * n) + 2 * align256(sizeof(double) * 2 * (size_t)nwg) +
           align256(sizeof(int32_t) * 2 * (size_t)nwg) + align256(sizeof(int32_t) * 2);
}

template <int U, int NW>
static void launch_step(const StepArgs& a, int t, hipStream_t st) {
    hipLaunchKernelGGL((steps_kernel<U, NW>), dim3((unsigned)a.nwg), dim3(64 * NW), 0, st, a, t);
}

// the factorisation; Rt, R11c, pos are the caller's (the same regions the
// register-resident path fills), ws the steps_bytes region
ids_status steps_factor(const void* Y, int32_t ydt, int64_t l, int64_t n, int64_t rs, int64_t cs, int64_t k,
                        int64_t* J, int64_t* keff, int32_t* status, double* Rt, double* R11c, int32_t* pos, char* ws,
                        hipStream_t st) {
    StepArgs a;
    a.Y = Y;
    a.ydt = ydt;
    a.l = l;
    a.n = n;
    a.rs = rs;
    a.cs = cs;
    a.k = k;
    steps_bytes(l, n, k, &a.ldw);
    const int64_t nwg = steps_workgroups(l, n);
    if (nwg > INT32_MAX) {
        set_error("id_select: too many columns for the column-steps factorisation");
        return IDS_EINVAL;
    }
    a.nwg = (int)nwg;
    char* p = ws;
    a.W = (double*)p;
    p += align256(sizeof(double) * (size_t)a.ldw * n);
    a.bn = (double*)p;
    p += align256(sizeof(double) * 2 * (size_t)nwg);
    a.ba = (double*)p;
    p += align256(sizeof(double) * 2 * (size_t)nwg);
    a.bj = (int32_t*)p;
    p += align256(sizeof(int32_t) * 2 * (size_t)nwg);
    a.ist = (int32_t*)p;
    a.Rt = Rt;
    a.R11c = R11c;
    a.pos = pos;
    a.J = J;
    a.keff = keff;
    a.status = status;
    const int U = l <= 128 ? 2 : l <= 256 ? 4 : l <= 512 ? 8 : l <= 1024 ? 16 : l <= 2048 ? 32 : 64;
    hipLaunchKernelGGL(steps_init_kernel, dim3(1), dim3(1), 0, st, a);
    for (int t = 0; t <= (int)k; ++t) {
        switch (U) {
            case 2: launch_step<2, 16>(a, t, st); break;
            case 4: launch_step<4, 16>(a, t, st); break;
            case 8: launch_step<8, 16>(a, t, st); break;
            case 16: launch_step<16, 16>(a, t, st); break;
            case 32: launch_step<32, 8>(a, t, st); break;
            default: launch_step<64, 4>(a, t, st); break;
        }
    }
    hipLaunchKernelGGL(steps_finish_kernel, dim3(1), dim3(1), 0, st, a);
    return check_launch("pivoted QR (column steps)");
}

}  // namespace ids

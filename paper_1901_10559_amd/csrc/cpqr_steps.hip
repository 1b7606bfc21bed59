// Algorithm 1 for sketches with more columns than the register-resident
// pivoted QR holds: the columns live in a working copy in HBM (FP64, column
// major) and each pivot step is two ordinary kernels, so no workgroup ever
// waits for another:
//   steps_update_kernel(t)  one wave per column: applies the reflector of step
//       t - 1 to the live columns and to the column chosen at t - 1 (whose
//       row t - 1 becomes beta), records row t - 1 of R (Rt; R11c for the
//       chosen column), then recomputes the trailing norms over rows >= t in
//       FP64 and leaves each workgroup's best (largest norm, smallest column
//       index) in a partials array;
//   steps_pivot_kernel(t)   one workgroup: reduces the partials to the winner,
//       forms its Householder reflector (v_t = 1, beta = -sign(alpha) ||x||,
//       tau = (beta - alpha) / beta; ||x||^2 is the winner's trailing norm, as
//       in the register-resident kernels) and stores v, tau, beta, J[t] and
//       the winner's step.
// A zero largest norm stops the factorisation (k_eff = t); later launches of
// the sequence return at once.  Lane q of a column's wave owns rows q + 64 u
// in every kernel, so a lane only ever reads rows it wrote itself.  The
// interpolation matrix is then solved from Rt / R11c by the same kernels as
// the register-resident path.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace ids {

constexpr int ST_WAVES = 4;  // columns per update workgroup, one wave each

struct StepArgs {
    const void* Y;
    int32_t ydt;
    int64_t l, n, rs, cs, k, ldw;
    double* W;        // working copy, column j at W + j ldw
    double* v;        // reflector of the last pivot step (rows >= its step)
    double* sc;       // [0] tau, [1] beta of the last pivot step
    double* bn;       // per update workgroup: best trailing norm^2
    int32_t* bj;      //                        and its column
    int32_t* ist;     // [0] k_eff so far (k until a stop), [1] non-finite flag
    double* Rt;       // n x k: column j's top k rows of R
    double* R11c;     // k x k: row t = top rows of the column chosen at step t
    int32_t* pos;     // step at which a column was chosen, -1 otherwise
    int64_t* J;
    int64_t* keff;
    int32_t* status;
};

// U = rows per lane (l <= 64 U); the column's rows in registers across the
// dot product and the update
template <int U>
__global__ __launch_bounds__(64 * ST_WAVES) void steps_update_kernel(StepArgs a, int t) {
    __shared__ double s_n[ST_WAVES];
    __shared__ int s_j[ST_WAVES];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * ST_WAVES + w;
    const int l = (int)a.l, k = (int)a.k;
    const int kstop = a.ist[0];
    double nu = -1.0;
    int cj = INT32_MAX;
    if (j < a.n) {
        double* col = a.W + j * a.ldw;
        double y[U];
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
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                y[u] = (i < l) ? col[i] : 0.0;
            }
        }
        const int32_t pj = (t == 0) ? -1 : a.pos[j];
        const int s = t - 1;  // the reflector to apply
        if (s >= 0 && s < kstop && (pj < 0 || pj == s)) {
            double d = 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                if (i >= s && i < l) d = fma(a.v[i], y[u], d);
            }
            d = wave_sum_dpp1(d);
            const double dt = d * a.sc[0];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                if (i >= s && i < l) {
                    y[u] = fma(-dt, a.v[i], y[u]);
                    if (pj == s && i == s) y[u] = a.sc[1];  // the chosen column: row s is beta
                    col[i] = y[u];
                }
            }
            // row s of R; the chosen column's top rows 0..s into R11c
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                if (i == s) a.Rt[j * k + s] = y[u];
                if (pj == s && i <= s) a.R11c[(int64_t)s * k + i] = y[u];
            }
        }
        if (t < kstop && t < k && pj < 0) {
            double q = 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = lane + 64 * u;
                if (i >= t && i < l) q = fma(y[u], y[u], q);
            }
            nu = wave_sum_dpp1(q);
            cj = (int)j;
            if (t == 0 && !__builtin_isfinite(nu) && lane == 0)
                __hip_atomic_store(a.ist + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (lane == 0) {
        s_n[w] = nu;
        s_j[w] = cj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bn = -1.0;
        int bj = INT32_MAX;
        for (int q = 0; q < ST_WAVES; ++q)
            if (s_j[q] != INT32_MAX && (s_n[q] > bn || (s_n[q] == bn && s_j[q] < bj))) {
                bn = s_n[q];
                bj = s_j[q];
            }
        a.bn[blockIdx.x] = bn;
        a.bj[blockIdx.x] = bj;
    }
}

constexpr int SP_THREADS = 256;
__global__ __launch_bounds__(SP_THREADS) void steps_pivot_kernel(StepArgs a, int t, int nwg) {
    __shared__ double s_n[SP_THREADS / 64];
    __shared__ int s_j[SP_THREADS / 64];
    __shared__ double s_r[3];
    __shared__ int s_w;
    if (t >= a.ist[0]) return;  // stopped at an earlier step
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double bn = -1.0;
    int bj = INT32_MAX;
    for (int q = tid; q < nwg; q += SP_THREADS) {
        const double nq = a.bn[q];
        const int jq = a.bj[q];
        if (jq != INT32_MAX && (nq > bn || (nq == bn && jq < bj))) {
            bn = nq;
            bj = jq;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double n2 = __shfl_xor(bn, o, 64);
        const int j2 = __shfl_xor(bj, o, 64);
        if (j2 != INT32_MAX && (n2 > bn || (n2 == bn && j2 < bj))) {
            bn = n2;
            bj = j2;
        }
    }
    if (lane == 0) {
        s_n[w] = bn;
        s_j[w] = bj;
    }
    __syncthreads();
    if (tid == 0) {
        double b = -1.0;
        int jb = INT32_MAX;
        for (int q = 0; q < SP_THREADS / 64; ++q)
            if (s_j[q] != INT32_MAX && (s_n[q] > b || (s_n[q] == b && s_j[q] < jb))) {
                b = s_n[q];
                jb = s_j[q];
            }
        s_w = (jb == INT32_MAX || !(b > 0.0)) ? -1 : jb;
        if (s_w >= 0) {
            const double alpha = a.W[(int64_t)jb * a.ldw + t];
            double tau, beta, scal;
            if (!(b > alpha * alpha)) {  // entries below t vanish to rounding: H = I
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
            a.sc[0] = tau;
            a.sc[1] = beta;
            a.J[t] = jb;
            a.pos[jb] = t;
        } else {
            a.ist[0] = t;  // no pivot left: k_eff = t
        }
    }
    __syncthreads();
    const int wj = s_w;
    if (wj < 0) return;
    const double scal = s_r[2];
    const double* x = a.W + (int64_t)wj * a.ldw;
    for (int i = t + tid; i < (int)a.l; i += SP_THREADS) a.v[i] = (i == t) ? 1.0 : x[i] * scal;
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

size_t steps_bytes(int64_t l, int64_t n, int64_t k, int64_t* ldw) {
    const int64_t lw = (l + 7) / 8 * 8;
    const int64_t nwg = (n + ST_WAVES - 1) / ST_WAVES;
    if (ldw) *ldw = lw;
    return align256(sizeof(double) * (size_t)lw * n) + align256(sizeof(double) * (size_t)l) +
           align256(sizeof(double) * 2) + align256(sizeof(double) * (size_t)nwg) +
           align256(sizeof(int32_t) * (size_t)nwg) + align256(sizeof(int32_t) * 2);
}

template <int U>
static void launch_update(const StepArgs& a, int t, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL(steps_update_kernel<U>, dim3(grid), dim3(64 * ST_WAVES), 0, st, a, t);
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
    const int64_t nwg = (n + ST_WAVES - 1) / ST_WAVES;
    char* p = ws;
    a.W = (double*)p;
    p += align256(sizeof(double) * (size_t)a.ldw * n);
    a.v = (double*)p;
    p += align256(sizeof(double) * (size_t)l);
    a.sc = (double*)p;
    p += align256(sizeof(double) * 2);
    a.bn = (double*)p;
    p += align256(sizeof(double) * (size_t)nwg);
    a.bj = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)nwg);
    a.ist = (int32_t*)p;
    a.Rt = Rt;
    a.R11c = R11c;
    a.pos = pos;
    a.J = J;
    a.keff = keff;
    a.status = status;
    const int U = l <= 128 ? 2 : l <= 256 ? 4 : l <= 512 ? 8 : l <= 1024 ? 16 : l <= 2048 ? 32 : 64;
    auto update = [&](int t) {
        switch (U) {
            case 2: launch_update<2>(a, t, (unsigned)nwg, st); break;
            case 4: launch_update<4>(a, t, (unsigned)nwg, st); break;
            case 8: launch_update<8>(a, t, (unsigned)nwg, st); break;
            case 16: launch_update<16>(a, t, (unsigned)nwg, st); break;
            case 32: launch_update<32>(a, t, (unsigned)nwg, st); break;
            default: launch_update<64>(a, t, (unsigned)nwg, st); break;
        }
    };
    hipLaunchKernelGGL(steps_init_kernel, dim3(1), dim3(1), 0, st, a);
    update(0);
    for (int t = 0; t < (int)k; ++t) {
        hipLaunchKernelGGL(steps_pivot_kernel, dim3(1), dim3(SP_THREADS), 0, st, a, t, (int)nwg);
        update(t + 1);  // applies reflector t (the last one: records R row k - 1 only)
    }
    hipLaunchKernelGGL(steps_finish_kernel, dim3(1), dim3(1), 0, st, a);
    return check_launch("pivoted QR (column steps)");
}

}  // namespace ids

// Batched mixed-precision matrix ID: thousands of independent dense problems
// A_p (m_p x n_p, BF16, row-major), each through Algorithm 2 with a Gaussian
// second stage and Algorithm 1:
//   batched_sketch_kernel  one workgroup per problem (largest first): the
//       CountSketch plan in LDS, then per 128-column panel and per group of 64
//       buckets (paired largest with smallest for the gather threads), Y1
//       rows summed in FP32 from 16-byte BF16 loads, split into
//       BF16 hi + lo, and multiplied by the BF16 Gaussian G on the matrix cores
//       (v_mfma_f32_16x16x32_bf16, FP32 accumulation): Y_p = G (S A_p) stays in
//       registers per panel and is written once (FP32, column-major).
//   batched_cpqr_kernel    one workgroup per problem (1024, 512 or 256
//       threads by n_p): column j of Y_p in lane j (rows 0..RL-1 in LDS, rows
//       RL.. in registers), FP32 data and Householder updates, trailing norms
//       recomputed in FP64 each step.
//   With tol > 0 (fixed-accuracy ID) problem p stops at the first step t with
//   |r_tt| <= tol |r_11| and returns k_eff_p = t (its adaptive rank).
//   batched_solve_kernel   one workgroup per problem: the interpolation
//       matrix P_p by FP64 block back-substitution on the matrix cores
//       (R11 blocks and their inverses in LDS), 16 consecutive columns of P_p
//       per wave at a time.
// Problem p draws its CountSketch from the stream (seed, tag = p) and uses
// the first l1_p = min(m_p, l1max) columns of the shared l x l1max G.
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "solve.hpp"
#include "tune.hpp"

namespace ids {

typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));
typedef unsigned int bu4 __attribute__((ext_vector_type(4)));

// A is read once: non-temporal 16-byte loads
__device__ __forceinline__ uint4 load_nt16(const uint16_t* p) {
    const bu4 v = __builtin_nontemporal_load(reinterpret_cast<const bu4*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
typedef float v4f32 __attribute__((ext_vector_type(4)));

struct BProb {
    int32_t m, n, l1, pad;
    int64_t a_off;  // element offset of A_p
    int64_t y_off;  // element offset of Y_p (l x n FP32, column-major)
    int64_t p_off;  // element offset of P_p (k x n FP64, row-major)
    int64_t r_off;  // element offset of Rt_p (n x k FP64) and pos_p (n int32)
};

struct BatchHdr {
    int64_t nprob, k, l, l1max;
    int64_t y_elems, r_elems;
    int32_t max_n, max_m;
};

// plan buffer layout (device): BatchHdr | BProb[nprob] | order_sketch[nprob] | order_cpqr[nprob]
static size_t plan_layout(int64_t nprob, size_t* off_prob, size_t* off_o1, size_t* off_o2) {
    size_t o = align256(sizeof(BatchHdr));
    *off_prob = o;
    o += align256(sizeof(BProb) * (size_t)nprob);
    *off_o1 = o;
    o += align256(sizeof(int32_t) * (size_t)nprob);
    *off_o2 = o;
    o += align256(sizeof(int32_t) * (size_t)nprob);
    return o;
}

struct BatchArgs {
    const BProb* prob;
    const int32_t* order;
    int64_t nprob, k, l, l1max;
    uint64_t seed;
    double tol2;        // fixed-accuracy stop: |r_tt|^2 <= tol2 |r_11|^2 (0: fixed rank k)
    const uint16_t* A;
    int64_t a_elems;    // elements of A (all problems)
    int32_t a_al16;     // A is 16-byte aligned
    const uint16_t* G;  // l x l1max BF16
    int32_t g_vec;      // G rows 16-byte aligned (l1max % 8 == 0, G aligned)
    float* Y;
    double* Rt;
    int32_t* pos;
    double* beta;       // nprob x k: R[t][J[t]] in FP64
    int64_t* J;
    double* P;
    int64_t* keff;
    int32_t* status;    // optional, per problem
};

// ---------------------------------------------------------------------------
// K1: CountSketch + projection
// ---------------------------------------------------------------------------
constexpr int BS_THREADS = 512;  // two problems per CU (LDS and registers allow it)
constexpr int BS_PANEL = 128;   // columns per panel
constexpr int BS_BG = 64;       // buckets per group (two MFMA K steps of 32)
constexpr int BS_YS = BS_BG + 8;  // LDS row of a sketch-tile column (u16; 16-byte multiple)
// column c of the sketch tile starts at ys_off(c): one extra 16-byte slot every
// 8 columns, so the gather's 8-column chunks (otherwise 8 * 144 B apart, all in
// one bank) spread over the banks
__device__ __forceinline__ int ys_off(int c) { return c * BS_YS + (c >> 3) * 8; }
constexpr int BS_YN = BS_PANEL * BS_YS + (BS_PANEL / 8) * 8;
constexpr int BS_LMAX = 128;    // padded sketch height (l <= 128)
constexpr int BS_MMAX = 4096;   // rows per problem
constexpr int BS_L1MAX = 512;   // buckets per problem
constexpr int BS_IIF = 4;       // row loads in flight per gather thread (aligned rows)
static_assert(BS_THREADS / 64 >= BS_L1MAX / BS_BG, "one wave per bucket group sorts its bucket sizes");

__device__ __forceinline__ uint16_t f2bf_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(BS_THREADS, 4) void batched_sketch_kernel(BatchArgs a) {  // 2 workgroups per CU
    __shared__ int32_t cnt[BS_L1MAX + 1];
    __shared__ int32_t off[BS_L1MAX + 1];
    __shared__ int32_t rows[BS_MMAX];
    // transposed sketch tile [column][bucket]; rows of 40 entries (80 bytes,
    // a multiple of 16) so each MFMA operand is one 16-byte LDS read
    __shared__ __attribute__((aligned(16))) uint16_t Y1h[BS_YN];
    __shared__ __attribute__((aligned(16))) uint16_t Y1l[BS_YN];
    __shared__ __attribute__((aligned(16))) uint16_t Gs[BS_LMAX][BS_YS];
    // per bucket group: slot s < 32 -> the s-th largest bucket, slot 32 + s ->
    // the s-th smallest (positions within the group)
    __shared__ uint8_t pairing[BS_L1MAX];

    const int p = a.order[blockIdx.x];
    const BProb pr = a.prob[p];
    const int m = pr.m, n = pr.n, L1 = pr.l1;
    const int l = (int)a.l;
    const int tid = threadIdx.x;
    const uint64_t key = stream_key(a.seed, (uint64_t)p);

    // ---- plan: bucket counts, offsets, rows grouped by bucket (ascending)
    for (int b = tid; b <= L1; b += BS_THREADS) cnt[b] = 0;
    __syncthreads();
    for (int i = tid; i < m; i += BS_THREADS) {
        uint32_t b;
        bool neg;
        hash_row(key, i, (uint32_t)L1, b, neg);
        atomicAdd(&cnt[b], 1);
    }
    __syncthreads();
    if (tid < 64) {
        // exclusive scan of L1 counts by one wave
        int carry = 0;
        for (int b0 = 0; b0 < L1; b0 += 64) {
            const int b = b0 + tid;
            const int v = b < L1 ? cnt[b] : 0;
            int x = v;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (tid >= o) x += y;
            }
            if (b < L1) off[b] = carry + x - v;
            carry += __shfl(x, 63, 64);
        }
        if (tid == 0) off[L1] = carry;
    }
    __syncthreads();
    for (int b = tid; b < L1; b += BS_THREADS) cnt[b] = off[b];
    __syncthreads();
    for (int i = tid; i < m; i += BS_THREADS) {
        uint32_t b;
        bool neg;
        hash_row(key, i, (uint32_t)L1, b, neg);
        const int q = atomicAdd(&cnt[b], 1);
        rows[q] = encode_row(i, neg);
    }
    __syncthreads();
    // rows of a bucket in increasing row order (insertion sort, buckets are short)
    for (int b = tid; b < L1; b += BS_THREADS) {
        for (int q = off[b] + 1; q < off[b + 1]; ++q) {
            const int32_t c = rows[q];
            const int32_t ci = c >= 0 ? c : -c - 1;
            int r = q - 1;
            while (r >= off[b]) {
                const int32_t d = rows[r];
                const int32_t di = d >= 0 ? d : -d - 1;
                if (di <= ci) break;
                rows[r + 1] = d;
                --r;
            }
            rows[r + 1] = c;
        }
    }
    // gather balance: a gather thread sums two buckets of a 64-bucket group,
    // the s-th largest with the s-th smallest, so each thread reads close to
    // the group's mean of 2 m / L1 rows instead of the largest bucket's count
    // (one wave per group: bitonic sort of (count, position) keys)
    {
        const int wv = tid >> 6, ln = tid & 63, g0 = wv * BS_BG;
        if (g0 < L1) {
            const int b = g0 + ln;
            uint32_t key = ((uint32_t)(b < L1 ? off[b + 1] - off[b] : 0) << 6) | (uint32_t)ln;
#pragma unroll
            for (int k2 = 2; k2 <= 64; k2 <<= 1)
#pragma unroll
                for (int j = k2 >> 1; j > 0; j >>= 1) {
                    const uint32_t o = (uint32_t)__shfl_xor((int)key, j, 64);
                    key = (((ln & j) == 0) == ((ln & k2) == 0)) ? min(key, o) : max(key, o);
                }
            pairing[g0 + (ln >= 32 ? 63 - ln : 32 + ln)] = (uint8_t)(key & 63);
        }
    }
    __syncthreads();

    const int w = tid >> 6, lane = tid & 63;
    // MFMA phase: wave w owns row tiles rt0 .. rt0 + 3 (16 rows of Y each) and
    // column tiles ct0, ct0 + 1 (16 columns of the panel each): 4 G and 4 Y1
    // operand reads per 32-bucket step instead of 1 and 16 for a 16 x 128
    // strip, so half the LDS reads and operand registers
    const int rt0 = 4 * (w >> 2);
    const int ct0 = 2 * (w & 3);
    const int bl = tid >> 4;        // pairing slot: buckets pairing[g0 + bl], pairing[g0 + 32 + bl] (gather)
    const int ch = tid & 15;        // 8-column chunk within panel (gather phase)
    const uint16_t* Ap = a.A + pr.a_off;
    float* Yp = a.Y + pr.y_off;

    for (int c0 = 0; c0 < n; c0 += BS_PANEL) {
        v4f32 acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = v4f32{0.f, 0.f, 0.f, 0.f};
        for (int g0 = 0; g0 < L1; g0 += BS_BG) {
            // G[:, g0 .. g0 + 64): two 16-byte row chunks per thread (rows >= l
            // and columns >= L1 are zero), loaded first and stored to LDS after
            // the gather, so the two loads' latencies overlap
            uint4 gvals[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                static_assert(2 * BS_THREADS == BS_LMAX * BS_BG / 8, "two G chunks per thread");
                const int id = tid + u * BS_THREADS;
                const int r = id >> 3, c8 = (id & 7) * 8, gc = g0 + c8;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (r < l) {
                    const uint16_t* gp = a.G + (int64_t)r * a.l1max + gc;
                    if (a.g_vec && gc + 8 <= L1) {
                        v = *reinterpret_cast<const uint4*>(gp);
                    } else {
                        uint32_t e[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) e[q] = (gc + q < L1) ? gp[q] : 0u;
                        v = make_uint4(e[0] | (e[1] << 16), e[2] | (e[3] << 16), e[4] | (e[5] << 16), e[6] | (e[7] << 16));
                    }
                }
                gvals[u] = v;
            }
            // gather: Y1[b][c0 + 8ch .. +8] for the two buckets b = g0 + pb[h]
            // paired for this thread's slot bl; the thread walks one stream of
            // qn[0] + qn[1] rows (bucket 0's, then bucket 1's), each bucket's rows
            // added in increasing row order
            {
                const int cc = c0 + 8 * ch;
                // rows 16-byte aligned (n % 8 == 0 and A_p aligned): one load per
                // chunk; otherwise a chunk spans two aligned 16-byte blocks and
                // is shifted out of them (uniform per problem)
                const bool vec = a.a_al16 && (n % 8) == 0 && (pr.a_off % 8) == 0;
                int qb[2], qn[2], pb[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    pb[h] = pairing[g0 + 32 * h + bl];
                    const int b = g0 + pb[h];
                    const bool ok = b < L1 && cc < n;
                    qb[h] = ok ? off[b] : 0;
                    qn[h] = ok ? off[b + 1] - off[b] : 0;
                }
                const int nq = qn[0] + qn[1];
                float s[2][8];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int e = 0; e < 8; ++e) s[h][e] = 0.f;
                // item q of the stream: its bucket slot h and row code (past the
                // stream: row 0, not added)
                auto item = [&](int q, int& h, int32_t& code) {
                    h = q >= qn[0] ? 1 : 0;
                    const int r = (q < nq) ? (h ? qb[1] + q - qn[0] : qb[0] + q) : 0;
                    code = rows[r];
                    code = (q < nq) ? code : 0;
                };
                // one chunk (8 BF16 in 4 words) into the sum of bucket slot h:
                // fma(g, x, s) with g = +-1 (the row's sign) in slot h and +0 in
                // the other adds exactly s +- x and s + 0 (for finite x), two
                // FMAs per element instead of a routed add.  Elements past column
                // n - 1 only reach discarded columns of Y.
                auto add = [&](int h, int32_t code, const uint32_t (&w4)[4]) {
                    const float sg = code < 0 ? -1.f : 1.f;
                    const float g0s = h ? 0.f : sg, g1s = h ? sg : 0.f;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const uint32_t wd = w4[e >> 1];
                        const float xe = __uint_as_float((e & 1) ? (wd & 0xffff0000u) : (wd << 16));
                        s[0][e] = fmaf(g0s, xe, s[0][e]);
                        s[1][e] = fmaf(g1s, xe, s[1][e]);
                    }
                };
                if (vec) {
                    for (int q0 = 0; q0 < nq; q0 += BS_IIF) {
                        uint32_t raw[BS_IIF][4];
                        int32_t code[BS_IIF];
                        int hs[BS_IIF];
                        // all loads issued before any is used
#pragma unroll
                        for (int u = 0; u < BS_IIF; ++u) {
                            item(q0 + u, hs[u], code[u]);
                            const int64_t i = code[u] >= 0 ? code[u] : -(int64_t)code[u] - 1;
                            const uint4 v = load_nt16(Ap + i * n + cc);
                            raw[u][0] = v.x; raw[u][1] = v.y; raw[u][2] = v.z; raw[u][3] = v.w;
                        }
                        asm volatile("" ::: "memory");
#pragma unroll
                        for (int u = 0; u < BS_IIF; ++u) {
                            if (q0 + u >= nq) break;
                            add(hs[u], code[u], raw[u]);
                        }
                    }
                } else {
                    for (int q0 = 0; q0 < nq; q0 += 2) {
                        uint32_t w[2][8];
                        int32_t code[2];
                        int hs[2], sh[2];
                        bool tail[2];
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            item(q0 + u, hs[u], code[u]);
                            const int64_t i = code[u] >= 0 ? code[u] : -(int64_t)code[u] - 1;
                            const int64_t e0 = pr.a_off + i * n + cc;  // element index in A
                            int64_t base = e0 & ~(int64_t)7;
                            // element loads where the second block would pass the end of
                            // A (or A itself is not 16-byte aligned)
                            tail[u] = !a.a_al16 || base + 16 > a.a_elems;
                            if (tail[u]) base = 0;
                            sh[u] = (int)(e0 - (e0 & ~(int64_t)7));
                            const uint4 b0 = load_nt16(a.A + base), b1 = load_nt16(a.A + base + 8);
                            w[u][0] = b0.x; w[u][1] = b0.y; w[u][2] = b0.z; w[u][3] = b0.w;
                            w[u][4] = b1.x; w[u][5] = b1.y; w[u][6] = b1.z; w[u][7] = b1.w;
                        }
                        asm volatile("" ::: "memory");
#pragma unroll
                        for (int u = 0; u < 2; ++u) {
                            if (q0 + u >= nq) continue;
                            uint32_t w4[4];
                            if (!tail[u]) {
                                // elements sh .. sh + 7 of the 16 loaded: words d .. d + 4
                                // (d = sh / 2), shifted by one element when sh is odd
                                // (words picked by the two bits of d in turn, as bit
                                // selects: a select of array elements would become an
                                // indexed private array)
                                const int d = sh[u] >> 1;
                                const uint32_t m2 = 0u - (uint32_t)((d >> 1) & 1), m1 = 0u - (uint32_t)(d & 1);
                                uint32_t u6[6], v5[5];
#pragma unroll
                                for (int q = 0; q < 6; ++q) u6[q] = (w[u][q + 2] & m2) | (w[u][q] & ~m2);
#pragma unroll
                                for (int q = 0; q < 5; ++q) v5[q] = (u6[q + 1] & m1) | (u6[q] & ~m1);
                                const uint32_t bs = (uint32_t)(sh[u] & 1) * 2u;
#pragma unroll
                                for (int q = 0; q < 4; ++q) w4[q] = __builtin_amdgcn_alignbyte(v5[q + 1], v5[q], bs);
                            } else {
                                const int64_t i = code[u] >= 0 ? code[u] : -(int64_t)code[u] - 1;
                                const uint16_t* rowp = Ap + i * n + cc;
                                uint32_t hh[8];
#pragma unroll
                                for (int e = 0; e < 8; ++e) hh[e] = (cc + e < n) ? rowp[e] : 0u;
#pragma unroll
                                for (int e = 0; e < 4; ++e) w4[e] = hh[2 * e] | (hh[2 * e + 1] << 16);
                            }
                            add(hs[u], code[u], w4);
                        }
                    }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const uint16_t hi = f2bf_rne(s[h][e]);
                        const float hf = bf16_to_f32(hi);
                        const int o = ys_off(8 * ch + e) + pb[h];
                        Y1h[o] = hi;
                        Y1l[o] = f2bf_rne(s[h][e] - hf);
                    }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int id = tid + u * BS_THREADS;
                *reinterpret_cast<uint4*>(&Gs[id >> 3][(id & 7) * 8]) = gvals[u];
            }
            __syncthreads();
            // Y(rows rt*16.., cols ct*16..) += G tile (16 x 64) * Y1 (64 x 16), hi and lo
#pragma unroll
            for (int kk = 0; kk < BS_BG / 32; ++kk) {
                v8bf16 av[4], bh[2], blo[2];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    av[i] = __builtin_bit_cast(v8bf16, *reinterpret_cast<const uint4*>(
                                                           &Gs[(rt0 + i) * 16 + (lane & 15)][32 * kk + 8 * (lane >> 4)]));
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int o = ys_off((ct0 + c) * 16 + (lane & 15)) + 32 * kk + 8 * (lane >> 4);
                    bh[c] = __builtin_bit_cast(v8bf16, *reinterpret_cast<const uint4*>(&Y1h[o]));
                    blo[c] = __builtin_bit_cast(v8bf16, *reinterpret_cast<const uint4*>(&Y1l[o]));
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        acc[2 * i + c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bh[c], acc[2 * i + c], 0, 0, 0);
                        acc[2 * i + c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], blo[c], acc[2 * i + c], 0, 0, 0);
                    }
            }
            __syncthreads();
        }
        // write the panel of Y_p (column-major, leading dimension l)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int col = c0 + (ct0 + (q & 1)) * 16 + (lane & 15);
            if (col >= n) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = (rt0 + (q >> 1)) * 16 + 4 * (lane >> 4) + r;
                if (row < l) Yp[(int64_t)col * l + row] = acc[q][r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K2: CPQR, FP32 data, FP64 norms
// ---------------------------------------------------------------------------
constexpr int BC_THREADS = 1024;  // largest workgroup: n_p <= 1024 columns, one per thread
constexpr int BC_ROWS = 122;  // sketch rows held per column (l <= 122)
constexpr int BC_RL = 36;     // rows in LDS for the 1024-thread class (a multiple of 4, so
                              // the register rows' reflector entries start 16-byte aligned)
static_assert(BC_ROWS <= BS_LMAX, "batched CPQR rows");

// wave argmax of (nu, j): DPP max tree for nu, then DPP min tree over the j
// of the lanes holding the maximum; both fold into lane 63 and are broadcast.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dppk_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dppk_i32(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ void wave_argmax_dpp(double& nu, int& j) {
    double m = nu;
    m = fmax(m, dppk_f64<0xB1, 0xf>(m));
    m = fmax(m, dppk_f64<0x4E, 0xf>(m));
    m = fmax(m, dppk_f64<0x141, 0xf>(m));
    m = fmax(m, dppk_f64<0x140, 0xf>(m));
    m = fmax(m, dppk_f64<0x142, 0xa>(m));
    m = fmax(m, dppk_f64<0x143, 0xc>(m));
    m = lane63_f64(m);
    int q = (nu == m) ? j : INT32_MAX;
    q = min(q, dppk_i32<0xB1, 0xf>(q));
    q = min(q, dppk_i32<0x4E, 0xf>(q));
    q = min(q, dppk_i32<0x141, 0xf>(q));
    q = min(q, dppk_i32<0x140, 0xf>(q));
    q = min(q, dppk_i32<0x142, 0xa>(q));
    q = min(q, dppk_i32<0x143, 0xc>(q));
    nu = m;
    j = __builtin_amdgcn_readlane(q, 63);
}

template <int N>
__device__ __forceinline__ double tree_sum_d(double (&s)[N]) {
#pragma unroll
    for (int h = N / 2; h > 0; h >>= 1)
#pragma unroll
        for (int q = 0; q < h; ++q) s[q] += s[q + h];
    return s[0];
}

// NT threads per problem, launched for the problems with NT/2 < n_p <= NT
// (n_p <= NT for the smallest NT), so small problems share a CU and hide each
// other's per-step latency.  RL of the BC_ROWS rows live in LDS (the first
// ones, frozen after step RL), the rest in registers: 1024 threads get at
// most 128 VGPRs each (4 waves per SIMD), so the widest class keeps 36 rows in
// LDS; 512 and 256 threads keep every row in registers (up to 256 VGPRs, 2
// waves per SIMD).
template <int NT, int RL>
__global__ __launch_bounds__(NT, RL ? 4 : 2) void batched_cpqr_kernel(BatchArgs a, int nt_min) {
    constexpr int RR = BC_ROWS - RL;          // rows in registers
    extern __shared__ float ylds[];           // RL x NT
    __shared__ __attribute__((aligned(16))) float xf[BS_LMAX];  // pivot column (FP32)
    __shared__ double s_hh[2];                                  // tau scal^2, beta
    __shared__ double s_nu[16];
    __shared__ int s_j[16];

    const int p = a.order[blockIdx.x];
    const BProb pr = a.prob[p];
    const int n = pr.n;
    if (n > NT || n <= nt_min) return;  // another launch owns this problem
    const int l = (int)a.l, k = (int)a.k;
    const int j = threadIdx.x;
    const int lane = j & 63, w = j >> 6;
    const bool wave_live = w * 64 < n;        // waves past the last column skip column work
    bool alive = j < n;
    const float* Yp = a.Y + pr.y_off;

    float y[RR];
    {
        // column j of Y_p (clamped addresses, so every load is unconditional
        // and all are in flight together; masked after compiler barriers):
        // the LDS rows travel through y first, then the register rows
        static_assert(RL <= RR, "LDS rows are staged in y");
        static_assert(RL % 4 == 0, "the pivot column is published in 16-byte stores");
        const float* colp = Yp + (int64_t)min(j, n - 1) * l;
#pragma unroll
        for (int r = 0; r < RL; ++r) y[r] = colp[min(r, l - 1)];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < RL; ++r) ylds[r * NT + j] = (alive && r < l) ? y[r] : 0.f;
#pragma unroll
        for (int r = 0; r < RR; ++r) y[r] = colp[min(RL + r, l - 1)];
        asm volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < RR; ++r) y[r] = (alive && RL + r < l) ? y[r] : 0.f;
    }
    // sum of squares over rows i >= t0: squares summed in FP32 over chunks of 8
    // rows, the chunk sums accumulated in FP64 (relative error <= 8 * 2^-24,
    // below the FP32 rounding of the data itself).  The LDS rows' loop is
    // unrolled by 4 so their reads overlap; a full unroll spills at 1024 threads.
    auto norm_from = [&](int t0) -> double {
        double s = 0.0;
        float f[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int r = t0; r < RL; ++r) {
            const float v = ylds[r * NT + j];
            f[r & 3] = fmaf(v, v, f[r & 3]);
        }
        s = (double)((f[0] + f[1]) + (f[2] + f[3]));
#pragma unroll
        for (int c = 0; c < RR; c += 8) {
            if (RL + c + 8 > t0) {
                float q = 0.f;
#pragma unroll
                for (int r = c; r < c + 8 && r < RR; ++r) {
                    const float v = (RL + r >= t0) ? y[r] : 0.f;
                    q = fmaf(v, v, q);
                }
                s += (double)q;
            }
        }
        return s;
    };
    double nu = wave_live ? norm_from(0) : 0.0;
    // a non-finite entry of Y_p (or an overflowing norm) is reported per problem
    const bool nonfinite = __syncthreads_or(alive && !__builtin_isfinite(nu)) != 0;
    bool rankdef = false;
    int keff = k;
    double nu0 = 0.0;  // |r_11|^2
    const int64_t roff = pr.r_off;
    if (alive) a.pos[roff + j] = -1;

    for (int t = 0; t < k; ++t) {
        // ---- argmax of (nu, j): per wave, then across waves by every wave
        {
            double m2 = alive ? nu : -1.0;
            int q2 = alive ? j : INT32_MAX;
            wave_argmax_dpp(m2, q2);
            if (lane == 0) {
                s_nu[w] = m2;
                s_j[w] = q2;
            }
        }
        __syncthreads();
        double wnu;
        int wj;
        {
            double m2 = (lane < NT / 64) ? s_nu[lane] : -1.0;
            int q2 = (lane < NT / 64) ? s_j[lane] : INT32_MAX;
            wave_argmax_dpp(m2, q2);
            wnu = m2;
            wj = q2;
        }
        if (t == 0) nu0 = wnu;
        // stop at rank deficiency, or (fixed accuracy) once the pivot's trailing
        // norm |r_tt| = sqrt(wnu) is at most tol |r_11|
        if (wj == INT32_MAX || !(wnu > 0.0) || (t > 0 && wnu <= a.tol2 * nu0)) {
            rankdef = wj == INT32_MAX || !(wnu > 0.0);
            keff = t;
            break;
        }
        // ---- pivot column x to LDS (rows above t zeroed) and the Householder
        //      scalars, formed by the pivot's owner lane in FP64 from
        //      alpha = x_t and the published trailing norm wnu = ||x_{t..}||^2:
        //      v = scal * x' with x'_t = alpha - beta (so v_t = 1) and x'_i = x_i
        //      below t, so the update needs x' and the scalars only -- one
        //      workgroup barrier for both.  The owner's register rows go out as
        //      they are, its LDS rows and the other rows < RL are copied by the
        //      threads j < RL (thread t leaves row t to the owner).
        if (j == wj) {
            // the register rows in 16-byte stores (RL is a multiple of 4)
#pragma unroll
            for (int r = 0; r + 3 < RR; r += 4) {
                float4 q;
                q.x = (RL + r < t) ? 0.f : y[r];
                q.y = (RL + r + 1 < t) ? 0.f : y[r + 1];
                q.z = (RL + r + 2 < t) ? 0.f : y[r + 2];
                q.w = (RL + r + 3 < t) ? 0.f : y[r + 3];
                *reinterpret_cast<float4*>(&xf[RL + r]) = q;
            }
#pragma unroll
            for (int r = RR & ~3; r < RR; ++r) xf[RL + r] = (RL + r < t) ? 0.f : y[r];
            const double alpha = (double)((t < RL) ? ylds[t * NT + j] : xf[t]);
            double tss_o, beta_o;
            if (!(wnu > alpha * alpha)) {
                tss_o = 0.0;  // H = I
                beta_o = alpha;
            } else {
                const double nrm = sqrt(wnu);
                beta_o = (alpha >= 0.0) ? -nrm : nrm;
                // tau scal^2 with tau = (beta - alpha) / beta, scal = 1 / (alpha - beta)
                tss_o = -1.0 / (beta_o * (alpha - beta_o));
            }
            xf[t] = (float)(alpha - beta_o);
            s_hh[0] = tss_o;  // H y = y - (tau scal^2 x'^T y) x'
            s_hh[1] = beta_o;
        }
        if (j < RL && j != t) xf[j] = (j < t) ? 0.f : ylds[j * NT + wj];
        __syncthreads();
        const double tss = s_hh[0], beta = s_hh[1];
        // ---- apply H to the live columns (FP32 dot and update), new norms
        if (wave_live) {
            if (alive) {
                float d[4] = {0.f, 0.f, 0.f, 0.f};
                if (t < RL) {
#pragma unroll 4
                    for (int r = t; r < RL; ++r) d[r & 3] = fmaf(xf[r], ylds[r * NT + j], d[r & 3]);
                }
#pragma unroll
                for (int c = 0; c < RR; c += 8)
                    if (RL + c + 8 > t) {
#pragma unroll
                        for (int r = c; r < c + 8 && r < RR; ++r)
                            if (RL + r < BS_LMAX) d[r & 3] = fmaf(xf[RL + r], y[r], d[r & 3]);
                    }
                const float dt = (float)((double)((d[0] + d[1]) + (d[2] + d[3])) * tss);
                // the update, with the new trailing norm (rows >= t + 1) summed
                // as the rows are written: the same rows in the same FP32
                // accumulators and order as norm_from(t + 1), without reading
                // the LDS rows a second time
                double s = 0.0;
                if (t < RL) {
                    float f[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
                    for (int r = t; r < RL; ++r) {
                        const float v = fmaf(-dt, xf[r], ylds[r * NT + j]);
                        ylds[r * NT + j] = v;
                        if (r > t) f[r & 3] = fmaf(v, v, f[r & 3]);
                    }
                    s = (double)((f[0] + f[1]) + (f[2] + f[3]));
                }
#pragma unroll
                for (int c = 0; c < RR; c += 8)
                    if (RL + c + 8 > t) {
                        float q = 0.f;
#pragma unroll
                        for (int r = c; r < c + 8 && r < RR; ++r) {
                            if (RL + r < BS_LMAX) y[r] = fmaf(-dt, xf[RL + r], y[r]);
                            const float v = (RL + r > t) ? y[r] : 0.f;
                            q = fmaf(v, v, q);
                        }
                        s += (double)q;
                    }
                nu = s;
                if (j == wj) {
                    alive = false;
                    a.pos[roff + j] = t;
                }
            }
        }
        if (j == 0) {
            a.J[(int64_t)p * k + t] = wj;
            a.beta[(int64_t)p * k + t] = beta;
        }
        // no barrier here: s_nu / s_j are read before the publication barrier
        // and next written after it; xf and s_hh are read in this update and
        // next written after the next step's argmax barrier, which every
        // thread reaches only when its update is done
    }
    // top keff rows of every column -> Rt (FP64); the pivots' diagonal is beta
    if (j < n) {
        double* Rj = a.Rt + roff * (int64_t)k + (int64_t)j * k;
        for (int i = 0; i < min(keff, RL); ++i) Rj[i] = (double)ylds[i * NT + j];
#pragma unroll
        for (int r = 0; r < RR; ++r)
            if (RL + r < keff) Rj[RL + r] = (double)y[r];
    }
    if (j == 0) {
        a.keff[p] = keff;
        for (int t = keff; t < k; ++t) a.J[(int64_t)p * k + t] = -1;
        if (a.status) a.status[p] = nonfinite ? IDS_ENONFINITE : (rankdef ? IDS_ERANKDEF : IDS_OK);
    }
}

// ---------------------------------------------------------------------------
// K3: interpolation matrix per problem on the FP64 matrix cores
// ---------------------------------------------------------------------------
// T = R11^{-1} R12 by block back-substitution over 16-row blocks,
//   T_i = R_ii^{-1} (R12_i - sum_{l > i} R_il T_l),   i = nb - 1, ..., 0,
// with R11 padded to 16 nb rows (identity past keff).  R11[t][t] is the FP64
// beta of step t, the entries above the diagonal are the top rows of the
// pivot columns (Rt).  The workgroup stages the blocks R_il (l > i, negated)
// and the inverses of the 16 x 16 diagonal blocks (back-substitution, one
// thread per column) in LDS, every block column-major so that the MFMA A
// operand of K slice q is the 64 consecutive doubles 64 q .. 64 q + 63.  Each
// wave then takes tiles of 16 consecutive columns of P_p on its own (no
// barrier), so its stores write whole 128-byte row segments: the tile's nb
// accumulators stay in registers, v_mfma_f64_16x16x4f64 forms every product
// (4 K slices per block), and since the FP64 result layout (register r: row
// 4 r + lane / 16, column lane % 16) is the B operand layout of K slice r, a
// solved block T_l feeds the later products without any exchange.  Columns
// are independent in every product, so a column's result does not depend on
// the tile it lands in; a pivot column J[t] in the tile gets e_t exactly
// (its right-hand side is not loaded).  Two waves per SIMD (256 VGPRs).
constexpr int BT_THREADS = 256;
constexpr int BT_NBMAX = 8;  // 16-row blocks (k <= 128)
typedef double v4f64 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int tri_blk(int i, int l) { return l * (l + 1) / 2 + i; }  // block (i, l), i <= l

size_t batched_solve_lds(int64_t k) {
    const int nb = (int)((k + 15) / 16);
    return sizeof(double) * 256 * (size_t)(nb * (nb + 1) / 2);
}

__global__ __launch_bounds__(BT_THREADS, 2) void batched_solve_kernel(BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) double blk[];  // nb (nb + 1) / 2 blocks of 256
    __shared__ int32_t Js[16 * BT_NBMAX];
    const int p = a.order[blockIdx.x];
    const BProb pr = a.prob[p];
    const int n = pr.n, k = (int)a.k;
    const int keff = (int)a.keff[p];
    const int nb = (keff + 15) / 16;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t* J = a.J + (int64_t)p * k;
    const double* bt = a.beta + (int64_t)p * k;
    const double* Rt = a.Rt + pr.r_off * (int64_t)k;
    const int32_t* pos = a.pos + pr.r_off;
    double* P = a.P + pr.p_off;
    for (int t = tid; t < 16 * nb; t += BT_THREADS) Js[t] = t < keff ? (int32_t)J[t] : 0;
    __syncthreads();
    // R11 blocks: element (m, kk) of block (i, l) = R11[16 i + m][16 l + kk] at
    // kk * 16 + m; thread tid holds element (tid & 15, tid >> 4) of every
    // block, and the loads of 8 blocks are issued before any is stored
    const int nblk = nb * (nb + 1) / 2;
    {
        const int m = tid & 15, kk = tid >> 4;
        for (int b0 = 0; b0 < nblk; b0 += 8) {
            double v[8];
            int rr[8], cc[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = min(b0 + u, nblk - 1);
                int l = 0;
                while ((l + 1) * (l + 2) / 2 <= b) ++l;
                rr[u] = 16 * (b - l * (l + 1) / 2) + m;
                cc[u] = 16 * l + kk;
                const bool above = rr[u] < cc[u] && cc[u] < keff;
                v[u] = Rt[above ? (int64_t)Js[cc[u]] * k + rr[u] : 0];
            }
            asm volatile("" ::: "memory");
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (b0 + u >= nblk) break;
                const int r = rr[u], c = cc[u];
                double x;
                if (r < keff && c < keff)
                    x = r < c ? v[u] : (r == c ? bt[r] : 0.0);
                else
                    x = (r == c) ? 1.0 : 0.0;
                // off-diagonal blocks negated (the updates subtract), diagonal
                // blocks as they are (inverted below)
                blk[256 * (b0 + u) + tid] = ((r >> 4) == (c >> 4)) ? x : -x;
            }
        }
    }
    __syncthreads();
    // diagonal blocks -> inverses: thread (di, dc) solves R_ii x = e_dc
    {
        const int di = tid >> 4, dc = tid & 15;
        double x[16];
        const double* D = blk + 256 * tri_blk(min(di, BT_NBMAX - 1), min(di, BT_NBMAX - 1));
        if (di < nb) {
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
            double* Dw = blk + 256 * tri_blk(di, di);
#pragma unroll
            for (int r = 0; r < 16; ++r) Dw[dc * 16 + r] = x[r];
        }
    }
    __syncthreads();
    // tiles of 16 consecutive columns, so every store below writes four
    // contiguous 128-byte row segments of P: a non-pivot column's lane solves
    // R11 x = R[0:keff, j]; a pivot column's lane (chosen at step t) writes e_t
    const int col = lane & 15, rq = lane >> 4;
    for (int t0 = 16 * w; t0 < n; t0 += 16 * (BT_THREADS / 64)) {
        const int jj = t0 + col;
        const int j = min(jj, n - 1);
        const int pj = pos[j];
        v4f64 acc[BT_NBMAX];
        // right-hand sides R[0:keff, j] (clamped loads, all in flight, then
        // masked); pivot columns load nothing
#pragma unroll
        for (int i = 0; i < BT_NBMAX; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[i][r] = (pj < 0) ? Rt[(int64_t)j * k + min(16 * i + 4 * r + rq, max(keff - 1, 0))] : 0.0;
        asm volatile("" ::: "memory");
#pragma unroll
        for (int i = 0; i < BT_NBMAX; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][r] = (16 * i + 4 * r + rq < keff) ? acc[i][r] : 0.0;
#pragma unroll
        for (int i = BT_NBMAX - 1; i >= 0; --i) {
            if (i >= nb) continue;
#pragma unroll
            for (int l = i + 1; l < BT_NBMAX; ++l) {
                if (l >= nb) continue;
                const double* A = blk + 256 * tri_blk(i, l);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[64 * q + lane], acc[l][q], acc[i], 0, 0, 0);
            }
            const double* Di = blk + 256 * tri_blk(i, i);
            v4f64 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 4; ++q) x = __builtin_amdgcn_mfma_f64_16x16x4f64(Di[64 * q + lane], acc[i][q], x, 0, 0, 0);
            acc[i] = x;
        }
        if (jj < n) {
#pragma unroll
            for (int i = 0; i < BT_NBMAX; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * i + 4 * r + rq;
                    if (row < k)
                        P[(int64_t)row * n + j] = (pj >= 0) ? (row == pj ? 1.0 : 0.0) : (row < keff ? acc[i][r] : 0.0);
                }
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
ids_status batched_plan_bytes(int64_t nprob, size_t* bytes) {
    size_t a, b, c;
    *bytes = plan_layout(nprob, &a, &b, &c);
    return IDS_OK;
}

ids_status batched_plan(int64_t nprob, const int64_t* m, const int64_t* n, int64_t k, int64_t l, int64_t l1max,
                        void* plan, size_t plan_bytes, size_t* ws_bytes, hipStream_t st) {
    size_t op, o1, o2;
    const size_t need = plan_layout(nprob, &op, &o1, &o2);
    if (plan_bytes < need) {
        set_error("plan buffer too small: need " + std::to_string(need) + " bytes");
        return IDS_EWORKSPACE;
    }
    std::vector<char> host(need, 0);
    BatchHdr* h = (BatchHdr*)host.data();
    BProb* pr = (BProb*)(host.data() + op);
    int32_t* ord1 = (int32_t*)(host.data() + o1);
    int32_t* ord2 = (int32_t*)(host.data() + o2);
    int64_t a_off = 0, y_off = 0, p_off = 0, r_off = 0;
    int32_t max_n = 0, max_m = 0;
    for (int64_t q = 0; q < nprob; ++q) {
        pr[q].m = (int32_t)m[q];
        pr[q].n = (int32_t)n[q];
        pr[q].l1 = (int32_t)std::min<int64_t>(m[q], l1max);
        pr[q].pad = 0;
        pr[q].a_off = a_off;
        pr[q].y_off = y_off;
        pr[q].p_off = p_off;
        pr[q].r_off = r_off;
        a_off += m[q] * n[q];
        y_off += l * n[q];
        p_off += k * n[q];
        r_off += n[q];
        max_n = std::max<int32_t>(max_n, (int32_t)n[q]);
        max_m = std::max<int32_t>(max_m, (int32_t)m[q]);
    }
    h->nprob = nprob;
    h->k = k;
    h->l = l;
    h->l1max = l1max;
    h->y_elems = y_off;
    h->r_elems = r_off;
    h->max_n = max_n;
    h->max_m = max_m;
    // largest problems first (longest-processing-time order for the dispatcher)
    std::vector<int32_t> idx(nprob);
    for (int64_t q = 0; q < nprob; ++q) idx[q] = (int32_t)q;
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return m[x] * n[x] > m[y] * n[y]; });
    std::copy(idx.begin(), idx.end(), ord1);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return n[x] > n[y]; });
    std::copy(idx.begin(), idx.end(), ord2);
    if (hipMemcpyAsync(plan, host.data(), need, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("batched plan upload failed");
        return IDS_EHIP;
    }
    // workspace: Y (FP32), Rt (FP64 n x k per problem), pos (int32), beta (FP64)
    *ws_bytes = align256(sizeof(float) * (size_t)y_off) + align256(sizeof(double) * (size_t)r_off * k) +
                align256(sizeof(int32_t) * (size_t)r_off) + align256(sizeof(double) * (size_t)nprob * k) +
                align256(sizeof(uint16_t) * (size_t)l * l1max);  // G drawn on the device when none is given
    return IDS_OK;
}

// Two extra streams per device (default priority, non-blocking) on which the
// 512- and 256-thread CPQR launches run beside the 1024-thread one, so the
// smaller problems fill the CUs the largest ones leave idle; created once (a
// failed creation is undone and remembered: that device then runs every
// class on the caller's stream).  The lock keeps one call's event records
// and waits together.
struct CpqrSide {
    hipStream_t s[2] = {nullptr, nullptr};
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    int state = 0;  // 0: not tried, 1: ready, -1: creation failed
};
static std::mutex g_side_mu;
static CpqrSide g_side[64];

static void side_destroy(CpqrSide& c) {
    for (auto& x : c.s)
        if (x) {
            hipStreamSynchronize(x);
            hipStreamDestroy(x);
            x = nullptr;
        }
    for (auto& e : c.ev)
        if (e) {
            hipEventDestroy(e);
            e = nullptr;
        }
}

static CpqrSide* cpqr_side() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    CpqrSide& c = g_side[dev];
    if (c.state == 0) {
        bool ok = true;
        for (auto& x : c.s) ok = ok && hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess;
        for (auto& e : c.ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (!ok) side_destroy(c);
        c.state = ok ? 1 : -1;
    }
    return c.state == 1 ? &c : nullptr;
}

// Library teardown (ids_finalize): the side streams of every device, after
// the work queued on them has finished.
void batched_release() {
    std::lock_guard<std::mutex> g(g_side_mu);
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    for (int d = 0; d < 64; ++d) {
        if (g_side[d].state != 1) continue;
        if (hipSetDevice(d) == hipSuccess) side_destroy(g_side[d]);
        g_side[d].state = 0;
    }
    if (have) hipSetDevice(cur);
}

ids_status batched_run(int64_t nprob, const void* plan, int64_t k, int64_t l, int64_t l1max, uint64_t seed,
                       double tol, const void* A, const void* G, int64_t* J, double* P, int64_t* keff,
                       int32_t* status, void* ws, size_t ws_bytes, int64_t a_elems, int64_t y_elems,
                       int64_t r_elems, hipStream_t st, bool prof) {
    size_t op, o1, o2;
    plan_layout(nprob, &op, &o1, &o2);
    BatchArgs a;
    a.prob = (const BProb*)((const char*)plan + op);
    a.nprob = nprob;
    a.k = k;
    a.l = l;
    a.l1max = l1max;
    a.seed = seed;
    a.tol2 = tol * tol;
    a.A = (const uint16_t*)A;
    a.a_elems = a_elems;
    a.a_al16 = ((uintptr_t)A & 15) == 0;
    a.G = (const uint16_t*)G;
    a.g_vec = (l1max % 8 == 0) && (((uintptr_t)G & 15) == 0);
    char* p = (char*)ws;
    a.Y = (float*)p;
    p += align256(sizeof(float) * (size_t)y_elems);
    a.Rt = (double*)p;
    p += align256(sizeof(double) * (size_t)r_elems * k);
    a.pos = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)r_elems);
    a.beta = (double*)p;
    p += align256(sizeof(double) * (size_t)nprob * k);
    uint16_t* gdraw = (uint16_t*)p;
    a.J = J;
    a.P = P;
    a.keff = keff;
    a.status = status;
    (void)ws_bytes;
    if (!G) {
        // the shared l x l1max Gaussian from the stream (seed, 0 | 2^63), BF16
        ids_status s = gaussian_fill(seed, 0, l, l1max, IDS_BF16, gdraw, st);
        if (s) return s;
        a.G = gdraw;
        a.g_vec = (l1max % 8 == 0);
    }
    {
        ProfScope ps(prof ? PK_CS : -1, st);
        a.order = (const int32_t*)((const char*)plan + o1);
        hipLaunchKernelGGL(batched_sketch_kernel, dim3((unsigned)nprob), dim3(BS_THREADS), 0, st, a);
    }
    {
        // the problems of each width class (n_p in (512, 1024], (256, 512],
        // (0, 256]) go through their CPQR on a stream of their own, so the
        // smaller classes fill the CUs the largest leave idle
        ProfScope ps(prof ? PK_CPQR : -1, st);
        a.order = (const int32_t*)((const char*)plan + o2);
        std::lock_guard<std::mutex> g(g_side_mu);
        CpqrSide* side = cpqr_side();
        hipStream_t s512 = st, s256 = st;
        if (side) {  // else all on the caller's stream, one after another
            // nothing is queued on the side streams yet: on failure here the
            // classes simply stay on the caller's stream
            if (hipEventRecord(side->ev[0], st) == hipSuccess &&
                hipStreamWaitEvent(side->s[0], side->ev[0], 0) == hipSuccess &&
                hipStreamWaitEvent(side->s[1], side->ev[0], 0) == hipSuccess) {
                s512 = side->s[0];
                s256 = side->s[1];
            }
        }
        // rows in LDS of the 512- and 256-thread classes: tuned knobs (36 or 0)
        const bool lds512 = tune_get("batched.rl512", BC_RL) != 0, lds256 = tune_get("batched.rl256", BC_RL) != 0;
        hipLaunchKernelGGL((batched_cpqr_kernel<1024, BC_RL>), dim3((unsigned)nprob), dim3(1024),
                           sizeof(float) * BC_RL * 1024, st, a, 512);
        if (lds512)
            hipLaunchKernelGGL((batched_cpqr_kernel<512, BC_RL>), dim3((unsigned)nprob), dim3(512),
                               sizeof(float) * BC_RL * 512, s512, a, 256);
        else
            hipLaunchKernelGGL((batched_cpqr_kernel<512, 0>), dim3((unsigned)nprob), dim3(512), 0, s512, a, 256);
        if (lds256)
            hipLaunchKernelGGL((batched_cpqr_kernel<256, BC_RL>), dim3((unsigned)nprob), dim3(256),
                               sizeof(float) * BC_RL * 256, s256, a, 0);
        else
            hipLaunchKernelGGL((batched_cpqr_kernel<256, 0>), dim3((unsigned)nprob), dim3(256), 0, s256, a, 0);
        if (s512 != st) {
            // join: the caller's stream waits for both side streams; if the
            // event route fails, wait for them on the host instead, so no work
            // on J, P or the workspace is still running when this returns
            if (hipEventRecord(side->ev[1], side->s[0]) != hipSuccess ||
                hipEventRecord(side->ev[2], side->s[1]) != hipSuccess ||
                hipStreamWaitEvent(st, side->ev[1], 0) != hipSuccess ||
                hipStreamWaitEvent(st, side->ev[2], 0) != hipSuccess) {
                hipStreamSynchronize(side->s[0]);
                hipStreamSynchronize(side->s[1]);
                set_error("batched ID: stream join failed (side streams synchronised on the host)");
                return IDS_EHIP;
            }
        }
    }
    {
        // interpolation matrices of all problems (largest n first)
        ProfScope ps(prof ? PK_TRSM : -1, st);
        a.order = (const int32_t*)((const char*)plan + o2);
        hipLaunchKernelGGL(batched_solve_kernel, dim3((unsigned)nprob), dim3(BT_THREADS), batched_solve_lds(k), st,
                           a);
    }
    return check_launch("batched ID");
}

// ---------------------------------------------------------------------------
// the whole batched call captured once into a HIP graph and replayed
// ---------------------------------------------------------------------------
// Captured on a private stream: the side streams join the capture through the
// fork event, so the graph holds the sketch, the three concurrent CPQR
// launches and the solve with the fork / join as edges.  No memset or
// allocation is recorded; replays reuse the caller's buffers.
struct BatchedGraph {
    hipGraphExec_t exec = nullptr;
};

ids_status batched_graph_create(int64_t nprob, const void* plan, int64_t k, int64_t l, int64_t l1max, uint64_t seed,
                                double tol, const void* A, const void* G, int64_t* J, double* P, int64_t* keff,
                                int32_t* status, void* ws, size_t ws_bytes, int64_t a_elems, int64_t y_elems,
                                int64_t r_elems, void** out) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        set_error("batched graph: stream creation failed");
        return IDS_EHIP;
    }
    ids_status s = IDS_OK;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        set_error("batched graph: hipStreamBeginCapture failed");
        s = IDS_EHIP;
    } else {
        s = batched_run(nprob, plan, k, l, l1max, seed, tol, A, G, J, P, keff, status, ws, ws_bytes, a_elems, y_elems,
                        r_elems, cs, false);
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        if (!s && (e != hipSuccess || !graph)) {
            set_error(std::string("batched graph: hipStreamEndCapture: ") + hipGetErrorString(e));
            s = IDS_EHIP;
        }
    }
    BatchedGraph* bg = nullptr;
    if (!s) {
        bg = new BatchedGraph;
        if (hipGraphInstantiate(&bg->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            set_error("batched graph: hipGraphInstantiate failed");
            delete bg;
            bg = nullptr;
            s = IDS_EHIP;
        }
    }
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cs);
    if (!s) *out = bg;
    return s;
}

ids_status batched_graph_launch(void* g, hipStream_t st) {
    BatchedGraph* bg = (BatchedGraph*)g;
    const hipError_t e = hipGraphLaunch(bg->exec, st);
    if (e != hipSuccess) {
        set_error(std::string("batched graph launch: ") + hipGetErrorString(e));
        return IDS_EHIP;
    }
    return IDS_OK;
}

void batched_graph_destroy(void* g) {
    BatchedGraph* bg = (BatchedGraph*)g;
    if (!bg) return;
    if (bg->exec) hipGraphExecDestroy(bg->exec);
    delete bg;
}

}  // namespace ids

// CountSketch Y1 = S A = Phi D A (Section 1.3; Algorithm 2, "compute the
// sketch implicitly") for dense row-major and CSR matrices on gfx950.
//
// Design (bucket owner, no atomics for dense input):
//   1. plan: every row i gets (h(i), D_ii) from the counter-based hash; a
//      stable counting sort groups the signed row codes by bucket, rows of a
//      bucket in increasing order (plan_count -> plan_rowscan -> plan_offsets
//      -> plan_place; one workgroup per plan for small inputs).
//   2. dense gather: workgroup (panel, bucket) walks the rows of its bucket and
//      accumulates them in registers, 16-byte loads per lane, several rows in
//      flight, then writes its slice of Y1 once.  Every entry of Y1 is the sum
//      of its bucket's signed rows in increasing row order, i.e. the same
//      sequence of additions as the textbook definition, so the result is
//      deterministic (and bit-identical to a sequential FP64 evaluation when
//      the accumulation type is FP64).
//   3. CSR: workgroup (bucket, row chunk) scatters the stored entries of its
//      rows into an LDS copy of the bucket's Y1 row (FP64 LDS atomics), then
//      adds it to Y1 in HBM (rows wider than LDS: global atomics).
//   4. CSR with IDS_DETERMINISTIC: the entries are binned stably by (bucket,
//      column range) and each range's sums are formed in row order, entries
//      sharing a column in lane order -- the definition's order, so the FP64
//      result equals a sequential evaluation bit for bit.
#include <algorithm>
#include "common.hpp"
#include "kernels.hpp"
#include "tune.hpp"

namespace ids {

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct PlanArgs {
    int64_t m;
    uint32_t L;
    uint64_t key;
    const int64_t* fr_pi;  // modified hash (optional)
    const int32_t* fr_x;
    int32_t seg_rows;      // rows per wave segment (multiple of 64)
    int32_t nseg;
    int32_t* seg;          // L x nseg counts -> offsets (bucket-major)
    int32_t* off;          // L + 1
    int32_t* rows;         // m signed row codes
};

__device__ __forceinline__ void plan_hash(const PlanArgs& a, int64_t i, uint32_t& b, bool& neg) {
    hash_row(a.key, i, a.L, b, neg);
    if (a.fr_pi) {
        int64_t q = a.fr_pi[i];
        b = (q < (int64_t)a.L) ? (uint32_t)q : (uint32_t)a.fr_x[q];
    }
}

// one wave per segment; LDS histogram of L counters
__global__ __launch_bounds__(64) void plan_count_kernel(PlanArgs a) {
    extern __shared__ int32_t hist[];
    const int s = blockIdx.x;
    const int lane = threadIdx.x;
    for (uint32_t b = lane; b < a.L; b += 64) hist[b] = 0;
    __syncthreads();
    const int64_t r0 = (int64_t)s * a.seg_rows;
    const int64_t r1 = min(a.m, r0 + a.seg_rows);
    for (int64_t i = r0 + lane; i < r1; i += 64) {
        uint32_t b;
        bool neg;
        plan_hash(a, i, b, neg);
        atomicAdd(&hist[b], 1);
    }
    __syncthreads();
    for (uint32_t b = lane; b < a.L; b += 64) a.seg[(int64_t)b * a.nseg + s] = hist[b];
}

// Offsets of the bucket-major L x nseg count matrix, in two steps:
//   plan_rowscan: one wave per bucket b, exclusive scan of row b over the
//                 segments (in place) and the bucket total tot[b];
//   plan_offsets: one workgroup, exclusive scan of the L totals -> off[b].
// plan_place then places row i of segment s at off[b] + seg[b][s] + rank.
__global__ __launch_bounds__(64) void plan_rowscan_kernel(PlanArgs a, int32_t* tot) {
    constexpr int U = 16;  // loads in flight per lane
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    int32_t* row = a.seg + (int64_t)b * a.nseg;
    int32_t carry = 0;
    for (int s0 = 0; s0 < a.nseg; s0 += 64 * U) {
        int32_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = s0 + 64 * u + lane;
            v[u] = s < a.nseg ? row[s] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = s0 + 64 * u + lane;
            int32_t x = v[u];
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (s < a.nseg) row[s] = carry + x - v[u];
            carry += __shfl(x, 63, 64);
        }
    }
    if (lane == 0) tot[b] = carry;
}

__global__ __launch_bounds__(1024) void plan_offsets_kernel(PlanArgs a, const int32_t* tot) {
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int64_t L = a.L;
    const int64_t per = (L + 1023) / 1024;
    const int64_t b0 = t * per, b1 = min(L, b0 + per);
    int32_t sum = 0;
    for (int64_t q = b0; q < b1; ++q) sum += tot[q];
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int32_t v = (t >= o) ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = (t == 0) ? 0 : part[t - 1];
    for (int64_t q = b0; q < b1; ++q) {
        a.off[q] = run;
        run += tot[q];
    }
    if (t == 0) a.off[L] = (int32_t)a.m;
}

// Lanes of the wave holding the same bucket b (valid lanes only), found with
// one ballot per bit of b: rank = how many of them precede this lane, same =
// how many there are -- the stable order of a 64-row chunk inside each bucket.
// Every lane of the wave must take part; nbits covers the largest bucket.
__device__ __forceinline__ void wave_bucket_rank(uint32_t b, bool valid, int nbits, int& rank, int& same) {
    uint64_t peers = __ballot(valid);
    for (int k = 0; k < nbits; ++k) {
        const bool bit = (b >> k) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    const int lane = threadIdx.x & 63;
    rank = __popcll(peers & ((1ull << lane) - 1ull));
    same = __popcll(peers);
}

constexpr int PLAN_FUSED_L = 1024;  // up to this many buckets the placement scans the totals itself

// one wave per segment: stable placement (rows of a bucket in increasing order).
// With tot != nullptr (few buckets) the bucket offsets are not read from off[]
// but scanned from the bucket totals by every workgroup (the first one also
// stores them to off[]), which saves the separate offsets launch.
__global__ __launch_bounds__(64) void plan_place_kernel(PlanArgs a, const int32_t* tot) {
    extern __shared__ int32_t run[];
    const int s = blockIdx.x;
    const int lane = threadIdx.x;
    const int nbits = (a.L > 1) ? 32 - __builtin_clz(a.L - 1) : 0;
    if (tot) {
        // lane: the buckets [b0, b1), at most PLAN_FUSED_L / 64 of them, all
        // loaded together from clamped indices
        constexpr int CBM = PLAN_FUSED_L / 64;
        const uint32_t cb = (a.L + 63) / 64;
        const uint32_t b0 = min(a.L, lane * cb), b1 = min(a.L, b0 + cb);
        int32_t tv[CBM], sv[CBM];
#pragma unroll
        for (int u = 0; u < CBM; ++u) {
            const uint32_t bb = min(b0 + u, a.L - 1);
            tv[u] = tot[bb];
            sv[u] = a.seg[(int64_t)bb * a.nseg + s];
        }
        asm volatile("" ::: "memory");
        int32_t sum = 0;
#pragma unroll
        for (int u = 0; u < CBM; ++u) sum += (b0 + u < b1) ? tv[u] : 0;
        int32_t x = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        int32_t base = x - sum;  // exclusive prefix of this lane's chunk
#pragma unroll
        for (int u = 0; u < CBM; ++u) {
            const uint32_t b = b0 + u;
            if (b < b1) {
                if (s == 0) a.off[b] = base;
                run[b] = base + sv[u];
                base += tv[u];
            }
        }
        if (s == 0 && lane == 0) a.off[a.L] = (int32_t)a.m;
    } else {
        constexpr int U = 8;  // loads in flight per lane
        for (uint32_t b0 = 0; b0 < a.L; b0 += 64 * U) {
            int32_t o[U], c[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t b = b0 + 64 * u + lane;
                o[u] = b < a.L ? a.off[b] : 0;
                c[u] = b < a.L ? a.seg[(int64_t)b * a.nseg + s] : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t b = b0 + 64 * u + lane;
                if (b < a.L) run[b] = o[u] + c[u];
            }
        }
    }
    __syncthreads();
    const int64_t r0 = (int64_t)s * a.seg_rows;
    const int64_t r1 = min(a.m, r0 + a.seg_rows);
    for (int64_t c0 = r0; c0 < r1; c0 += 64) {
        const int64_t i = c0 + lane;
        const bool valid = i < r1;
        uint32_t b = 0xffffffffu;
        bool neg = false;
        if (valid) plan_hash(a, i, b, neg);
        int rank, same;
        wave_bucket_rank(b, valid, nbits, rank, same);
        int32_t base = 0;
        if (valid) base = run[b];
        __syncthreads();
        if (valid) {
            a.rows[base + rank] = encode_row(i, neg);
            if (rank == same - 1) run[b] = base + same;
        }
        __syncthreads();
    }
}

// Small inputs (m <= PLAN_SMALL_M): the whole plan in one workgroup per plan,
// one launch for several plans.  PS_W waves each own a contiguous quarter of
// the rows: per-wave LDS histograms, one scan that turns them into per-wave
// start offsets (bucket-major, waves in row order, so placement stays
// stable), then each wave places its rows 64 at a time in increasing order.
constexpr int PS_W = 4;
constexpr int64_t PLAN_SMALL_M = 16384;
constexpr int64_t PLAN_SMALL_L = 6144;  // PS_W x L int32 counters in LDS
constexpr int PLAN_MANY = 8;
struct PlanSmallArgs {
    PlanArgs p[PLAN_MANY];
};

__global__ __launch_bounds__(64 * PS_W) void plan_small_kernel(PlanSmallArgs s) {
    extern __shared__ int32_t h[];  // PS_W x L
    __shared__ int32_t part[64 * PS_W];
    const PlanArgs& a = s.p[blockIdx.x];
    constexpr int NT = 64 * PS_W;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t L = a.L;
    for (int64_t e = tid; e < PS_W * L; e += NT) h[e] = 0;
    __syncthreads();
    const int64_t per = (a.m + PS_W - 1) / PS_W;
    const int64_t r0 = min(a.m, w * per), r1 = min(a.m, r0 + per);
    for (int64_t i = r0 + lane; i < r1; i += 64) {
        uint32_t b;
        bool neg;
        plan_hash(a, i, b, neg);
        atomicAdd(&h[w * L + b], 1);
    }
    __syncthreads();
    // thread t owns buckets [t cb, t cb + cb): totals, block scan, then
    // h[w][b] <- start of wave w's rows of bucket b
    const int64_t cb = (L + NT - 1) / NT;
    const int64_t b0 = min(L, tid * cb), b1 = min(L, b0 + cb);
    int32_t sum = 0;
    for (int64_t b = b0; b < b1; ++b)
#pragma unroll
        for (int q = 0; q < PS_W; ++q) sum += h[q * L + b];
    part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < NT; o <<= 1) {
        const int32_t v = (tid >= o) ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - sum;
    for (int64_t b = b0; b < b1; ++b) {
        a.off[b] = run;
#pragma unroll
        for (int q = 0; q < PS_W; ++q) {
            const int32_t c = h[q * L + b];
            h[q * L + b] = run;
            run += c;
        }
    }
    if (tid == NT - 1) a.off[L] = (int32_t)a.m;
    __syncthreads();
    // stable placement, wave w over its rows in order (no other wave touches
    // h[w][.], and the read of a bucket's start precedes its update in the wave)
    int32_t* hw = h + w * L;
    const int nbits = (L > 1) ? 32 - __builtin_clz((uint32_t)(L - 1)) : 0;
    for (int64_t c0 = r0; c0 < r1; c0 += 64) {
        const int64_t i = c0 + lane;
        const bool valid = i < r1;
        uint32_t b = 0xffffffffu;
        bool neg = false;
        if (valid) plan_hash(a, i, b, neg);
        int rank, same;
        wave_bucket_rank(b, valid, nbits, rank, same);
        const int32_t base = valid ? hw[b] : 0;
        if (valid) {
            a.rows[base + rank] = encode_row(i, neg);
            if (rank == same - 1) hw[b] = base + same;
        }
    }
}

static bool plan_is_small(const PlanShape& ps) { return ps.m <= PLAN_SMALL_M && ps.L <= PLAN_SMALL_L; }

static PlanArgs plan_args(const PlanShape& ps, uint64_t key, const int64_t* fr_pi, const int32_t* fr_x,
                          const PlanBufs& pb) {
    PlanArgs a;
    a.m = ps.m;
    a.L = (uint32_t)ps.L;
    a.key = key;
    a.fr_pi = fr_pi;
    a.fr_x = fr_x;
    a.seg_rows = ps.seg_rows;
    a.nseg = ps.nseg;
    a.seg = pb.seg;
    a.off = pb.off;
    a.rows = pb.rows;
    return a;
}

ids_status plan_build_many(int count, const PlanShape* ps, const uint64_t* keys, const PlanBufs* pb,
                           hipStream_t st) {
    bool small = count <= PLAN_MANY;
    int64_t Lmax = 0;
    for (int q = 0; q < count; ++q) {
        small = small && plan_is_small(ps[q]);
        Lmax = std::max<int64_t>(Lmax, ps[q].L);
    }
    if (!small) {
        for (int q = 0; q < count; ++q)
            if (ids_status s = plan_build(ps[q], keys[q], nullptr, nullptr, pb[q], st)) return s;
        return IDS_OK;
    }
    PlanSmallArgs sa;
    for (int q = 0; q < count; ++q) sa.p[q] = plan_args(ps[q], keys[q], nullptr, nullptr, pb[q]);
    hipLaunchKernelGGL(plan_small_kernel, dim3(count), dim3(64 * PS_W), sizeof(int32_t) * PS_W * Lmax, st, sa);
    return check_launch("countsketch plan");
}

ids_status plan_build(const PlanShape& ps, uint64_t key, const int64_t* fr_pi, const int32_t* fr_x,
                      const PlanBufs& pb, hipStream_t st) {
    PlanArgs a = plan_args(ps, key, fr_pi, fr_x, pb);
    if (plan_is_small(ps)) {
        PlanSmallArgs sa;
        sa.p[0] = a;
        hipLaunchKernelGGL(plan_small_kernel, dim3(1), dim3(64 * PS_W), sizeof(int32_t) * PS_W * ps.L, st, sa);
        return check_launch("countsketch plan");
    }
    size_t lds = sizeof(int32_t) * (size_t)ps.L;
    hipLaunchKernelGGL(plan_count_kernel, dim3(ps.nseg), dim3(64), lds, st, a);
    hipLaunchKernelGGL(plan_rowscan_kernel, dim3((unsigned)ps.L), dim3(64), 0, st, a, pb.tot);
    if (ps.L <= PLAN_FUSED_L) {  // offsets scanned inside the placement
        hipLaunchKernelGGL(plan_place_kernel, dim3(ps.nseg), dim3(64), lds, st, a, (const int32_t*)pb.tot);
    } else {
        hipLaunchKernelGGL(plan_offsets_kernel, dim3(1), dim3(1024), 0, st, a, (const int32_t*)pb.tot);
        hipLaunchKernelGGL(plan_place_kernel, dim3(ps.nseg), dim3(64), lds, st, a, (const int32_t*)nullptr);
    }
    return check_launch("countsketch plan");
}

PlanShape plan_shape(int64_t m, int64_t L) {
    PlanShape ps;
    ps.m = m;
    ps.L = L;
    // segments of 256 rows (4 chunks of 64 per wave); keep the L x nseg count
    // matrix at most ~4M entries
    int64_t seg = 256;
    int64_t need = (m * L + (int64_t(1) << 22) - 1) >> 22;
    if (need > seg) seg = need;
    seg = (seg + 63) / 64 * 64;
    ps.seg_rows = (int32_t)seg;
    ps.nseg = (int32_t)((m + seg - 1) / seg);
    if (ps.nseg < 1) ps.nseg = 1;
    return ps;
}

size_t plan_bytes(const PlanShape& ps) {
    return align256(sizeof(int32_t) * (size_t)ps.L * ps.nseg) + align256(sizeof(int32_t) * (ps.L + 1)) +
           align256(sizeof(int32_t) * (size_t)ps.m) + align256(sizeof(int32_t) * (size_t)ps.L);
}

PlanBufs plan_carve(const PlanShape& ps, char*& p) {
    PlanBufs pb;
    pb.seg = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)ps.L * ps.nseg);
    pb.off = (int32_t*)p;
    p += align256(sizeof(int32_t) * (ps.L + 1));
    pb.rows = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)ps.m);
    pb.tot = (int32_t*)p;
    p += align256(sizeof(int32_t) * (size_t)ps.L);
    return pb;
}

// ---------------------------------------------------------------------------
// dense gather  (BEGIN dense CountSketch kernel)
// ---------------------------------------------------------------------------
// 16-byte row-segment loads.  A is streamed exactly once, so the loads are
// non-temporal: they do not displace reusable lines in the caches (measured
// +9% sustained read bandwidth on this pass).
typedef float ntf4 __attribute__((ext_vector_type(4)));
typedef double ntd2 __attribute__((ext_vector_type(2)));
typedef unsigned int ntu4 __attribute__((ext_vector_type(4)));

template <typename T, int VEC>
struct VecLoad;
template <>
struct VecLoad<double, 2> {
    using V = ntd2;
    __device__ static V load(const double* p) { return __builtin_nontemporal_load(reinterpret_cast<const V*>(p)); }
    __device__ static void get(const V& v, double* o) { o[0] = v.x; o[1] = v.y; }
};
template <>
struct VecLoad<float, 4> {
    using V = ntf4;
    __device__ static V load(const float* p) { return __builtin_nontemporal_load(reinterpret_cast<const V*>(p)); }
    __device__ static void get(const V& v, float* o) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
};
template <>
struct VecLoad<uint16_t, 8> {
    using V = ntu4;
    __device__ static V load(const uint16_t* p) { return __builtin_nontemporal_load(reinterpret_cast<const V*>(p)); }
    __device__ static void get(const V& v, uint16_t* o) {
        o[0] = v.x & 0xffff; o[1] = v.x >> 16; o[2] = v.y & 0xffff; o[3] = v.y >> 16;
        o[4] = v.z & 0xffff; o[5] = v.z >> 16; o[6] = v.w & 0xffff; o[7] = v.w >> 16;
    }
};

template <typename ACC, typename T>
__device__ __forceinline__ ACC to_acc(T v) { return (ACC)v; }
template <>
__device__ __forceinline__ float to_acc<float, uint16_t>(uint16_t v) { return bf16_to_f32(v); }
template <>
__device__ __forceinline__ double to_acc<double, uint16_t>(uint16_t v) { return (double)bf16_to_f32(v); }

constexpr int CS_THREADS = 256;
constexpr int CS_UNROLL = 8;

template <typename T, typename ACC, int VEC>
__global__ __launch_bounds__(CS_THREADS) void cs_dense_kernel(const T* __restrict__ A, int64_t lda,
                                                                int64_t n, const int32_t* __restrict__ off,
                                                                const int32_t* __restrict__ rows,
                                                                ACC* __restrict__ Y, int64_t rs, int64_t cs) {
    const int b = blockIdx.y;
    const int64_t v = (int64_t)blockIdx.x * CS_THREADS + threadIdx.x;
    const int64_t c0 = v * VEC;
    if (c0 >= n) return;
    const int nvalid = (int)min<int64_t>(VEC, n - c0);
    const int beg = off[b], end = off[b + 1];
    ACC acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = (ACC)0;

    bool done = false;
    if constexpr (VEC > 1) {
        if (nvalid == VEC) {
            done = true;
            using VL = VecLoad<T, VEC>;
            using V = typename VL::V;
            int p = beg;
            for (; p + CS_UNROLL <= end; p += CS_UNROLL) {
                int32_t code[CS_UNROLL];
#pragma unroll
                for (int u = 0; u < CS_UNROLL; ++u) code[u] = rows[p + u];
                V raw[CS_UNROLL];
#pragma unroll
                for (int u = 0; u < CS_UNROLL; ++u) {
                    int64_t i = code[u] >= 0 ? code[u] : -(int64_t)code[u] - 1;
                    raw[u] = VL::load(A + i * lda + c0);
                }
#pragma unroll
                for (int u = 0; u < CS_UNROLL; ++u) {
                    T x[VEC];
                    VL::get(raw[u], x);
                    const bool neg = code[u] < 0;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        ACC xv = to_acc<ACC, T>(x[e]);
                        acc[e] = neg ? acc[e] - xv : acc[e] + xv;
                    }
                }
            }
            for (; p < end; ++p) {
                int32_t code = rows[p];
                int64_t i = code >= 0 ? code : -(int64_t)code - 1;
                V raw = VL::load(A + i * lda + c0);
                T x[VEC];
                VL::get(raw, x);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    ACC xv = to_acc<ACC, T>(x[e]);
                    acc[e] = code < 0 ? acc[e] - xv : acc[e] + xv;
                }
            }
        }
    }
    if (!done) {
        for (int p = beg; p < end; ++p) {
            int32_t code = rows[p];
            int64_t i = code >= 0 ? code : -(int64_t)code - 1;
            const T* row = A + i * lda + c0;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if (e < nvalid) {
                    ACC xv = to_acc<ACC, T>(row[e]);
                    acc[e] = code < 0 ? acc[e] - xv : acc[e] + xv;
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        if (e < nvalid) Y[(int64_t)b * rs + (c0 + e) * cs] = acc[e];
}

// Workgroups resident per CU (tuned knob "cs.dense.wpc", 0 = as many as fit):
// a dynamic LDS reservation the kernel does not use caps residency, so fewer
// buckets stream their rows at once (fewer DRAM pages contended).
static size_t dense_lds_reserve() {
    const int64_t wpc = tune_get("cs.dense.wpc", 0);
    if (wpc <= 0) return 0;
    return std::min<size_t>(lds_limit(), (size_t)(160 * 1024) / (size_t)wpc);
}

template <typename T, typename ACC, int VEC>
static void launch_dense(const void* A, int64_t lda, int64_t n, const PlanBufs& pb, int64_t L, void* Y,
                         int64_t rs, int64_t cs, hipStream_t st) {
    int64_t nvec = (n + VEC - 1) / VEC;
    dim3 grid((unsigned)((nvec + CS_THREADS - 1) / CS_THREADS), (unsigned)L);
    hipLaunchKernelGGL((cs_dense_kernel<T, ACC, VEC>), grid, dim3(CS_THREADS), dense_lds_reserve(), st, (const T*)A,
                       lda, n, (const int32_t*)pb.off, (const int32_t*)pb.rows, (ACC*)Y, rs, cs);
}

ids_status cs_dense(int32_t dtype, int32_t acc, const void* A, int64_t lda, int64_t n, const PlanBufs& pb,
                    int64_t L, void* Y, int64_t rs, int64_t cs, hipStream_t st) {
    const uintptr_t base = (uintptr_t)A;
    auto vec_ok = [&](int esize, int vec) {
        return (base % 16 == 0) && ((lda * esize) % 16 == 0) && vec * esize == 16;
    };
    if (dtype == IDS_F64 && acc == IDS_F64) {
        if (vec_ok(8, 2)) launch_dense<double, double, 2>(A, lda, n, pb, L, Y, rs, cs, st);
        else launch_dense<double, double, 1>(A, lda, n, pb, L, Y, rs, cs, st);
    } else if (dtype == IDS_F32 && acc == IDS_F32) {
        if (vec_ok(4, 4)) launch_dense<float, float, 4>(A, lda, n, pb, L, Y, rs, cs, st);
        else launch_dense<float, float, 1>(A, lda, n, pb, L, Y, rs, cs, st);
    } else if (dtype == IDS_F32 && acc == IDS_F64) {
        if (vec_ok(4, 4)) launch_dense<float, double, 4>(A, lda, n, pb, L, Y, rs, cs, st);
        else launch_dense<float, double, 1>(A, lda, n, pb, L, Y, rs, cs, st);
    } else if (dtype == IDS_BF16 && acc == IDS_F32) {
        if (vec_ok(2, 8)) launch_dense<uint16_t, float, 8>(A, lda, n, pb, L, Y, rs, cs, st);
        else launch_dense<uint16_t, float, 1>(A, lda, n, pb, L, Y, rs, cs, st);
    } else if (dtype == IDS_BF16 && acc == IDS_F64) {
        if (vec_ok(2, 8)) launch_dense<uint16_t, double, 8>(A, lda, n, pb, L, Y, rs, cs, st);
        else launch_dense<uint16_t, double, 1>(A, lda, n, pb, L, Y, rs, cs, st);
    } else {
        set_error("unsupported (input dtype, accumulation dtype) for dense CountSketch");
        return IDS_EDTYPE;
    }
    return check_launch("countsketch dense");
}

// (END dense CountSketch kernel)
// ---------------------------------------------------------------------------
// CSR scatter (FP64)
// ---------------------------------------------------------------------------
constexpr int CSR_THREADS = 1024;
constexpr int CSR_GROUP = 8;  // lanes per row (global-atomic variant)
constexpr int CSR_U = 8;      // 64-entry chunks in flight per wave

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ int64_t wave_incl_scan(int64_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// inclusive max-scan over the wave of values >= 0: row_shr 1, 2, 4, 8 inside
// each row of 16 lanes (lanes shifted in from outside the row read 0), then
// row_bcast15 / row_bcast31 carry the row maxima into the later rows
__device__ __forceinline__ int wave_max_scan(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
    return x;
}

// one batch of up to 64 rows of a bucket's row list, one row per lane: the
// lengths scanned over the wave so that the batch's entries form one sequence
struct CsrBatch {
    int64_t T;      // entries in the batch
    int64_t pre;    // start of this lane's row in the batch's sequence
    int64_t len;    // this lane's row length (0 past the list's end)
    int64_t base2;  // 2 (first entry of the row - pre) + sign bit
    int64_t e_any;  // an entry index every lane may load
};

__device__ __forceinline__ CsrBatch csr_batch(const int64_t* __restrict__ rowptr, bool have, int32_t code,
                                              int64_t nnz) {
    CsrBatch q;
    int64_t e0 = 0;
    q.len = 0;
    if (have) {
        const int64_t i = code >= 0 ? code : -(int64_t)code - 1;
        e0 = rowptr[i];
        q.len = rowptr[i + 1] - e0;
    }
    const int64_t inc = wave_incl_scan(q.len);
    q.T = __shfl(inc, 63, 64);
    q.pre = inc - q.len;
    q.base2 = 2 * (e0 - q.pre) + (code < 0 ? 1 : 0);
    const uint64_t nz = __ballot(q.len > 0);
    q.e_any = nz ? min(__shfl(e0, __ffsll((unsigned long long)nz) - 1, 64), nnz - 1) : 0;
    return q;
}

// entry index (e), validity (ok) and row sign (sg) of this lane's entry in
// each of the CSR_U 64-entry chunks that start at entry B of the batch.  The
// row holding entry Bu is the last row whose start is <= Bu: the row running
// into the chunk comes from one ballot (rows are in start order), each row
// starting inside the chunk announces its index at its start lane with one
// forward permute, and a max-scan over the lanes hands every lane its row.
// Branch-free, so the searches of the chunks interleave; lanes past the end
// get e_any.
__device__ __forceinline__ void csr_chunk_entries(const CsrBatch& q, int64_t B, int64_t nnz, int64_t (&e)[CSR_U],
                                                  bool (&ok)[CSR_U], bool (&sg)[CSR_U]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < CSR_U; ++u) {
        const int64_t Bu = B + 64 * u;
        const int rc = __popcll(__ballot(q.pre <= Bu)) - 1;
        const int64_t d = q.pre - Bu;
        const bool in = q.len > 0 && d > 0 && d < 64;
        const int post = __builtin_amdgcn_ds_permute(in ? (int)d * 4 : 0, in ? lane + 1 : 0);
        const int r = min(63, max(rc, wave_max_scan(post) - 1));
        const int64_t bb = __shfl(q.base2, r, 64);
        const int64_t qq = Bu + lane;
        ok[u] = qq < q.T;
        sg[u] = bb & 1;
        e[u] = ok[u] ? max((int64_t)0, min((bb >> 1) + qq, nnz - 1)) : q.e_any;
    }
}

// LDS-privatised variant: the whole bucket row of Y1 (n <= CSR_LDS_MAX) lives in
// LDS; a workgroup handles positions [p0, p1) of the bucket's row list.
// Entry-parallel: a wave takes a batch of 64 consecutive rows of the list
// (batches are handed out through an LDS counter), scans their lengths, and
// then walks the batch's entries 64 at a time, lane q taking the q-th entry of
// the chunk, so the loads of val / colind are coalesced whatever the row
// lengths are (csr_batch, csr_chunk_entries).  CSR_U chunks are loaded before
// their LDS adds, so that many loads are in flight.
__global__ __launch_bounds__(CSR_THREADS) void cs_csr_lds_kernel(const int64_t* __restrict__ rowptr,
                                                                  const int32_t* __restrict__ colind,
                                                                  const double* __restrict__ val, int64_t m,
                                                                  int64_t n, const int32_t* __restrict__ off,
                                                                  const int32_t* __restrict__ rows, int nchunk,
                                                                  double* __restrict__ Y, int64_t rs, int64_t cs,
                                                                  int use_atomic) {
    extern __shared__ double ybuf[];
    __shared__ int s_next;
    const int b = blockIdx.x / nchunk;
    const int ch = blockIdx.x % nchunk;
    for (int64_t j = threadIdx.x; j < n; j += CSR_THREADS) ybuf[j] = 0.0;
    if (threadIdx.x == 0) s_next = 0;
    __syncthreads();
    const int beg = off[b], end = off[b + 1];
    const int64_t cnt = end - beg;
    const int p0 = beg + (int)(cnt * ch / nchunk);
    const int p1 = beg + (int)(cnt * (ch + 1) / nchunk);
    const int nbat = (p1 - p0 + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int64_t nnz = rowptr[m];  // entry indices are clamped into [0, nnz)

    auto grab = [&]() -> int {
        int bi = 0;
        if (lane == 0) bi = atomicAdd(&s_next, 1);
        return __shfl(bi, 0, 64);
    };
    int bi = grab();
    int32_t code = 0;
    bool have = false;
    if (bi < nbat) {
        const int p = p0 + bi * 64 + lane;
        have = p < p1;
        code = have ? rows[p] : 0;
    }
    while (bi < nbat) {
        const CsrBatch q = csr_batch(rowptr, have, code, nnz);
        // next batch's row codes load while this one is summed
        const int bn = grab();
        bool have_n = false;
        int32_t code_n = 0;
        if (bn < nbat) {
            const int p = p0 + bn * 64 + lane;
            have_n = p < p1;
            code_n = have_n ? rows[p] : 0;
        }
        for (int64_t B = 0; B < q.T; B += 64 * CSR_U) {
            // (1) entry index of every chunk
            int64_t e[CSR_U];
            bool ok[CSR_U], sg[CSR_U];
            csr_chunk_entries(q, B, nnz, e, ok, sg);
            // (2) all loads in flight
            double v[CSR_U];
            int32_t c[CSR_U];
#pragma unroll
            for (int u = 0; u < CSR_U; ++u) {
                v[u] = val[e[u]];
                c[u] = colind[e[u]];
            }
            // (3) signed adds into the LDS row (a column index outside [0, n)
            // is dropped rather than written outside the row)
#pragma unroll
            for (int u = 0; u < CSR_U; ++u)
                if (ok[u] && (uint32_t)c[u] < (uint32_t)n) atomicAdd(&ybuf[c[u]], sg[u] ? -v[u] : v[u]);
        }
        bi = bn;
        code = code_n;
        have = have_n;
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j < n; j += CSR_THREADS) {
        double* dst = Y + (int64_t)b * rs + j * cs;
        if (use_atomic) atomicAdd(dst, ybuf[j]);
        else *dst = ybuf[j];
    }
}

// global-atomic variant for rows wider than LDS
__global__ __launch_bounds__(256) void cs_csr_global_kernel(const int64_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ colind,
                                                           const double* __restrict__ val,
                                                           const int32_t* __restrict__ rows, int64_t m,
                                                           const int32_t* __restrict__ bucket_of_pos,
                                                           double* __restrict__ Y, int64_t rs, int64_t cs) {
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t p = gid / CSR_GROUP;
    const int gl = (int)(gid % CSR_GROUP);
    if (p >= m) return;
    int32_t code = rows[p];
    int64_t i = code >= 0 ? code : -(int64_t)code - 1;
    const int b = bucket_of_pos[p];
    const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
    for (int64_t e = e0 + gl; e < e1; e += CSR_GROUP) {
        double v = val[e];
        atomicAdd(Y + (int64_t)b * rs + (int64_t)colind[e] * cs, code < 0 ? -v : v);
    }
}

// Ordered variant (IDS_DETERMINISTIC): every entry of Y1 is the sum of its
// bucket's signed entries in increasing row order, the entries of one row in
// storage order -- the sequence of additions of the textbook definition, so
// repeated runs agree bit for bit.  Workgroup (bucket, panel) of CSD_W waves;
// wave w owns a contiguous range of at most CSD_WR columns and keeps their
// sums in LDS, so no two waves ever add to one location.  Every wave walks all
// rows of the bucket in list order (64-row batches, 64-entry chunks as above)
// and keeps the entries of its own range.  Inside a chunk, entries that fall
// on the same column are added in lane order, i.e. entry order: each round,
// the lowest pending lane of every tag slot (slot = column mod CSD_SLOTS; a
// minimum over the lane indices) adds its entry and leaves.  A wave's LDS
// operations complete in issue order; the wavefront fences only keep the
// compiler from moving them.  Every wave reads every entry of its bucket, so
// the cost grows with the number of column ranges (n / CSD_WR).
constexpr int CSD_W = 4;
constexpr int CSD_WR = 2048;
constexpr int CSD_SLOTS = 256;

__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// *dst += x for the lanes with pend set (one 64-entry chunk), lanes that share
// a column added in lane order: each round, the lowest pending lane of every
// tag slot (slot = column mod CSD_SLOTS; tg holds the wave's CSD_SLOTS slots,
// 64 = free, and is left free) adds its entry and leaves
__device__ __forceinline__ void ordered_add(bool pend, int col, double* dst, double x, int* tg) {
    const int lane = threadIdx.x & 63;
    const int slot = col & (CSD_SLOTS - 1);
    while (__ballot(pend)) {
        if (pend) __hip_atomic_fetch_min(tg + slot, lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        wave_fence();
        const bool go = pend && __hip_atomic_load(tg + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) == lane;
        if (go) {
            const double y = __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            __hip_atomic_store(dst, y + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
        if (pend) __hip_atomic_store(tg + slot, 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        wave_fence();
        pend = pend && !go;
    }
}

__global__ __launch_bounds__(64 * CSD_W) void cs_csr_ordered_kernel(const int64_t* __restrict__ rowptr,
                                                                    const int32_t* __restrict__ colind,
                                                                    const double* __restrict__ val, int64_t m,
                                                                    const int32_t* __restrict__ off,
                                                                    const int32_t* __restrict__ rows, int npanel,
                                                                    int64_t n, int64_t wr, double* __restrict__ Y,
                                                                    int64_t rs, int64_t cs) {
    __shared__ double acc[CSD_W][CSD_WR];
    __shared__ int tag[CSD_W][CSD_SLOTS];
    const int b = blockIdx.x / npanel;
    const int pnl = blockIdx.x % npanel;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t c0 = ((int64_t)pnl * CSD_W + w) * wr;
    const int64_t c1 = min(n, c0 + wr);
    if (c0 >= c1) return;  // wave-uniform; the waves never synchronise with each other
    double* my = acc[w];
    int* tg = tag[w];
    for (int64_t j = lane; j < c1 - c0; j += 64) __hip_atomic_store(my + j, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    for (int q = lane; q < CSD_SLOTS; q += 64) __hip_atomic_store(tg + q, 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    wave_fence();
    const int beg = off[b], end = off[b + 1];
    const int64_t nnz = rowptr[m];
    for (int p0 = beg; p0 < end; p0 += 64) {
        const int p = p0 + lane;
        const bool have = p < end;
        const CsrBatch q = csr_batch(rowptr, have, have ? rows[p] : 0, nnz);
        for (int64_t B = 0; B < q.T; B += 64 * CSR_U) {
            int64_t e[CSR_U];
            bool ok[CSR_U], sg[CSR_U];
            csr_chunk_entries(q, B, nnz, e, ok, sg);
            double v[CSR_U];
            int32_t c[CSR_U];
#pragma unroll
            for (int u = 0; u < CSR_U; ++u) {
                v[u] = val[e[u]];
                c[u] = colind[e[u]];
            }
#pragma unroll
            for (int u = 0; u < CSR_U; ++u) {
                const bool in = ok[u] && c[u] >= c0 && c[u] < c1;
                ordered_add(in, c[u], my + (in ? c[u] - c0 : 0), sg[u] ? -v[u] : v[u], tg);
            }
        }
    }
    for (int64_t j = c0 + lane; j < c1; j += 64)
        Y[(int64_t)b * rs + j * cs] = __hip_atomic_load(my + (j - c0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Ordered sketch through a stable binning of the entries (IDS_DETERMINISTIC,
// n <= CSB_WR * CSB_RMAX).  The unbinned kernel above makes every wave of a
// bucket walk all of the bucket's entries; here the entries are walked twice
// in all and then read once in sequence:
//   1. csr_bin_count_kernel: wave (bucket b, row chunk ch) walks its rows of
//      the bucket's list and counts its entries per column range r (ranges
//      of wr <= CSB_WR columns) in LDS -> counts[(b R + r) C + ch];
//   2. csr_bin_scan_kernel: exclusive prefix sum in that (b, r, ch) order;
//   3. csr_bin_place_kernel: the same walk, each entry (column, signed value)
//      stored at its range's running offset plus its rank among the chunk's
//      lanes of the same range (lane order = entry order), so the entries of
//      (b, r) end up contiguous, in increasing row order, a row's entries in
//      storage order;
//   4. csr_bin_sum_kernel: one wave per (b, r) adds its contiguous entries
//      into its columns' LDS sums in that order (entries of one 64-entry
//      chunk that share a column in lane order, as in the unbinned kernel)
//      and writes row b of Y1 for those columns.
constexpr int CSB_WR = 1024;         // columns per range (4 workgroups of the summing pass per CU)
constexpr int CSB_RMAX = 4096;       // ranges (LDS counters per wave)
constexpr int CSB_ROWS = 256;        // rows per (bucket, chunk) walk, about
constexpr int64_t CSB_CNT_MAX = int64_t(1) << 24;  // counters (L R C)

struct CsrBinShape {
    int64_t R, C, wr, ncnt;  // ranges, chunks per bucket, range width, counters
    size_t cnt_b, col_b, val_b, total;
};

static CsrBinShape csr_bin_shape(int64_t m, int64_t n, int64_t nnz, int64_t L) {
    CsrBinShape s{};
    s.R = (n + CSB_WR - 1) / CSB_WR;
    s.wr = (n + s.R - 1) / s.R;
    s.C = std::min<int64_t>(64, std::max<int64_t>(1, (m / std::max<int64_t>(L, 1) + CSB_ROWS - 1) / CSB_ROWS));
    while (s.C > 1 && L * s.R * s.C > CSB_CNT_MAX) s.C /= 2;
    s.ncnt = L * s.R * s.C;
    if (s.R > CSB_RMAX || s.ncnt > CSB_CNT_MAX) {
        s.total = 0;  // too wide: the unbinned ordered kernel
        return s;
    }
    s.cnt_b = align256(sizeof(int64_t) * (size_t)(s.ncnt + 1));
    s.col_b = align256(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
    s.val_b = align256(sizeof(double) * (size_t)std::max<int64_t>(nnz, 1));
    s.total = s.cnt_b + s.col_b + s.val_b;
    return s;
}

size_t csr_bin_bytes(int64_t m, int64_t n, int64_t nnz, int64_t L) { return csr_bin_shape(m, n, nnz, L).total; }

struct CsrBinArgs {
    const int64_t* rowptr;
    const int32_t* colind;
    const double* val;
    int64_t m, n, nnz_cap;
    const int32_t* off;   // plan: bucket offsets into rows
    const int32_t* rows;  // plan: signed row codes grouped by bucket
    int64_t L, R, C, wr;
    int rbits;            // bits of a range index
    int64_t* cnt;         // L R C + 1 counters -> offsets
    int32_t* bcol;
    double* bval;
    double* Y;
    int64_t rs, cs;
};

constexpr int CSB_W = 4;  // waves per workgroup in the binning walks

// rows [p0, p1) of bucket b's list for chunk ch
__device__ __forceinline__ void csb_chunk_rows(const CsrBinArgs& a, int64_t b, int64_t ch, int& p0, int& p1) {
    const int beg = a.off[b], end = a.off[b + 1];
    const int64_t cnt = end - beg;
    p0 = beg + (int)(cnt * ch / a.C);
    p1 = beg + (int)(cnt * (ch + 1) / a.C);
}

// every entry of the wave's rows, in order: f(in, col, signed value) is
// called by all lanes for each 64-entry chunk (in: the lane holds an entry
// with a column in [0, n))
template <typename F>
__device__ __forceinline__ void csb_walk(const CsrBinArgs& a, int p0, int p1, F&& f) {
    const int lane = threadIdx.x & 63;
    const int64_t nnz = a.rowptr[a.m];
    for (int q0 = p0; q0 < p1; q0 += 64) {
        const int p = q0 + lane;
        const bool have = p < p1;
        const CsrBatch q = csr_batch(a.rowptr, have, have ? a.rows[p] : 0, nnz);
        for (int64_t B = 0; B < q.T; B += 64 * CSR_U) {
            int64_t e[CSR_U];
            bool ok[CSR_U], sg[CSR_U];
            csr_chunk_entries(q, B, nnz, e, ok, sg);
            double v[CSR_U];
            int32_t c[CSR_U];
#pragma unroll
            for (int u = 0; u < CSR_U; ++u) {
                v[u] = a.val[e[u]];
                c[u] = a.colind[e[u]];
            }
#pragma unroll
            for (int u = 0; u < CSR_U; ++u) {
                const bool in = ok[u] && c[u] >= 0 && c[u] < a.n;
                f(in, c[u], sg[u] ? -v[u] : v[u]);
            }
        }
    }
}

__global__ __launch_bounds__(64 * CSB_W) void csr_bin_count_kernel(CsrBinArgs a) {
    extern __shared__ int csb_hist[];  // CSB_W x R
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * CSB_W + w;
    if (q >= a.L * a.C) return;  // wave-uniform; no workgroup barrier here
    const int64_t b = q / a.C, ch = q % a.C;
    int* h = csb_hist + w * a.R;
    for (int r = lane; r < a.R; r += 64) h[r] = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    int p0, p1;
    csb_chunk_rows(a, b, ch, p0, p1);
    csb_walk(a, p0, p1, [&](bool in, int32_t c, double) {
        if (in) __hip_atomic_fetch_add(h + c / a.wr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    });
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int r = lane; r < a.R; r += 64)
        a.cnt[(b * a.R + r) * a.C + ch] = __hip_atomic_load(h + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// exclusive prefix sum of cnt[0 .. N) in place, cnt[N] = total; one workgroup
// walks tiles of CSB_SCAN * 8 counters (8 consecutive per thread, so the loads
// are coalesced), scanned through the waves and carried from tile to tile
constexpr int CSB_SCAN = 1024;
constexpr int CSB_SCAN_ITEMS = 8;
__global__ __launch_bounds__(CSB_SCAN) void csr_bin_scan_kernel(int64_t* cnt, int64_t N) {
    __shared__ int64_t wtot[CSB_SCAN / 64];
    __shared__ int64_t s_carry;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < N; base += (int64_t)CSB_SCAN * CSB_SCAN_ITEMS) {
        const int64_t i0 = base + (int64_t)t * CSB_SCAN_ITEMS;
        int64_t v[CSB_SCAN_ITEMS];
#pragma unroll
        for (int q = 0; q < CSB_SCAN_ITEMS; ++q) v[q] = (i0 + q < N) ? cnt[i0 + q] : 0;
        int64_t mine = 0;
#pragma unroll
        for (int q = 0; q < CSB_SCAN_ITEMS; ++q) mine += v[q];
        const int64_t inc = wave_incl_scan(mine);
        if (lane == 63) wtot[w] = inc;
        __syncthreads();
        int64_t before = s_carry;  // this tile's start
        for (int q = 0; q < w; ++q) before += wtot[q];
        int64_t run = before + inc - mine;  // exclusive start of this thread's items
#pragma unroll
        for (int q = 0; q < CSB_SCAN_ITEMS; ++q) {
            if (i0 + q < N) cnt[i0 + q] = run;
            run += v[q];
        }
        __syncthreads();  // every thread has read s_carry and wtot
        if (t == CSB_SCAN - 1) s_carry = run;  // the last thread's end = the tile's end
        __syncthreads();
    }
    if (t == 0) cnt[N] = s_carry;
}

__global__ __launch_bounds__(64 * CSB_W) void csr_bin_place_kernel(CsrBinArgs a) {
    extern __shared__ int64_t csb_run[];  // CSB_W x R
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * CSB_W + w;
    if (q >= a.L * a.C) return;
    const int64_t b = q / a.C, ch = q % a.C;
    int64_t* o = csb_run + w * a.R;
    for (int r = lane; r < a.R; r += 64) o[r] = a.cnt[(b * a.R + r) * a.C + ch];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes below this one
    int p0, p1;
    csb_chunk_rows(a, b, ch, p0, p1);
    csb_walk(a, p0, p1, [&](bool in, int32_t c, double x) {
        const int rg = in ? c / (int)a.wr : 0;
        // lanes holding an entry of the same range: one ballot per range bit
        uint64_t peers = __ballot(in);
        for (int bit = 0; bit < a.rbits; ++bit) {
            const bool on = (rg >> bit) & 1;
            const uint64_t mset = __ballot(on);
            peers &= on ? mset : ~mset;
        }
        if (in) {
            const int rank = __popcll(peers & lt);
            const int64_t base = __hip_atomic_load(o + rg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            const int64_t dst = base + rank;
            if (rank == 0)
                __hip_atomic_store(o + rg, base + __popcll(peers), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            if (dst < a.nnz_cap) {
                a.bcol[dst] = c;
                a.bval[dst] = x;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    });
}

__global__ __launch_bounds__(64 * CSD_W) void csr_bin_sum_kernel(CsrBinArgs a) {
    __shared__ double acc[CSD_W][CSB_WR];
    __shared__ int tag[CSD_W][CSD_SLOTS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * CSD_W + w;
    if (q >= a.L * a.R) return;
    const int64_t b = q / a.R, r = q % a.R;
    const int64_t c0 = r * a.wr, c1 = min(a.n, c0 + a.wr);
    double* my = acc[w];
    int* tg = tag[w];
    for (int64_t j = lane; j < c1 - c0; j += 64) __hip_atomic_store(my + j, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    for (int s2 = lane; s2 < CSD_SLOTS; s2 += 64) __hip_atomic_store(tg + s2, 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    wave_fence();
    const int64_t e0 = a.cnt[q * a.C], e1 = min(a.cnt[(q + 1) * a.C], a.nnz_cap);
    for (int64_t B = e0; B < e1; B += 64 * CSR_U) {
        int32_t c[CSR_U];
        double x[CSR_U];
        bool ok[CSR_U];
#pragma unroll
        for (int u = 0; u < CSR_U; ++u) {
            const int64_t e = B + 64 * u + lane;
            ok[u] = e < e1;
            c[u] = ok[u] ? a.bcol[e] : (int32_t)c0;
            x[u] = ok[u] ? a.bval[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < CSR_U; ++u) {
            const bool in = ok[u] && c[u] >= c0 && c[u] < c1;
            ordered_add(in, c[u], my + (in ? c[u] - c0 : 0), x[u], tg);
        }
    }
    for (int64_t j = c0 + lane; j < c1; j += 64)
        a.Y[b * a.rs + j * a.cs] = __hip_atomic_load(my + (j - c0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

static ids_status cs_csr_binned(const int64_t* rowptr, const int32_t* colind, const double* val, int64_t m,
                                int64_t n, int64_t nnz, const PlanBufs& pb, int64_t L, double* Y, int64_t rs,
                                int64_t cs, char* ws, hipStream_t st) {
    const CsrBinShape sh = csr_bin_shape(m, n, nnz, L);
    CsrBinArgs a;
    a.rowptr = rowptr;
    a.colind = colind;
    a.val = val;
    a.m = m;
    a.n = n;
    a.nnz_cap = std::max<int64_t>(nnz, 0);
    a.off = (const int32_t*)pb.off;
    a.rows = (const int32_t*)pb.rows;
    a.L = L;
    a.R = sh.R;
    a.C = sh.C;
    a.wr = sh.wr;
    a.rbits = 0;
    while ((int64_t(1) << a.rbits) < sh.R) ++a.rbits;
    a.cnt = (int64_t*)ws;
    a.bcol = (int32_t*)(ws + sh.cnt_b);
    a.bval = (double*)(ws + sh.cnt_b + sh.col_b);
    a.Y = Y;
    a.rs = rs;
    a.cs = cs;
    const unsigned gw = (unsigned)((L * sh.C + CSB_W - 1) / CSB_W);
    hipLaunchKernelGGL(csr_bin_count_kernel, dim3(gw), dim3(64 * CSB_W), sizeof(int) * CSB_W * sh.R, st, a);
    hipLaunchKernelGGL(csr_bin_scan_kernel, dim3(1), dim3(CSB_SCAN), 0, st, a.cnt, sh.ncnt);
    hipLaunchKernelGGL(csr_bin_place_kernel, dim3(gw), dim3(64 * CSB_W), sizeof(int64_t) * CSB_W * sh.R, st, a);
    hipLaunchKernelGGL(csr_bin_sum_kernel, dim3((unsigned)((L * sh.R + CSD_W - 1) / CSD_W)), dim3(64 * CSD_W), 0,
                       st, a);
    return check_launch("countsketch csr (ordered, binned)");
}

// bucket index of every position of the plan's row list
__global__ void plan_bucket_of_pos_kernel(const int32_t* off, int64_t L, int32_t* bop) {
    const int b = blockIdx.x;
    if (b >= L) return;
    for (int p = off[b] + threadIdx.x; p < off[b + 1]; p += blockDim.x) bop[p] = b;
}

__global__ void fill_f64_kernel(double* y, int64_t rows, int64_t cols, int64_t rs, int64_t cs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * cols) return;
    const int64_t r = t / cols, c = t % cols;
    y[r * rs + c * cs] = 0.0;
}

ids_status cs_csr(const int64_t* rowptr, const int32_t* colind, const double* val, int64_t m, int64_t n,
                  const PlanBufs& pb, int64_t L, double* Y, int64_t rs, int64_t cs, int32_t* scratch_bop,
                  bool ordered, int64_t nnz, char* bin_ws, hipStream_t st) {
    // the binned form unless the shape is too wide for it or the cs.csr.bin
    // knob selects the unbinned kernel (same results)
    if (ordered && bin_ws && csr_bin_bytes(m, n, nnz, L) > 0 && tune_get("cs.csr.bin", 1))
        return cs_csr_binned(rowptr, colind, val, m, n, nnz, pb, L, Y, rs, cs, bin_ws, st);
    if (ordered) {
        // column ranges of at most CSD_WR, CSD_W of them per workgroup
        const int64_t nr = (n + CSD_WR - 1) / CSD_WR;
        const int npanel = (int)((nr + CSD_W - 1) / CSD_W);
        const int64_t wr = (n + (int64_t)npanel * CSD_W - 1) / ((int64_t)npanel * CSD_W);
        if (L * npanel > INT32_MAX) {
            set_error("id_sketch: IDS_DETERMINISTIC: l1 * ceil(n / 8192) workgroups exceed the grid");
            return IDS_EINVAL;
        }
        hipLaunchKernelGGL(cs_csr_ordered_kernel, dim3((unsigned)(L * npanel)), dim3(64 * CSD_W), 0, st, rowptr,
                           colind, val, m, (const int32_t*)pb.off, (const int32_t*)pb.rows, npanel, n, wr, Y, rs, cs);
        return check_launch("countsketch csr (ordered)");
    }
    const size_t lds = sizeof(double) * (size_t)n;
    if (lds + 256 <= CSR_LDS_MAX_BYTES) {  // + the static batch counter
        // about one workgroup per compute unit (one fits, the LDS row is large);
        // several per bucket only when there are fewer buckets than units
        int nchunk = (int)(256 / L);
        int64_t rows_per_bucket = (m + L - 1) / L;
        int64_t maxch = rows_per_bucket / 256;
        if (nchunk > maxch) nchunk = (int)(maxch > 1 ? maxch : 1);
        if (nchunk < 1) nchunk = 1;
        const int use_atomic = nchunk > 1;
        if (use_atomic) {
            int64_t tot = L * n;
            hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Y, L, n,
                               rs, cs);
        }
        hipLaunchKernelGGL(cs_csr_lds_kernel, dim3((unsigned)(L * nchunk)), dim3(CSR_THREADS), lds, st, rowptr,
                           colind, val, m, n, (const int32_t*)pb.off, (const int32_t*)pb.rows, nchunk, Y, rs, cs,
                           use_atomic);
    } else {
        int64_t tot = L * n;
        hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Y, L, n, rs,
                           cs);
        hipLaunchKernelGGL(plan_bucket_of_pos_kernel, dim3((unsigned)L), dim3(256), 0, st, (const int32_t*)pb.off,
                           L, scratch_bop);
        int64_t thr = m * CSR_GROUP;
        hipLaunchKernelGGL(cs_csr_global_kernel, dim3((unsigned)((thr + 255) / 256)), dim3(256), 0, st, rowptr,
                           colind, val, (const int32_t*)pb.rows, m, (const int32_t*)scratch_bop, Y, rs, cs);
    }
    return check_launch("countsketch csr");
}

}  // namespace ids

// Shared device helpers for the idsketch library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace ids {

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based stream:
// output i of the stream with key K is mix64(K + (i+1)*GAMMA).
// ---------------------------------------------------------------------------
constexpr uint64_t GAMMA = 0x9e3779b97f4a7c15ULL;

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint64_t tag) {
    return mix64(seed ^ mix64(tag));
}

// bucket in [0, L) by multiply-shift of the high 32 bits; sign from bit 0.
// Returns the signed row code used by the sketch plans: i for +1, -(i+1) for -1.
__device__ __forceinline__ void hash_row(uint64_t key, int64_t i, uint32_t L, uint32_t& b,
                                         bool& neg) {
    uint64_t z = mix64(key + (uint64_t)(i + 1) * GAMMA);
    b = (uint32_t)(((z >> 32) * (uint64_t)L) >> 32);
    neg = (z & 1ULL) != 0;
}

__device__ __forceinline__ int32_t encode_row(int64_t i, bool neg) {
    return neg ? (int32_t)(-(i + 1)) : (int32_t)i;
}

// ---------------------------------------------------------------------------
// wave64 reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// DPP-based FP64 wave64 sum (GFX9 DPP controls): pairwise, quad, half-row,
// row, then row_bcast15 / row_bcast31 fold the four rows into lane 63, whose
// value is broadcast.  Fixed tree, so the result is deterministic.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane63_f64(double v) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

template <int NV>
__device__ __forceinline__ void wave_sum_dpp(double (&v)[NV]) {
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] += dpp_f64<0xB1, 0xf>(v[c]);  // quad_perm [1,0,3,2]
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] += dpp_f64<0x4E, 0xf>(v[c]);  // quad_perm [2,3,0,1]
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] += dpp_f64<0x141, 0xf>(v[c]); // row_half_mirror
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] += dpp_f64<0x140, 0xf>(v[c]); // row_mirror
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] += dpp_f64<0x142, 0xa>(v[c]); // row_bcast15 -> rows 1, 3
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] += dpp_f64<0x143, 0xc>(v[c]); // row_bcast31 -> rows 2, 3
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = lane63_f64(v[c]);
}

__device__ __forceinline__ double wave_sum_dpp1(double x) {
    double v[1] = {x};
    wave_sum_dpp<1>(v);
    return v[0];
}

// bf16 bits -> float
__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// thread-local last error message (set by the C-ABI layer)
void set_error(const std::string& msg);

}  // namespace ids

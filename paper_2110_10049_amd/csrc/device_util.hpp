// Device helpers for gfx950: Philox4x32-10, BF16 conversions, lane-group
// reductions on DPP, and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gosh {

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3"
// (SC'11): each round multiplies counter words 0 and 2 by fixed odd
// constants; the high halves are xored with the other two words and the
// round key, the low halves pass through; the key advances by a Weyl step.
__host__ __device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = static_cast<uint64_t>(kM0) * c.x;
        const uint64_t p1 = static_cast<uint64_t>(kM1) * c.z;
        const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c.y ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c.w ^ k1;
        c = make_uint4(n0, static_cast<uint32_t>(p1), n2, static_cast<uint32_t>(p0));
        k0 += kW0;
        k1 += kW1;
    }
    return c;
}

// Counter word 2 and word 3 of the method's random stream.
__host__ __device__ __forceinline__ uint32_t stream_word2(int32_t level, uint32_t tag) {
    return (static_cast<uint32_t>(level) & 0xFFu) | (tag << 8);
}
__host__ __device__ __forceinline__ uint32_t stream_word3(uint32_t kind, uint32_t slot,
                                                          uint32_t block) {
    return (kind << 24) | ((slot & 0xFFu) << 16) | (block & 0xFFFFu);
}

// floor(r * N / 2^32) for 0 <= N < 2^32
__host__ __device__ __forceinline__ int64_t scale_u32(uint32_t r, int64_t N) {
    return static_cast<int64_t>((static_cast<uint64_t>(r) * static_cast<uint64_t>(N)) >> 32);
}

// ---------------------------------------------------------------- BF16
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// FP32 -> BF16 by stochastic rounding with 16 random bits: the random bits
// are added below the kept half, so the magnitude rounds up with
// probability (dropped bits) / 2^16.  NaN stays a quiet NaN, Inf stays Inf.
__device__ __forceinline__ uint32_t bf16_sr(float x, uint32_t r16) {
    const uint32_t u = __float_as_uint(x);
    const uint32_t rounded = (u + r16) >> 16;
    const uint32_t special = (u >> 16) | ((u & 0x007FFFFFu) ? 0x40u : 0u);
    return ((u & 0x7F800000u) == 0x7F800000u) ? special : rounded;
}

// ---------------------------------------------------------------- lane groups
// Sum over aligned groups of G lanes (G in 1..32), every lane of the group
// receives the sum.  Groups must be uniformly active.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    if constexpr (G >= 2)   // swap neighbours: quad_perm [1,0,3,2]
        v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
    if constexpr (G >= 4)   // swap pairs: quad_perm [2,3,0,1]
        v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
    if constexpr (G >= 8)   // row_half_mirror: lane i <-> 7-i within 8
        v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));
    if constexpr (G >= 16)  // row_mirror: lane i <-> 15-i within 16
        v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, true));
    if constexpr (G >= 32)  // swap 16-lane halves of each 32: ds_swizzle xor 0x10
        v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
    return v;
}

__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace gosh

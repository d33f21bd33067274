// Wavefront (64-lane) helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bmf {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Butterfly sum over the 64 lanes, partners at distance 1, 2, 4, ..., 32.
// Every lane ends with the same bits: at each level a lane adds its
// partner's partial, and IEEE addition is commutative, so both partners
// form identical sums.
__device__ __forceinline__ float wave_sum_xor(float v) {
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ double wave_sum_xor_f64(double v) {
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// The same butterfly as wave_sum_xor with the four levels inside a 16-lane
// row done by DPP moves.  At levels 4 and 8 the mirror moves pick a lane
// whose partial equals the xor partner's (all lanes of a quad, resp. of an
// 8-lane half, already hold the same bits), so the association order, and
// hence the result, is identical to wave_sum_xor.
__device__ __forceinline__ float dpp_xor1(float v) {
    // quad_perm [1,0,3,2]
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_xor2(float v) {
    // quad_perm [2,3,0,1]
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_row_half_mirror(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));
}
__device__ __forceinline__ float dpp_row_mirror(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, true));
}

// Sum within each 16-lane row: after the call every lane of a row holds the
// row's total (all lanes of the row identical).
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp_xor1(v);
    v += dpp_xor2(v);
    v += dpp_row_half_mirror(v);  // lanes 0-3 <-> 7-4 of each 8: after the quad sums, partner holds the other quad's sum
    v += dpp_row_mirror(v);       // 0-7 <-> 15-8
    return v;
}

// Full 64-lane sum: row16_sum, then the partners at distance 16 and 32.
__device__ __forceinline__ float wave_sum_dpp(float v) {
    v = row16_sum(v);
    v += __shfl_xor(v, 16, WAVE);
    v += __shfl_xor(v, 32, WAVE);
    return v;
}

// Full 64-lane sum: row16_sum, then rows (0,1), (2,3) and halves combined
// with the gfx950 permlane swaps.  permlane16_swap(v, v) returns
// {rows 0,0,2,2 ; rows 1,1,3,3} of v, permlane32_swap(v, v) returns
// {halves lo,lo ; hi,hi}: adding the two results gives every lane the
// partner sums of the xor butterfly's last two levels, with the same
// association order (so the bits equal wave_sum_xor's).
__device__ __forceinline__ float wave_sum_perm(float v) {
    v = row16_sum(v);
    {
        const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    {
        const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        v = __uint_as_float(s[0]) + __uint_as_float(s[1]);
    }
    return v;
}

__device__ __forceinline__ uint32_t float_to_ordered(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ordered_to_float(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(b);
}

// 64-bit ranking key: larger is better; score descending, then smaller item.
__device__ __forceinline__ uint64_t rank_key(float score, int32_t item) {
    return ((uint64_t)float_to_ordered(score) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)item);
}
__device__ __forceinline__ float key_score(uint64_t key) { return ordered_to_float((uint32_t)(key >> 32)); }
__device__ __forceinline__ int32_t key_item(uint64_t key) { return (int32_t)(0xFFFFFFFFu - (uint32_t)key); }

}  // namespace bmf

// Byte and packed 16-bit helpers of the sweep kernels, each one VALU
// instruction on gfx950: byte selection (v_perm_b32) and alignment
// (v_alignbyte_b32), and two unsigned 16-bit lanes per word (v_pk_sub_u16
// with and without clamp, v_pk_min_u16).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Bytes of {hi, lo} chosen by the selector bytes of sel (0-3: lo, 4-7: hi;
// 12: 0x00, 13 and above: 0xFF).
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}
// The 32 bits of {hi, lo} starting at byte s.
__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t s) {
    return __builtin_amdgcn_alignbyte(hi, lo, s);
}
__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
// Per 16-bit lane: max(a - b, 0), a - b modulo 2^16, min(a, b).
__device__ __forceinline__ uint32_t sub_sat16(uint32_t a, uint32_t b) {
    return as_u32(__builtin_elementwise_sub_sat(as_u16x2(a), as_u16x2(b)));
}
__device__ __forceinline__ uint32_t sub16(uint32_t a, uint32_t b) { return as_u32(as_u16x2(a) - as_u16x2(b)); }
__device__ __forceinline__ uint32_t min16(uint32_t a, uint32_t b) {
    return as_u32(__builtin_elementwise_min(as_u16x2(a), as_u16x2(b)));
}

// 0/1 bytes mapped through a two-entry byte table (each byte selects byte 0
// or 1 of the table): one byte-permute, where the equivalent shifts and
// subtraction ((b << 8) - b and the like) are combined by the compiler into
// a 32-bit multiply.
__device__ __forceinline__ uint32_t bytes_ff(uint32_t b) { return perm(0u, 0x0000FF00u, b); }   // 0x00 / 0xFF
__device__ __forceinline__ uint32_t bytes_fe(uint32_t b) { return perm(0u, 0x0000FE00u, b); }   // 0x00 / 0xFE
__device__ __forceinline__ uint32_t bytes_pm1(uint32_t b) { return perm(0u, 0x0000FF01u, b); }  // +1 / -1

}  // namespace smc

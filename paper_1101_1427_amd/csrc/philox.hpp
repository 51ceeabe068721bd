// Device-side Philox4x32-10 and the stream layout of the random numbers.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (hi0,lo0) = M0*x0, (hi1,lo1) = M1*x2, x' = (hi1^x1^k0, lo1, hi0^x3^k1, lo0)
// with the key advanced by the Weyl constants between rounds.  The key is
// uniform across a launch, so its schedule lives in scalar registers; only
// the counter word that carries the site index varies per lane.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Stream tags (counter word 3 = 2*tag + colour).
constexpr uint32_t kTagInit = 1, kTagCoup = 2, kTagHead = 3, kTagTail = 4, kTagHeis = 5, kTagSwap = 6;

struct Key {
    uint32_t k0, k1;
};

__host__ __device__ inline Key make_key(uint64_t seed) { return Key{(uint32_t)seed, (uint32_t)(seed >> 32)}; }

// Three-input XOR in one VALU instruction (gfx950 v_bitop3_b32, truth table
// 0x96 = odd parity of the three inputs).
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
    return __builtin_amdgcn_bitop3_b32(a, b, k, 0x96);
}

// One Philox round: the two 32x32 -> 64-bit products are single
// v_mad_u64_u32 instructions.  The key is xored into the counter word first:
// in the early rounds that word is uniform across the wave, so the pair
// costs one scalar and one vector xor.
__device__ __forceinline__ uint4 philox_round(uint4 x, uint32_t k0, uint32_t k1) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * x.x;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * x.z;
    return make_uint4((uint32_t)(p1 >> 32) ^ (x.y ^ k0), (uint32_t)p1, (uint32_t)(p0 >> 32) ^ (x.w ^ k1),
                      (uint32_t)p0);
}

__device__ __forceinline__ uint4 philox_round_x3(uint4 x, uint32_t k0, uint32_t k1) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * x.x;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * x.z;
    return make_uint4(xor3_key((uint32_t)(p1 >> 32), x.y, k0), (uint32_t)p1, xor3_key((uint32_t)(p0 >> 32), x.w, k1),
                      (uint32_t)p0);
}

// Philox4x32-10 of counter x.  Counter words 1..3 are wave-uniform in every
// use here, so the first two rounds are left to the compiler (it keeps the
// uniform parts in scalar registers); from the third round on two of the
// xored words vary per lane and the three-input XOR takes the place of two
// instructions.
__device__ __forceinline__ uint4 philox4x32_10(uint4 x, Key key) {
    uint32_t k0 = key.k0, k1 = key.k1;
    x = philox_round(x, k0, k1);
#pragma unroll
    for (int round = 1; round < 2; ++round) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
        x = philox_round(x, k0, k1);
    }
#pragma unroll
    for (int round = 2; round < 10; ++round) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
        x = philox_round_x3(x, k0, k1);
    }
    return x;
}

// 32 x 32 -> 64-bit product of a per-lane word and a constant as one
// v_mad_u64_u32.  The compiler selects the same instruction from the plain
// product in most places but splits the last round's products of a single
// draw into separate low and high multiplies where the draw feeds packed
// 16-bit code; this form keeps the one instruction.  Register operands only.
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t m) {
    uint64_t p, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(p), "=s"(carry) : "v"(a), "s"(m));
    (void)carry;
    return p;
}

// philox4x32_10 with the products of rounds 3 to 10 as mul_wide (for
// kernels whose code is inlined in full: the asm statements raise the
// compiler's inlining cost, so callers that rely on inlining of large
// device functions keep the plain form).
__device__ __forceinline__ uint4 philox4x32_10_wide(uint4 x, Key key) {
    uint32_t k0 = key.k0, k1 = key.k1;
    x = philox_round(x, k0, k1);
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
    x = philox_round(x, k0, k1);
#pragma unroll
    for (int round = 2; round < 10; ++round) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
        const uint64_t p0 = mul_wide(x.x, kPhiloxM0);
        const uint64_t p1 = mul_wide(x.z, kPhiloxM1);
        x = make_uint4(xor3_key((uint32_t)(p1 >> 32), x.y, k0), (uint32_t)p1, xor3_key((uint32_t)(p0 >> 32), x.w, k1),
                       (uint32_t)p0);
    }
    return x;
}

// N independent draws advanced round by round together (independent
// dependency chains interleave in the instruction stream).
template <int NC>
__device__ __forceinline__ void philox4x32_10_multi(uint4 (&x)[NC], Key key) {
    uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = philox_round(x[c], k0, k1);
#pragma unroll
    for (int round = 1; round < 2; ++round) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = philox_round(x[c], k0, k1);
    }
#pragma unroll
    for (int round = 2; round < 10; ++round) {
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
#pragma unroll
        for (int c = 0; c < NC; ++c) x[c] = philox_round_x3(x[c], k0, k1);
    }
}

__device__ __forceinline__ uint32_t word_of(const uint4 &w, uint32_t j) {
    return j == 0 ? w.x : j == 1 ? w.y : j == 2 ? w.z : w.w;
}

// 16-bit head of the Metropolis uniform of in-colour index h: half (h & 7) of
// the draw (h>>3, t, r, 2*HEAD + c), the low half of word 0 first.
__device__ __forceinline__ uint32_t head16_of(const uint4 &w, uint32_t h8) {
    const uint32_t word = word_of(w, h8 >> 1);
    return (h8 & 1) ? (word >> 16) : (word & 0xFFFFu);
}

// 16-bit tail: low half of word 0 of the draw (h, t, r, 2*TAIL + c).
__device__ __forceinline__ uint32_t tail16(uint32_t h, uint32_t t, uint32_t r, uint32_t c, Key key) {
    return philox4x32_10(make_uint4(h, t, r, 2 * kTagTail + c), key).x & 0xFFFFu;
}

// Threshold of a positive energy change, split into the part compared with
// the head (0 .. 65536) and the part compared with the tail (0 .. 65535):
// thr = hi * 2^16 + lo = floor(2^32 exp(-beta dE)).
// u = head*2^16 + tail < thr  <=>  head < hi  or  (head == hi and tail < lo).
__device__ __forceinline__ bool metropolis_accept(uint32_t head, uint2 thr, uint32_t h, uint32_t t,
                                                  uint32_t r, uint32_t c, Key key) {
    if (head != thr.x) return head < thr.x;
    return tail16(h, t, r, c, key) < thr.y;
}

// Uniform (k + 1/2) 2^-23 from the top 23 bits of a word: exact in float.
__device__ __forceinline__ float unit23f(uint32_t w) {
    return ((float)(w >> 9) + 0.5f) * (1.0f / 8388608.0f);
}

// 53-bit uniform in [0, 1) from two words.
__device__ __forceinline__ double unit53(uint32_t w0, uint32_t w1) {
    return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6)) * (1.0 / 9007199254740992.0);
}

}  // namespace smc

// Byte-parallel Metropolis update of one 16-site row segment of a 3D Ising
// or +-J EA lattice (Eq. 2 on the simple cubic lattice), shared by the
// half-sweep kernel (sweep3d.hip) and the 3D double checkerboard
// (dcb3d.hip).  Spins are int8 +-1 bytes (0x01 / 0xFF), row-major in x.
//
// The eight colour-c sites of a segment starting at even x0 are its odd-x
// sites (A = 1) or even-x sites (A = 0); they are the in-colour indices
// h0 .. h0 + 7 (h0 = first site / 2, a multiple of 8), whose 16-bit heads
// are the eight halves of the Philox block (h0 / 8, t, r, 2*HEAD + c) in
// order.  Unsatisfied bonds are counted four sites to a word, the flip
// decision compares heads with the thresholds' high halves in packed 16-bit
// lanes, and a head equal to a high half takes the exact (tail) decision.
#pragma once
#include "internal.hpp"

namespace smc {
namespace seg3d {

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}
__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t s) {
    return __builtin_amdgcn_alignbyte(hi, lo, s);
}
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ __forceinline__ uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ uint32_t sub_sat16(uint32_t a, uint32_t b) {
    return as_u32(__builtin_elementwise_sub_sat(as_u16x2(a), as_u16x2(b)));
}
__device__ __forceinline__ uint32_t sub16(uint32_t a, uint32_t b) { return as_u32(as_u16x2(a) - as_u16x2(b)); }
__device__ __forceinline__ uint32_t min16(uint32_t a, uint32_t b) {
    return as_u32(__builtin_elementwise_min(as_u16x2(a), as_u16x2(b)));
}

// Spin bytes +1 / -1 (0x01 / 0xFF) to bits 0 / 1, four per word.
__device__ __forceinline__ uint32_t bits(uint32_t v) { return (v >> 1) & 0x01010101u; }
__device__ __forceinline__ uint2 bits2(uint2 v) { return make_uint2(bits(v.x), bits(v.y)); }

// Even-x (sel 0x06040200) or odd-x (sel 0x07050301) bytes of a segment.
__device__ __forceinline__ uint2 half_of(uint4 w, uint32_t sel) {
    return make_uint2(perm(w.y, w.x, sel), perm(w.w, w.z, sel));
}

// High 16 bits of the thresholds for n = 0, 1, 2 unsatisfied bonds (Delta E
// = 12, 8, 4) as low and high bytes indexed by n; n >= 3 (Delta E <= 0)
// reads 0xFFFF, and a head of 0xFFFF takes the exact path.  A high half of
// 0x10000 (threshold 2^32, beta = 0) enters as 0xFFFF: every smaller head
// accepts, as it should, and a head of 0xFFFF is decided exactly.
struct Lut3 {
    uint32_t lo, hi;
};

__device__ __forceinline__ Lut3 lut_of(const ThrRow &row) {
    const uint32_t t3 = min(row.m[3].x, 0xFFFFu), t2 = min(row.m[2].x, 0xFFFFu), t1 = min(row.m[1].x, 0xFFFFu);
    Lut3 k;
    k.lo = (t3 & 0xFFu) | ((t2 & 0xFFu) << 8) | ((t1 & 0xFFu) << 16) | 0xFF000000u;
    k.hi = (t3 >> 8) | ((t2 >> 8) << 8) | ((t1 >> 8) << 16) | 0xFF000000u;
    return k;
}

// Flip flags (0/1 bytes) of four sites with counts n (bytes 0..6) and heads
// in wa (sites 0, 1) and wb (sites 2, 3); eq collects threshold - head per
// 16-bit lane, zero where a head equals the high half of its threshold.
__device__ __forceinline__ uint32_t decide4(uint32_t n, uint32_t wa, uint32_t wb, Lut3 k, uint32_t one2,
                                            uint32_t &eq) {
    const uint32_t tl = perm(0xFFFFFFFFu, k.lo, n);
    const uint32_t th = perm(0xFFFFFFFFu, k.hi, n);
    const uint32_t ta = perm(th, tl, 0x05010400u);
    const uint32_t tb = perm(th, tl, 0x07030602u);
    const uint32_t ra = min16(sub_sat16(ta, wa), one2);
    const uint32_t rb = min16(sub_sat16(tb, wb), one2);
    eq = min16(eq, min16(sub16(ta, wa), sub16(tb, wb)));
    return perm(rb, ra, 0x06040200u);
}

// Flip flags of the eight own sites of a segment and their bond counts.
struct RowOut {
    uint32_t F0, F1, n0, n1;
};

// True where a 16-bit lane of eq is zero (a head equal to its high half).
__device__ __forceinline__ bool has_tie(uint32_t eq) { return ((eq & 0xFFFFu) == 0u) || ((eq >> 16) == 0u); }

// Exact decisions of the eight sites of o (heads w, in-colour indices h0 ..
// h0 + 7) on the lanes with tie set: a head equal to the high half of its
// threshold (probability 2^-16 per site) compares the tail draw with the low
// half.
__device__ __forceinline__ void exact_decisions(RowOut &o, const uint4 &w, const ThrRow &th, uint32_t h0, uint32_t c,
                                                uint32_t t, uint32_t r, Key key, uint32_t four, bool tie) {
    if (!tie) return;
    // the heads as two 64-bit words and the three thresholds as values, so
    // that the selections below stay in registers
    const uint64_t wlo = ((uint64_t)w.y << 32) | w.x, whi = ((uint64_t)w.w << 32) | w.z;
    const uint64_t T3 = ((uint64_t)th.m[3].y << 32) | th.m[3].x, T2 = ((uint64_t)th.m[2].y << 32) | th.m[2].x,
                   T1 = ((uint64_t)th.m[1].y << 32) | th.m[1].x;
    uint32_t f0 = 0u, f1 = 0u;
#pragma unroll 1
    for (uint32_t i = 0; i < 2u * four; ++i) {
        const uint32_t ns = ((i < 4u ? o.n0 : o.n1) >> (8u * (i & 3u))) & 0xFFu;
        const uint32_t head = (uint32_t)((i < 4u ? wlo : whi) >> (16u * (i & 3u))) & 0xFFFFu;
        uint32_t flip = 1u;
        if (ns < 3u) {
            const uint64_t T = ns == 0u ? T3 : ns == 1u ? T2 : T1;  // Delta E = 12 - 4 ns
            flip = metropolis_accept(head, make_uint2((uint32_t)T, (uint32_t)(T >> 32)), h0 + i, t, r, c, key);
        }
        if (i < 4u)
            f0 |= flip << (8u * (i & 3u));
        else
            f1 |= flip << (8u * (i & 3u));
    }
    o.F0 = f0;
    o.F1 = f1;
}

// One segment: own row raw bytes, neighbours' raw bytes, the extra x
// neighbour bit eb, the per-row bond arrays (EA), Philox block index h0.
// Bonds of the eight own sites (bit 1 where J = -1, one byte per site, in
// the order of the own array): b pairs with the other array of the row
// unshifted, s with it shifted by one site (see segment_update), and the
// bonds to y + 1, y - 1, z + 1, z - 1.
struct Bonds3 {
    uint2 b, s, yp, ym, zp, zm;
};

// From the int8 bond rows: +x bonds of the row (jx) and the bond entering
// it from x0 - 1 (bit jeb), +y bonds of the row (jy) and of row y - 1
// (jym), +z bonds of the row (jz) and of row z - 1 (jzm).
__device__ __forceinline__ Bonds3 bonds_from_bytes(const uint4 &jx, uint32_t jeb, const uint4 &jy, const uint4 &jym,
                                                   const uint4 &jz, const uint4 &jzm, int A) {
    const uint32_t sa = A ? 0x07050301u : 0x06040200u, sb = A ? 0x06040200u : 0x07050301u;
    const uint2 jxa = bits2(half_of(jx, sa)), jxb = bits2(half_of(jx, sb));
    Bonds3 bd;
    // paired with the unshifted other array: x -> x + 1 of even-x sites
    // (array a), x - 1 -> x of odd-x sites (array b); with the shifted one:
    // x + 1 of odd-x sites (array a), x - 1 of even-x sites (array b shifted
    // up, x0 - 1 entering)
    bd.b = A ? jxb : jxa;
    bd.s.x = A ? jxa.x : ((jxb.x << 8) | jeb);
    bd.s.y = A ? jxa.y : alignbyte(jxb.y, jxb.x, 3);
    bd.yp = bits2(half_of(jy, sa));
    bd.ym = bits2(half_of(jym, sa));
    bd.zp = bits2(half_of(jz, sa));
    bd.zm = bits2(half_of(jzm, sa));
    return bd;
}

// Eight bits to eight 0/1 bytes.
__device__ __forceinline__ uint2 spread8(uint32_t m) {
    return make_uint2(((m & 15u) * 0x00204081u) & 0x01010101u, (((m >> 4) & 15u) * 0x00204081u) & 0x01010101u);
}

// From bit-packed bond masks of one direction and segment: bits 0..7 the
// even-x sites, bits 8..15 the odd-x sites (bit 1 where J = -1).  jx, jy, jz
// are the row's masks, jym and jzm those of rows y - 1 and z - 1, jeb the
// bond entering the row from x0 - 1.
__device__ __forceinline__ Bonds3 bonds_from_bits(uint32_t jx, uint32_t jeb, uint32_t jy, uint32_t jym, uint32_t jz,
                                                  uint32_t jzm, int A) {
    const int sh = A ? 8 : 0;
    const uint32_t ax = (jx >> sh) & 0xFFu, bx = (jx >> (8 - sh)) & 0xFFu;
    Bonds3 bd;
    bd.b = spread8(A ? bx : ax);
    bd.s = spread8(A ? ax : (((bx << 1) | jeb) & 0xFFu));
    bd.yp = spread8((jy >> sh) & 0xFFu);
    bd.ym = spread8((jym >> sh) & 0xFFu);
    bd.zp = spread8((jz >> sh) & 0xFFu);
    bd.zm = spread8((jzm >> sh) & 0xFFu);
    return bd;
}

// Four 0/1 bytes to four bits.
__device__ __forceinline__ uint32_t gather4(uint32_t w) { return (w * 0x01020408u) >> 24; }

// One segment: own row raw bytes, the neighbour rows' raw bytes, the x
// neighbour beyond the segment (bit eb: x0 + 16 for odd-x own sites, x0 - 1
// for even-x), the bonds (EA), Philox block index h0 of the own sites.
template <bool EA>
__device__ __forceinline__ RowOut segment_update(const uint4 &own, const uint4 &rym, const uint4 &ryp,
                                                 const uint4 &rzm, const uint4 &rzp, uint32_t eb, int A,
                                                 const Bonds3 &bd, const ThrRow &th, uint32_t h0, uint32_t c,
                                                 uint32_t t, uint32_t r, Key key, uint32_t one2, uint32_t four) {
    const uint32_t sa = A ? 0x07050301u : 0x06040200u, sb = A ? 0x06040200u : 0x07050301u;
    const uint2 Sa = bits2(half_of(own, sa));
    const uint2 Sb = bits2(half_of(own, sb));
    const uint2 ym = bits2(half_of(rym, sa));
    const uint2 yp = bits2(half_of(ryp, sa));
    const uint2 zm = bits2(half_of(rzm, sa));
    const uint2 zp = bits2(half_of(rzp, sa));
    // the other array shifted by one site: odd-x sites see x + 1 (down by a
    // byte, x0 + 16 entering at the top), even-x sites x - 1 (up by a byte)
    uint2 sh;
    sh.x = A ? alignbyte(Sb.y, Sb.x, 1) : ((Sb.x << 8) | eb);
    sh.y = A ? ((Sb.y >> 8) | (eb << 24)) : alignbyte(Sb.y, Sb.x, 3);
    RowOut o;
    if constexpr (EA) {
        o.n0 = ((Sa.x ^ Sb.x ^ bd.b.x) + (Sa.x ^ sh.x ^ bd.s.x)) + ((Sa.x ^ yp.x ^ bd.yp.x) + (Sa.x ^ ym.x ^ bd.ym.x)) +
               ((Sa.x ^ zp.x ^ bd.zp.x) + (Sa.x ^ zm.x ^ bd.zm.x));
        o.n1 = ((Sa.y ^ Sb.y ^ bd.b.y) + (Sa.y ^ sh.y ^ bd.s.y)) + ((Sa.y ^ yp.y ^ bd.yp.y) + (Sa.y ^ ym.y ^ bd.ym.y)) +
               ((Sa.y ^ zp.y ^ bd.zp.y) + (Sa.y ^ zm.y ^ bd.zm.y));
    } else {
        o.n0 = ((Sa.x ^ Sb.x) + (Sa.x ^ sh.x)) + ((Sa.x ^ yp.x) + (Sa.x ^ ym.x)) + ((Sa.x ^ zp.x) + (Sa.x ^ zm.x));
        o.n1 = ((Sa.y ^ Sb.y) + (Sa.y ^ sh.y)) + ((Sa.y ^ yp.y) + (Sa.y ^ ym.y)) + ((Sa.y ^ zp.y) + (Sa.y ^ zm.y));
    }
    const uint4 w = philox4x32_10(make_uint4(h0 >> 3, t, r, 2 * kTagHead + c), key);
    const Lut3 K = lut_of(th);
    uint32_t eq = 0xFFFFFFFFu;
    o.F0 = decide4(o.n0, w.x, w.y, K, one2, eq);
    o.F1 = decide4(o.n1, w.z, w.w, K, one2, eq);
    if (__builtin_expect(__any(has_tie(eq)), 0)) exact_decisions(o, w, th, h0, c, t, r, key, four, has_tie(eq));
    return o;
}

// The segment with the flagged own sites flipped (+1 <-> -1: byte ^ 0xFE).
__device__ __forceinline__ uint4 apply_flips(const uint4 &own, const RowOut &o, int A) {
    const uint32_t m0 = (o.F0 << 8) - (o.F0 << 1), m1 = (o.F1 << 8) - (o.F1 << 1);  // 0xFE where flipped
    const uint32_t slo = A ? 0x01040004u : 0x04010400u, shi = A ? 0x03040204u : 0x04030402u;
    return make_uint4(own.x ^ perm(0u, m0, slo), own.y ^ perm(0u, m0, shi), own.z ^ perm(0u, m1, slo),
                      own.w ^ perm(0u, m1, shi));
}

// Energy change of the segment's flips: 12 - 4n for a site with n
// unsatisfied bonds.
__device__ __forceinline__ long long flip_energy(const RowOut &o) {
    const uint32_t f0 = (o.F0 << 8) - o.F0, f1 = (o.F1 << 8) - o.F1;  // 0xFF where flipped
    const uint32_t cnt = __builtin_amdgcn_sad_u8(o.F0, 0u, __builtin_amdgcn_sad_u8(o.F1, 0u, 0u));
    const uint32_t nsum = __builtin_amdgcn_sad_u8(o.n0 & f0, 0u, __builtin_amdgcn_sad_u8(o.n1 & f1, 0u, 0u));
    return 12 * (long long)cnt - 4 * (long long)nsum;
}

}  // namespace seg3d
}  // namespace smc

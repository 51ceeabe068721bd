// Byte-parallel Metropolis update of one 16-site row segment of a 3D Ising
// or +-J EA lattice (Eq. 2 on the simple cubic lattice), shared by the
// half-sweep kernel (sweep3d.hip) and the 3D double checkerboard
// (dcb3d.hip).  Spins are int8 +-1 bytes (0x01 / 0xFF), row-major in x.
//
// The eight colour-c sites of a segment starting at even x0 are its odd-x
// sites (A = 1) or even-x sites (A = 0); they are the in-colour indices
// h0 .. h0 + 7 (h0 = first site / 2, a multiple of 8), whose 16-bit heads
// are the eight halves of the Philox block (h0 / 8, t, r, 2*HEAD + c) in
// order.  Unsatisfied bonds are counted four sites to a word ((a ^ b) & 2
// per byte of two +-1 spin bytes, one v_bitop3 per neighbour word), the
// flip decision compares heads with the thresholds' high halves in packed
// 16-bit lanes, and a head equal to a high half takes the exact (tail)
// decision.
#pragma once
#include "internal.hpp"
#include "intrin.hpp"

namespace smc {
namespace seg3d {

// +-1 bytes (0x01 / 0xFF) to bits 0 / 1, four per word (bond packing).
__device__ __forceinline__ uint32_t bits(uint32_t v) { return (v >> 1) & 0x01010101u; }
__device__ __forceinline__ uint2 bits2(uint2 v) { return make_uint2(bits(v.x), bits(v.y)); }

// (a ^ b) & m in one instruction: with m = 0x02020202, 2 in each byte where
// two +-1 spin bytes (0x01 / 0xFF) differ, or where bit 1 of the xor of
// three such bytes or bond bytes is set.
__device__ __forceinline__ uint32_t unsat(uint32_t a, uint32_t b, uint32_t m) {
    return __builtin_amdgcn_bitop3_b32(a, b, m, 0x28);
}

// Bits o .. o + 7 of m to eight bytes whose bit 1 is the bit (four bits per
// 24-bit product: bit i of a nibble lands on bits i + 1, i + 8, i + 15 and
// i + 22, so bit 8 i + 1 holds it and no two land on one position).  The
// other bits of each byte are left as they come: every use masks bit 1.
__device__ __forceinline__ uint2 spread8b(uint32_t m, uint32_t o) {
    return make_uint2(__umul24(__builtin_amdgcn_ubfe(m, o, 4), 0x00408102u),
                      __umul24(__builtin_amdgcn_ubfe(m, o + 4, 4), 0x00408102u));
}

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

// Exact decisions of the sites of o (heads w, in-colour indices h0 .. h0 + 7,
// counts in o.n0 / o.n1) whose head equals the high half of the table entry
// (probability 2^-16 per site), on the lanes with tie set.  A wavefront that
// meets a tie holds up its workgroup at the next barrier, so the path is
// short: a mask of the tied sites, then one pass per tied site of the lane
// with most of them (almost always one), each drawing the single tail it
// needs.
__device__ __forceinline__ void exact_decisions(RowOut &o, const uint4 &w, const ThrRow &th, const Lut3 &K,
                                                uint32_t h0, uint32_t c, uint32_t t, uint32_t r, Key key, bool tie) {
    uint32_t tm = 0;  // bit s: site s (0 .. 7) is tied
    if (tie) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const uint32_t n = q ? o.n1 : o.n0;
            const uint32_t tl = perm(0xFFFFFFFFu, K.lo, n), thh = perm(0xFFFFFFFFu, K.hi, n);
            const uint32_t da = perm(thh, tl, 0x05010400u) ^ (q ? w.z : w.x);
            const uint32_t db = perm(thh, tl, 0x07030602u) ^ (q ? w.w : w.y);
            const uint32_t m4 = ((da & 0xFFFFu) == 0u ? 1u : 0u) | ((da >> 16) == 0u ? 2u : 0u) |
                                ((db & 0xFFFFu) == 0u ? 4u : 0u) | ((db >> 16) == 0u ? 8u : 0u);
            tm |= m4 << (4 * q);
        }
    }
    // values, not references, below: a selected reference would put the
    // structure it points into in scratch memory
    const uint32_t n0 = o.n0, n1 = o.n1, w0 = w.x, w1 = w.y, w2 = w.z, w3 = w.w;
    const uint32_t t3x = th.m[3].x, t3y = th.m[3].y, t2x = th.m[2].x, t2y = th.m[2].y, t1x = th.m[1].x,
                   t1y = th.m[1].y;
    while (__any(tm != 0u)) {
        if (tm != 0u) {
            const uint32_t s = __builtin_ctz(tm), b = 8u * (s & 3u);
            tm &= tm - 1u;
            const uint32_t ns = ((s < 4u ? n0 : n1) >> b) & 0xFFu;
            const uint32_t word = s < 2u ? w0 : s < 4u ? w1 : s < 6u ? w2 : w3;
            const uint32_t head = (s & 1u) ? (word >> 16) : (word & 0xFFFFu);
            uint32_t flip = 1u;  // Delta E <= 0
            if (ns < 3u) {
                // Delta E = 12 - 4 ns
                const uint32_t tx = ns == 0u ? t3x : ns == 1u ? t2x : t1x;
                const uint32_t ty = ns == 0u ? t3y : ns == 1u ? t2y : t1y;
                flip = metropolis_accept(head, make_uint2(tx, ty), h0 + s, t, r, c, key) ? 1u : 0u;
            }
            const uint32_t keep = ~(0xFFu << b), set = flip << b;
            if (s < 4u)
                o.F0 = (o.F0 & keep) | set;
            else
                o.F1 = (o.F1 & keep) | set;
        }
    }
}

// Bonds of the eight own sites (bit 1 of a byte set where J = -1, the
// byte's other bits arbitrary, one byte per site in the order of the own
// array): b pairs with the other array of the row unshifted, s with it
// shifted by one site (see segment_update), and the bonds to y + 1, y - 1,
// z + 1, z - 1.
struct Bonds3 {
    uint2 b, s, yp, ym, zp, zm;
};

// From the int8 bond rows: +x bonds of the row (jx) and the bond entering
// it from x0 - 1 (bit jeb), +y bonds of the row (jy) and of row y - 1
// (jym), +z bonds of the row (jz) and of row z - 1 (jzm).
// (int8 +-1 bonds have bit 1 set exactly where J = -1, so their bytes are
// used as they are.)
__device__ __forceinline__ Bonds3 bonds_from_bytes(const uint4 &jx, uint32_t jeb, const uint4 &jy, const uint4 &jym,
                                                   const uint4 &jz, const uint4 &jzm, int A) {
    const uint32_t sa = A ? 0x07050301u : 0x06040200u, sb = A ? 0x06040200u : 0x07050301u;
    const uint2 jxa = half_of(jx, sa), jxb = half_of(jx, sb);
    Bonds3 bd;
    // paired with the unshifted other array: x -> x + 1 of even-x sites
    // (array a), x - 1 -> x of odd-x sites (array b); with the shifted one:
    // x + 1 of odd-x sites (array a), x - 1 of even-x sites (array b shifted
    // up, x0 - 1 entering)
    bd.b = A ? jxb : jxa;
    bd.s.x = A ? jxa.x : ((jxb.x << 8) | (jeb << 1));
    bd.s.y = A ? jxa.y : alignbyte(jxb.y, jxb.x, 3);
    bd.yp = half_of(jy, sa);
    bd.ym = half_of(jym, sa);
    bd.zp = half_of(jz, sa);
    bd.zm = half_of(jzm, sa);
    return bd;
}

// From bit-packed bond masks of one direction and segment: bits 0..7 the
// even-x sites, bits 8..15 the odd-x sites (bit 1 where J = -1).  jx, jy, jz
// are the row's masks, jym and jzm those of rows y - 1 and z - 1, jeb the
// bond entering the row from x0 - 1.
__device__ __forceinline__ Bonds3 bonds_from_bits(uint32_t jx, uint32_t jeb, uint32_t jy, uint32_t jym, uint32_t jz,
                                                  uint32_t jzm, int A) {
    const uint32_t sh = A ? 8u : 0u;
    Bonds3 bd;
    // the unshifted pairs are joined by the even-x sites' +x bonds (bits
    // 0-7) for either parity; the shifted pairs by the odd-x sites' bonds
    // (bits 8-15), which the even-x sites see moved up by one site with the
    // bond from x0 - 1 entering at the bottom
    bd.b = spread8b(jx, 0u);
    bd.s = A ? spread8b(jx, 8u) : spread8b(((jx >> 7) & 0xFEu) | jeb, 0u);
    bd.yp = spread8b(jy, sh);
    bd.ym = spread8b(jym, sh);
    bd.zp = spread8b(jz, sh);
    bd.zm = spread8b(jzm, sh);
    return bd;
}

// Four 0/1 bytes to four bits.
__device__ __forceinline__ uint32_t gather4(uint32_t w) { return (w * 0x01020408u) >> 24; }

// Bond counts of the eight own sites (bytes 0 .. 6) from the own array Sa,
// the other array Sb, the other array shifted by one site (sh) and the y
// and z neighbour arrays, all raw spin bytes in the order of the own sites.
template <bool EA>
__device__ __forceinline__ void count_unsat(const uint2 &Sa, const uint2 &Sb, const uint2 &sh, const uint2 &ym,
                                            const uint2 &yp, const uint2 &zm, const uint2 &zp, const Bonds3 &bd,
                                            uint32_t &n0, uint32_t &n1) {
    const uint32_t m2 = 0x02020202u;
    if constexpr (EA) {
        n0 = (unsat(Sa.x ^ bd.b.x, Sb.x, m2) + unsat(Sa.x ^ bd.s.x, sh.x, m2) + unsat(Sa.x ^ bd.yp.x, yp.x, m2) +
              unsat(Sa.x ^ bd.ym.x, ym.x, m2) + unsat(Sa.x ^ bd.zp.x, zp.x, m2) + unsat(Sa.x ^ bd.zm.x, zm.x, m2)) >>
             1;
        n1 = (unsat(Sa.y ^ bd.b.y, Sb.y, m2) + unsat(Sa.y ^ bd.s.y, sh.y, m2) + unsat(Sa.y ^ bd.yp.y, yp.y, m2) +
              unsat(Sa.y ^ bd.ym.y, ym.y, m2) + unsat(Sa.y ^ bd.zp.y, zp.y, m2) + unsat(Sa.y ^ bd.zm.y, zm.y, m2)) >>
             1;
    } else {
        n0 = (unsat(Sa.x, Sb.x, m2) + unsat(Sa.x, sh.x, m2) + unsat(Sa.x, yp.x, m2) + unsat(Sa.x, ym.x, m2) +
              unsat(Sa.x, zp.x, m2) + unsat(Sa.x, zm.x, m2)) >>
             1;
        n1 = (unsat(Sa.y, Sb.y, m2) + unsat(Sa.y, sh.y, m2) + unsat(Sa.y, yp.y, m2) + unsat(Sa.y, ym.y, m2) +
              unsat(Sa.y, zp.y, m2) + unsat(Sa.y, zm.y, m2)) >>
             1;
    }
}

// One segment: own row raw bytes, the neighbour rows' raw bytes, the x
// neighbour beyond the segment (eb, its raw byte: x0 + 16 for odd-x own
// sites, x0 - 1 for even-x), the bonds (EA), Philox block index h0 of the
// own sites.
template <bool EA>
__device__ __forceinline__ RowOut segment_update(const uint4 &own, const uint4 &rym, const uint4 &ryp,
                                                 const uint4 &rzm, const uint4 &rzp, uint32_t eb, int A,
                                                 const Bonds3 &bd, const ThrRow &th, uint32_t h0, uint32_t c,
                                                 uint32_t t, uint32_t r, Key key, uint32_t one2) {
    const uint32_t sa = A ? 0x07050301u : 0x06040200u, sb = A ? 0x06040200u : 0x07050301u;
    const uint2 Sa = half_of(own, sa);
    const uint2 Sb = half_of(own, sb);
    // the other array shifted by one site: odd-x sites see x + 1 (down by a
    // byte, x0 + 16 entering at the top), even-x sites x - 1 (up by a byte)
    uint2 sh;
    sh.x = A ? alignbyte(Sb.y, Sb.x, 1) : ((Sb.x << 8) | eb);
    sh.y = A ? ((Sb.y >> 8) | (eb << 24)) : alignbyte(Sb.y, Sb.x, 3);
    RowOut o;
    count_unsat<EA>(Sa, Sb, sh, half_of(rym, sa), half_of(ryp, sa), half_of(rzm, sa), half_of(rzp, sa), bd, o.n0,
                    o.n1);
    const uint4 w = philox4x32_10_wide(make_uint4(h0 >> 3, t, r, 2 * kTagHead + c), key);
    const Lut3 K = lut_of(th);
    uint32_t eq = 0xFFFFFFFFu;
    o.F0 = decide4(o.n0, w.x, w.y, K, one2, eq);
    o.F1 = decide4(o.n1, w.z, w.w, K, one2, eq);
    if (__builtin_expect(__any(has_tie(eq)), 0)) exact_decisions(o, w, th, K, h0, c, t, r, key, has_tie(eq));
    return o;
}

// The segment with the flagged own sites flipped (+1 <-> -1: byte ^ 0xFE).
__device__ __forceinline__ uint4 apply_flips(const uint4 &own, const RowOut &o, int A) {
    const uint32_t m0 = bytes_fe(o.F0), m1 = bytes_fe(o.F1);  // 0xFE where flipped
    const uint32_t slo = A ? 0x01040004u : 0x04010400u, shi = A ? 0x03040204u : 0x04030402u;
    return make_uint4(own.x ^ perm(0u, m0, slo), own.y ^ perm(0u, m0, shi), own.z ^ perm(0u, m1, slo),
                      own.w ^ perm(0u, m1, shi));
}

// Energy change of the segment's flips: 12 - 4n for a site with n
// unsatisfied bonds.
__device__ __forceinline__ long long flip_energy(const RowOut &o) {
    const uint32_t f0 = bytes_ff(o.F0), f1 = bytes_ff(o.F1);  // 0xFF where flipped
    const uint32_t cnt = __builtin_amdgcn_sad_u8(o.F0, 0u, __builtin_amdgcn_sad_u8(o.F1, 0u, 0u));
    const uint32_t nsum = __builtin_amdgcn_sad_u8(o.n0 & f0, 0u, __builtin_amdgcn_sad_u8(o.n1 & f1, 0u, 0u));
    return 12 * (long long)cnt - 4 * (long long)nsum;
}

}  // namespace seg3d
}  // namespace smc

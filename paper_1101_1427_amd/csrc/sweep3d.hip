// Checkerboard half-sweeps of uniform 3D Ising and +-J EA batches (Eq. 2 on
// the simple cubic lattice, the 3D update of Sec. 3) with an edge L that is
// a multiple of 16, in place on the caller's row-major int8 spins.
//
// One thread owns one 16-site row segment (x0 .. x0 + 15 of row (y, z)).  It
// loads the segment, the segments of rows y +- 1 and z +- 1 and the one
// site beyond the segment's end that its x neighbours need, splits even-x
// and odd-x sites with byte permutes (the colour-c sites of row (y, z) are
// the even-x ones iff (y + z) & 1 == c), counts the unsatisfied bonds of its
// eight colour-c sites four to a word, and decides them against one Philox
// block: they are the in-colour indices h0 .. h0 + 7 with h0 = i0 / 2 for
// the segment's first site i0, so the block (h0 / 8, t, r, 2*HEAD + c)
// holds their 16-bit heads in order.  The results are those of the per-site
// kernels bit for bit.
//
// Sites of the other colour are stored back unchanged, so a thread that
// reads a segment while its owner writes it sees the same values either way.
#include <stdlib.h>

#include "internal.hpp"

namespace smc {
namespace {

constexpr int kThreads = 256;

struct Sweep3dArgs {
    int8_t *spins;          // replica r at r * L^3
    const int8_t *coup;     // EA: [sample][3][L^3] (bond i -> i + mu at mu * L^3 + i), or nullptr
    int rep_per_sample;
    const ThrRow *thr;      // per replica (high halves <= 0xFFFF, checked on the host)
    int64_t *dE;            // per replica, or nullptr
    Key key;
    uint32_t t;
    int L, c;
    int blocks_per_rep;
    uint32_t one2;  // 0x00010001 (opaque to the compiler, keeps the packed 16-bit ops)
    uint32_t four;  // 4 (opaque trip count of the rarely taken exact-decision loop)
};

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
// reads 0xFFFF, and a head of 0xFFFF takes the exact path.
struct Lut3 {
    uint32_t lo, hi;
};

__device__ __forceinline__ Lut3 lut_of(const ThrRow &row) {
    const uint32_t t3 = row.m[3].x, t2 = row.m[2].x, t1 = row.m[1].x;
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

// One segment: own row raw bytes, neighbours' raw bytes, the extra x
// neighbour bit eb, the per-row bond arrays (EA), Philox block index h0.
template <bool EA>
__device__ __forceinline__ RowOut segment_update(const uint4 &own, const uint4 &rym, const uint4 &ryp,
                                                 const uint4 &rzm, const uint4 &rzp, uint32_t eb, int A,
                                                 const uint4 &jx, uint32_t jeb, const uint4 &jy, const uint4 &jym,
                                                 const uint4 &jz, const uint4 &jzm, const ThrRow &th, uint32_t h0,
                                                 const Sweep3dArgs &a, uint32_t r) {
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
        const uint2 jxa = bits2(half_of(jx, sa)), jxb = bits2(half_of(jx, sb));
        // bond paired with Sb: x -> x + 1 of even-x sites (array a), x - 1 -> x
        // of odd-x sites (array b); bond paired with sh: x + 1 of odd-x sites
        // (array a), x - 1 of even-x sites (array b shifted up, x0 - 1 entering)
        const uint2 bB = A ? jxb : jxa;
        uint2 bS;
        bS.x = A ? jxa.x : ((jxb.x << 8) | jeb);
        bS.y = A ? jxa.y : alignbyte(jxb.y, jxb.x, 3);
        const uint2 jyp = bits2(half_of(jy, sa)), jymb = bits2(half_of(jym, sa));
        const uint2 jzp = bits2(half_of(jz, sa)), jzmb = bits2(half_of(jzm, sa));
        o.n0 = ((Sa.x ^ Sb.x ^ bB.x) + (Sa.x ^ sh.x ^ bS.x)) + ((Sa.x ^ yp.x ^ jyp.x) + (Sa.x ^ ym.x ^ jymb.x)) +
               ((Sa.x ^ zp.x ^ jzp.x) + (Sa.x ^ zm.x ^ jzmb.x));
        o.n1 = ((Sa.y ^ Sb.y ^ bB.y) + (Sa.y ^ sh.y ^ bS.y)) + ((Sa.y ^ yp.y ^ jyp.y) + (Sa.y ^ ym.y ^ jymb.y)) +
               ((Sa.y ^ zp.y ^ jzp.y) + (Sa.y ^ zm.y ^ jzmb.y));
    } else {
        o.n0 = ((Sa.x ^ Sb.x) + (Sa.x ^ sh.x)) + ((Sa.x ^ yp.x) + (Sa.x ^ ym.x)) + ((Sa.x ^ zp.x) + (Sa.x ^ zm.x));
        o.n1 = ((Sa.y ^ Sb.y) + (Sa.y ^ sh.y)) + ((Sa.y ^ yp.y) + (Sa.y ^ ym.y)) + ((Sa.y ^ zp.y) + (Sa.y ^ zm.y));
    }
    const uint32_t c = (uint32_t)a.c;
    const uint4 w = philox4x32_10(make_uint4(h0 >> 3, a.t, r, 2 * kTagHead + c), a.key);
    const Lut3 K = lut_of(th);
    uint32_t eq = 0xFFFFFFFFu;
    o.F0 = decide4(o.n0, w.x, w.y, K, a.one2, eq);
    o.F1 = decide4(o.n1, w.z, w.w, K, a.one2, eq);
    const bool tie = ((eq & 0xFFFFu) == 0u) || ((eq >> 16) == 0u);
    if (__builtin_expect(__any(tie), 0)) {
        if (tie) {
            // exact decisions of the eight sites (a head equal to the high
            // half of its threshold: probability 2^-16 per site)
            uint32_t f0 = 0u, f1 = 0u;
#pragma unroll 1
            for (uint32_t i = 0; i < 2u * a.four; ++i) {
                const uint32_t ns = ((i < 4u ? o.n0 : o.n1) >> (8u * (i & 3u))) & 0xFFu;
                const uint32_t j = i >> 1;
                const uint32_t word = (j & 2u) ? ((j & 1u) ? w.w : w.z) : ((j & 1u) ? w.y : w.x);
                const uint32_t head = (i & 1u) ? (word >> 16) : (word & 0xFFFFu);
                uint32_t flip = 1u;
                if (ns < 3u) flip = metropolis_accept(head, th.m[3u - ns], h0 + i, a.t, r, c, a.key);
                if (i < 4u)
                    f0 |= flip << (8u * (i & 3u));
                else
                    f1 |= flip << (8u * (i & 3u));
            }
            o.F0 = f0;
            o.F1 = f1;
        }
    }
    return o;
}

// Z rows per thread: the segments (x0, y, z0 .. z0 + Z - 1), each row's
// z + 1 neighbour becoming the next row, the row itself the next z - 1.
template <bool EA, int Z, bool NT>
__global__ __launch_bounds__(kThreads) void k_ising3d_half(Sweep3dArgs a) {
    __shared__ long long red[kThreads / 64];
    const int L = a.L;
    const int r = (int)blockIdx.x / a.blocks_per_rep;
    const int64_t g = (int64_t)((int)blockIdx.x % a.blocks_per_rep) * kThreads + threadIdx.x;
    const int segs = L >> 4;
    const int64_t LL = L, P = LL * LL, N = P * LL;
    const bool valid = g < N / (16 * Z);
    long long dE = 0;
    if (valid) {
        const int64_t rowq = g / segs;  // zq * L + y
        const int x0 = (int)(g - rowq * segs) << 4;
        const int y = (int)(rowq % L), z0 = (int)(rowq / L) * Z;
        int8_t *S = a.spins + (int64_t)r * N;
        const int8_t *J = EA ? a.coup + (int64_t)(r / a.rep_per_sample) * 3 * N : nullptr;
        const int64_t dym = y == 0 ? (LL - 1) * LL : -LL, dyp = y == L - 1 ? -(LL - 1) * LL : LL;
        const int64_t xl = x0 == 0 ? L - 1 : x0 - 1, xr = x0 + 16 == L ? 0 : x0 + 16;
        const ThrRow th = a.thr[r];
        int64_t i0 = ((int64_t)z0 * L + y) * LL + x0;
        uint4 rzm = *(const uint4 *)(S + (z0 == 0 ? i0 + (LL - 1) * P : i0 - P));
        uint4 own = *(const uint4 *)(S + i0);
        uint4 jzm = make_uint4(0u, 0u, 0u, 0u), jz = jzm;
        if constexpr (EA) {
            jzm = *(const uint4 *)(J + 2 * N + (z0 == 0 ? i0 + (LL - 1) * P : i0 - P));
            jz = *(const uint4 *)(J + 2 * N + i0);
        }
#pragma unroll(Z < 4 ? Z : 4)
        for (int j = 0; j < Z; ++j) {
            const int z = z0 + j;
            const int64_t izp = z == L - 1 ? i0 - (LL - 1) * P : i0 + P;
            const uint4 rzp = *(const uint4 *)(S + izp);
            const uint4 rym = *(const uint4 *)(S + i0 + dym);
            const uint4 ryp = *(const uint4 *)(S + i0 + dyp);
            const int A = ((y + z) & 1) ^ a.c;
            const int64_t iex = i0 - x0 + (A ? xr : xl);
            const uint32_t eb = ((uint32_t)(uint8_t)S[iex] >> 1) & 1u;
            uint4 jx = make_uint4(0u, 0u, 0u, 0u), jy = jx, jym = jx, jzn = jx;
            uint32_t jeb = 0u;
            if constexpr (EA) {
                jx = *(const uint4 *)(J + i0);
                jeb = ((uint32_t)(uint8_t)J[iex] >> 1) & 1u;
                jy = *(const uint4 *)(J + N + i0);
                jym = *(const uint4 *)(J + N + i0 + dym);
                if (j + 1 < Z) jzn = *(const uint4 *)(J + 2 * N + izp);
            }
            const RowOut o = segment_update<EA>(own, rym, ryp, rzm, rzp, eb, A, jx, jeb, jy, jym, jz, jzm, th,
                                                (uint32_t)(i0 >> 1), a, (uint32_t)r);
            if (o.F0 | o.F1) {
                // byte masks 0xFE (flips +1 <-> -1) placed on the own sites
                const uint32_t m0 = (o.F0 << 8) - (o.F0 << 1), m1 = (o.F1 << 8) - (o.F1 << 1);
                const uint32_t slo = A ? 0x01040004u : 0x04010400u, shi = A ? 0x03040204u : 0x04030402u;
                const uint4 out = make_uint4(own.x ^ perm(0u, m0, slo), own.y ^ perm(0u, m0, shi),
                                             own.z ^ perm(0u, m1, slo), own.w ^ perm(0u, m1, shi));
                if constexpr (NT)
                    __builtin_nontemporal_store(v4u{out.x, out.y, out.z, out.w}, (v4u *)(S + i0));
                else
                    *(uint4 *)(S + i0) = out;
            }
            if (a.dE) {
                // Delta E of a flip with n unsatisfied bonds is 12 - 4n
                const uint32_t f0 = (o.F0 << 8) - o.F0, f1 = (o.F1 << 8) - o.F1;  // 0xFF where flipped
                const uint32_t cnt = __builtin_amdgcn_sad_u8(o.F0, 0u, __builtin_amdgcn_sad_u8(o.F1, 0u, 0u));
                const uint32_t nsum =
                    __builtin_amdgcn_sad_u8(o.n0 & f0, 0u, __builtin_amdgcn_sad_u8(o.n1 & f1, 0u, 0u));
                dE += 12 * (long long)cnt - 4 * (long long)nsum;
            }
            // next row: z + 1 is its own row, this row its z - 1 neighbour (only
            // the other colour's bytes are read from it, which did not change)
            rzm = own;
            own = rzp;
            if constexpr (EA) {
                jzm = jz;
                jz = jzn;
            }
            i0 = izp;
        }
    }
    if (a.dE) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dE += __shfl_xor(dE, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dE;
        __syncthreads();
        if (threadIdx.x == 0) {
            const long long tot = red[0] + red[1] + red[2] + red[3];
            if (tot != 0) atomicAdd((unsigned long long *)&a.dE[r], (unsigned long long)tot);
        }
    }
}

}  // namespace

bool sweep3d_supported(int L) { return L >= 16 && L % 16 == 0; }

namespace {

// Rows per thread along z: Z rows fetch Z + 2 row segments of every column
// instead of 3 Z, so a launch reads the lattice (Z + 2) / Z times.  Z = 4
// (the default) runs the Ising sweep at 512^3 and 1024^3 about 20 % faster
// than Z = 1; 8 and 16 fetch less but leave fewer threads and are no
// faster.  SPINMC_SWEEP3D_Z = 1, 2, 4, 8 or 16 sets it; non-temporal stores
// of the updated segments are on unless SPINMC_SWEEP3D_NT = 0.
int sweep3d_rows() {
    const char *env = getenv("SPINMC_SWEEP3D_Z");
    if (env && env[0]) {
        const int z = atoi(env);
        if (z == 1 || z == 2 || z == 4 || z == 8 || z == 16) return z;
    }
    return 4;
}

bool sweep3d_nt() {
    const char *env = getenv("SPINMC_SWEEP3D_NT");
    return !(env && env[0] == '0');
}

template <bool EA, int Z>
void launch_rows(bool nt, unsigned blocks, const Sweep3dArgs &a, hipStream_t s) {
    if (nt)
        hipLaunchKernelGGL((k_ising3d_half<EA, Z, true>), dim3(blocks), dim3(kThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_ising3d_half<EA, Z, false>), dim3(blocks), dim3(kThreads), 0, s, a);
}

template <bool EA>
void launch_model(int Z, bool nt, unsigned blocks, const Sweep3dArgs &a, hipStream_t s) {
    if (Z == 16)
        launch_rows<EA, 16>(nt, blocks, a, s);
    else if (Z == 8)
        launch_rows<EA, 8>(nt, blocks, a, s);
    else if (Z == 4)
        launch_rows<EA, 4>(nt, blocks, a, s);
    else if (Z == 2)
        launch_rows<EA, 2>(nt, blocks, a, s);
    else
        launch_rows<EA, 1>(nt, blocks, a, s);
}

}  // namespace

hipError_t launch_ising3d_half(int8_t *spins, const int8_t *coup, int rep_per_sample, const ThrRow *thr,
                               int64_t *dE, int n_rep, int L, Key key, uint32_t t, int c, hipStream_t s) {
    if (!sweep3d_supported(L) || rep_per_sample < 1 || n_rep < 1) return hipErrorInvalidValue;
    // a replica's (L / 16)^3 workgroups of one-row threads regroup into whole
    // workgroups of Z-row threads when Z divides (L / 16)^3
    const int B = L / 16;
    int Z = sweep3d_rows();
    while ((B * B * B) % Z) Z >>= 1;
    const int64_t threads = (int64_t)L * L * L / (16 * Z);  // per replica
    Sweep3dArgs a;
    a.spins = spins;
    a.coup = coup;
    a.rep_per_sample = rep_per_sample;
    a.thr = thr;
    a.dE = dE;
    a.key = key;
    a.t = t;
    a.L = L;
    a.c = c;
    a.blocks_per_rep = (int)((threads + kThreads - 1) / kThreads);
    a.one2 = 0x00010001u;
    a.four = 4u;
    const int64_t blocks = (int64_t)n_rep * a.blocks_per_rep;
    if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
    if (coup)
        launch_model<true>(Z, sweep3d_nt(), (unsigned)blocks, a, s);
    else
        launch_model<false>(Z, sweep3d_nt(), (unsigned)blocks, a, s);
    return hipGetLastError();
}

}  // namespace smc

// One-pass checkerboard sweep of large 2D Ising lattices (L a multiple of
// 1024) on an internal colour-split layout.
//
// Layout.  Inside a multi-sweep call the lattice lives in two byte planes
// per replica: plane c, row y, index k holds the spin at x = 2k + ((y+c)&1)
// (the colour-c sites of the row), as 0 (+1) or 1 (-1).  A colour-c site at
// (k, y) then has its four neighbours in plane 1-c: (k, y-1), (k, y+1) and,
// in its own row, (k-1, k) when (y+c) is even or (k, k+1) when it is odd.
// Every 32-bit word holds four sites of one colour, so all arithmetic is on
// sites that are updated together.
//
// Sweep.  Colour 0 then colour 1 (Sec. 3.2) in a single pass: a workgroup
// owns whole rows [Y0, Y0+H) and streams down them.  For row j it first
// updates colour 0 (including the halo rows Y0-1 and Y0+H, recomputed
// identically by the neighbouring band because every draw is keyed by the
// site), then colour 1 of row j-1 from the new colour-0 rows j-2, j-1, j.
// Reads come from one buffer and writes go to the other (ping-pong), so
// bands never see each other's new values.  HBM traffic per sweep: each
// spin read once and written once (plus 4 halo rows per band).  Rows are
// stored in lattice order with a padded pitch.
//
// Caller's layout.  The first sweep of a call can read the caller's
// row-major int8 +-1 lattice directly (a feed is then one whole row, split
// into the two planes by the compute waves, whose plane-0 half is kept in
// registers for the next step), and the last sweep can write it directly
// (both planes of a finished row interleaved back into the row), so a call
// moves no bytes beyond its sweeps.
//
// Decision (Eq. 2 with integer thresholds).  Per site the number n of
// antiparallel neighbours gives dE = 8 - 4n; n >= 2 always flips.  The
// 16-bit head of the site's uniform is compared with the 16-bit high part
// T of the threshold by packed saturating subtraction, two sites per
// instruction; T per site comes from a byte-permute lookup on n.  Equality
// head == T (probability 2^-16) sends the wave to an exact per-site path
// that draws the 16-bit tail.
#include <stdlib.h>

#include "internal.hpp"
#include "intrin.hpp"
#include "lattice2d.hpp"

namespace smc {
namespace {

// (a ^ b) + c in one v_xad_u32 (register operands only, no memory access).
__device__ __forceinline__ uint32_t xad(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_xad_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Per-replica constants of the decision.
struct Lut {
    uint32_t tlo_lo, tlo_hi, thi_lo, thi_hi;  // T(n): low / high bytes, selectors n = 0..7
    uint32_t de_lo, de_hi;                    // dE/4 + 2 for index n + 4F
    uint32_t one2;                            // 0x00010001
    uint2 thr1, thr2;                         // exact thresholds of dE = 4 and dE = 8
};

// The row is the workgroup's (one replica per band).  With SCALAR its
// words are moved to scalar registers: the compiler loads the row with a
// vector load (the kernel also writes global memory) and holds the exact
// thresholds of the tie path in vector registers, which the variant reading
// the caller's rows spilled to scratch, reloading them from memory at every
// tie while the rest of the workgroup waited at the next barrier (about 50
// us more for that sweep at 3 x 16384^2).  The other variants do not spill
// and run 0.5 % faster with the vector copy.
template <bool SCALAR>
__device__ __forceinline__ Lut make_lut(const ThrRow &row_in, uint32_t one2) {
    ThrRow row = row_in;
    if constexpr (SCALAR) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            row.m[i] = make_uint2(__builtin_amdgcn_readfirstlane(row_in.m[i].x),
                                  __builtin_amdgcn_readfirstlane(row_in.m[i].y));
    }
    Lut k;
    const uint32_t t2 = row.m[2].x, t1 = row.m[1].x;  // both <= 0xFFFF (checked on the host)
    k.tlo_lo = (t2 & 0xFFu) | ((t1 & 0xFFu) << 8) | 0xFFFF0000u;
    k.thi_lo = (t2 >> 8) | ((t1 >> 8) << 8) | 0xFFFF0000u;
    k.tlo_hi = 0xFFFFFFFFu;
    k.thi_hi = 0xFFFFFFFFu;
    // index n + 4F: F=0 -> 2 (no change); F=1 -> 4 - n; index 8 (n = 4) reads
    // the sign of byte 1 (= 2 > 0), i.e. 0 = 4 - 4.
    k.de_lo = 0x02020202u;
    k.de_hi = 0x01020304u;
    k.one2 = one2;
    k.thr1 = row.m[1];
    k.thr2 = row.m[2];
    return k;
}

template <int C>
struct Row {
    uint32_t d[2 * C];  // 8*C sites of one plane row (4 per word)
};

template <int C>
__device__ __forceinline__ Row<C> load_row(const uint8_t *p) {
    Row<C> r;
    if constexpr (C == 1) {
        const uint2 v = *(const uint2 *)p;
        r.d[0] = v.x;
        r.d[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < C / 2; ++i) {
            const uint4 v = ((const uint4 *)p)[i];
            r.d[4 * i] = v.x;
            r.d[4 * i + 1] = v.y;
            r.d[4 * i + 2] = v.z;
            r.d[4 * i + 3] = v.w;
        }
    }
    return r;
}

// Rows are written once per sweep and read again only by the next sweep, so
// the stores are non-temporal (streamed past the caches).
template <int C>
__device__ __forceinline__ void store_row(uint8_t *p, const Row<C> &r) {
    typedef uint32_t v2 __attribute__((ext_vector_type(2)));
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    if constexpr (C == 1) {
        const v2 x = {r.d[0], r.d[1]};
        __builtin_nontemporal_store(x, (v2 *)p);
    } else {
#pragma unroll
        for (int i = 0; i < C / 2; ++i) {
            const v4 x = {r.d[4 * i], r.d[4 * i + 1], r.d[4 * i + 2], r.d[4 * i + 3]};
            __builtin_nontemporal_store(x, (v4 *)p + i);
        }
    }
}

// Number of antiparallel neighbours of the four sites in word i of `own`
// (0/1 bytes): vertical words va, vb, horizontal row hz with the word of the
// neighbouring lane `edge` (left neighbour word if p == 0, right if p == 1).
template <int C>
__device__ __forceinline__ uint32_t count_anti(uint32_t own, uint32_t va, uint32_t vb, const Row<C> &hz, int i,
                                               uint32_t edge, int p) {
    uint32_t sh;
    if (p == 0) {
        const uint32_t lo = i == 0 ? edge : hz.d[i - 1];
        sh = alignbyte(hz.d[i], lo, 3);
    } else {
        const uint32_t hi = i == 2 * C - 1 ? edge : hz.d[i + 1];
        sh = alignbyte(hi, hz.d[i], 1);
    }
    // one xor and three xor-adds (the compiler otherwise rebalances the sum
    // into four xors and two adds)
    uint32_t n = own ^ sh;
    n = xad(own, hz.d[i], n);
    n = xad(own, vb, n);
    return xad(own, va, n);
}

// Flip flags (bit 0 of each byte) of the four sites with counts n and heads
// in words wa (sites 0, 1) and wb (sites 2, 3); eq collects head - T.
__device__ __forceinline__ uint32_t decide4(uint32_t n, uint32_t wa, uint32_t wb, const Lut &K, uint32_t &eq) {
    const uint32_t tl = perm(K.tlo_hi, K.tlo_lo, n);
    const uint32_t th = perm(K.thi_hi, K.thi_lo, n);
    const uint32_t ta = perm(th, tl, 0x05010400u);
    const uint32_t tb = perm(th, tl, 0x07030602u);
    const uint32_t ra = min16(sub_sat16(ta, wa), K.one2);
    const uint32_t rb = min16(sub_sat16(tb, wb), K.one2);
    eq = min16(eq, min16(sub16(ta, wa), sub16(tb, wb)));
    return perm(rb, ra, 0x06040200u);
}

struct Lattice2dArgs {
    const uint8_t *src;  // replica 0 read: split planes, or the caller's int8 rows (IO & kAbiIn)
    uint8_t *dst;        // replica 0 written: split planes, or the caller's int8 rows (IO & kAbiOut)
    int64_t src_rep, dst_rep;      // bytes per replica (split: 2 planes of L rows at the pitch; rows: L*L)
    int64_t src_pitch, dst_pitch;  // bytes between consecutive rows (split plane: >= L/2; rows: L)
    const ThrRow *thr;   // per replica
    int64_t *dE_part;    // per compute wave of every workgroup (workgroup-major), or nullptr
    int dE_first;        // 1: this launch writes the partial sums, 0: adds to them
    Key key;
    uint32_t t;
    int L, H, bands, n_rep;
    int H2, nb1;    // bands 0 .. nb1-1 of a replica have H rows, the others H2 rows
    uint32_t one2;  // 0x00010001, passed in so that the compiler keeps the packed ops
};

// Decide and apply colour c of one lane-row: own (updated in place),
// vertical rows va / vb, horizontal row hz with the neighbouring lane's word
// `edge`, draws w[q] of chunk q.  Adds sum(dE/4 + 2) into de_total when
// `count`.
template <int C>
__device__ __forceinline__ void apply_row(Row<C> &own, const Row<C> &va, const Row<C> &vb, const Row<C> &hz,
                                          uint32_t edge, int p, const uint4 (&w)[C], uint32_t g0, uint32_t c,
                                          const Lut &K, Key key, uint32_t t, uint32_t r, bool count,
                                          uint32_t &de_total) {
    uint32_t n[2 * C], F[2 * C];
    uint32_t eq = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < 2 * C; ++i) {
        n[i] = count_anti<C>(own.d[i], va.d[i], vb.d[i], hz, i, edge, p);
        const uint4 &wq = w[i >> 1];
        F[i] = decide4(n[i], (i & 1) ? wq.z : wq.x, (i & 1) ? wq.w : wq.y, K, eq);
    }
    // a head equal to the high half of its threshold: decide those sites exactly
    const bool tie = ((eq & 0xFFFFu) == 0u) || ((eq >> 16) == 0u);
    if (__builtin_expect(__any(tie), 0)) {
        // Ties are rare (probability 2^-16 per site), but a wavefront that
        // meets one holds up its workgroup at the next barrier, so this path
        // is kept short: a mask of the tied sites (bit 4 i + s for site s of
        // word i), then one pass per tied site of the lane with most of them
        // (almost always one), each drawing the single tail it needs.
        uint32_t tm = 0;
#pragma unroll
        for (int i = 0; i < 2 * C; ++i) {
            const uint4 &wq = w[i >> 1];
            const uint32_t tl = perm(K.tlo_hi, K.tlo_lo, n[i]), th = perm(K.thi_hi, K.thi_lo, n[i]);
            const uint32_t da = perm(th, tl, 0x05010400u) ^ ((i & 1) ? wq.z : wq.x);
            const uint32_t db = perm(th, tl, 0x07030602u) ^ ((i & 1) ? wq.w : wq.y);
            const uint32_t m4 = ((da & 0xFFFFu) == 0u ? 1u : 0u) | ((da >> 16) == 0u ? 2u : 0u) |
                                ((db & 0xFFFFu) == 0u ? 4u : 0u) | ((db >> 16) == 0u ? 8u : 0u);
            tm |= m4 << (4 * i);
        }
        while (__any(tm != 0u)) {
            if (tm != 0u) {
                const uint32_t s = __builtin_ctz(tm), wi = s >> 2, s4 = s & 3u;
                tm &= tm - 1u;
                uint32_t nw = n[0];
#pragma unroll
                for (int i = 1; i < 2 * C; ++i) nw = wi == (uint32_t)i ? n[i] : nw;
                const uint32_t ns = (nw >> (8u * s4)) & 0xFFu;
                uint32_t flip = 1u;  // a head of 0xFFFF at a site with Delta E <= 0
                if (ns < 2u) {
                    // the head equals the threshold's high half: compare the tail
                    const uint2 th = ns == 0u ? K.thr2 : K.thr1;
                    const uint32_t h = (g0 + (s >> 3)) * 8u + (s & 7u);
                    flip = tail16(h, t, r, c, key) < th.y ? 1u : 0u;
                }
                const uint32_t keep = ~(0xFFu << (8u * s4)), set = flip << (8u * s4);
#pragma unroll
                for (int i = 0; i < 2 * C; ++i) F[i] = wi == (uint32_t)i ? (F[i] & keep) | set : F[i];
            }
        }
    }
    uint32_t de = 0;
#pragma unroll
    for (int i = 0; i < 2 * C; ++i) {
        own.d[i] ^= F[i];
        de += perm(K.de_hi, K.de_lo, (F[i] << 2) + n[i]);
    }
    if (count) de_total = __builtin_amdgcn_sad_u8(de, 0u, de_total);
}

// Neighbour-lane words: every lane receives the last word of the lane to
// its left (dir 0, DPP wave_shr:1) or the first word of the lane to its
// right (dir 1, wave_shl:1); the lanes at a wave's ends take the word of the
// neighbouring wave through LDS, and the row wraps around the workgroup.
template <int DIR>
__device__ __forceinline__ void exchange2(uint32_t v1, uint32_t v0, uint32_t *xch, int par, uint32_t &e1,
                                          uint32_t &e0, int nw) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == (DIR ? 0 : 63)) {
        xch[(par * nw + wave) * 2] = v1;
        xch[(par * nw + wave) * 2 + 1] = v0;
    }
    __syncthreads();
    const int other = DIR ? (wave + 1 == nw ? 0 : wave + 1) : (wave == 0 ? nw - 1 : wave - 1);
    const uint32_t o1 = xch[(par * nw + other) * 2];
    const uint32_t o0 = xch[(par * nw + other) * 2 + 1];
    constexpr int ctrl = DIR ? 0x130 : 0x138;  // wave_shl:1 : wave_shr:1
    e1 = (uint32_t)__builtin_amdgcn_update_dpp((int)o1, (int)v1, ctrl, 0xF, 0xF, false);
    e0 = (uint32_t)__builtin_amdgcn_update_dpp((int)o0, (int)v0, ctrl, 0xF, 0xF, false);
}

// ------------------------------------------------------------ pipeline ----
// Warp-specialised band pipeline.  A workgroup = NCW compute waves that span
// one full row + one loader wave.  The loader streams the rows the compute
// waves need into an LDS ring with direct global->LDS loads, kDepth steps
// ahead; the compute waves read new rows from LDS and only store to global
// memory.  On this target loads and stores share one completion counter, so
// a wave that both loads and stores must drain its stores whenever it waits
// for data; with the roles split, the loader waits only for its own loads
// (in issue order, so the wait count is exact) and the compute waves never
// wait for global memory at all.
constexpr int kDepth = 3;                // feeds in flight ahead of the consumer
constexpr int kSlots = kDepth + 1;       // LDS ring slots per plane

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(3))) uint8_t lds_u8_t;

template <int C>
__device__ __forceinline__ Row<C> lds_row(const uint8_t *p) {
    Row<C> r;
    if constexpr (C == 1) {
        const uint2 v = *(const uint2 *)p;
        r.d[0] = v.x;
        r.d[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < C / 2; ++i) {
            const uint4 v = ((const uint4 *)p)[i];
            r.d[4 * i] = v.x;
            r.d[4 * i + 1] = v.y;
            r.d[4 * i + 2] = v.z;
            r.d[4 * i + 3] = v.w;
        }
    }
    return r;
}

// s_waitcnt for vmcnt <= N only (expcnt / lgkmcnt left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}


// IO flags of a launch: the source / destination is the caller's row-major
// int8 +-1 lattice instead of the split planes.
constexpr int kAbiIn = 1, kAbiOut = 2;

template <int C>
struct Band {
    const uint8_t *S0, *S1;  // split source planes (S0 alone: the source rows when reading the caller's layout)
    uint8_t *D0, *D1;        // split destination planes (D0 alone: the destination rows)
    int L, half, Y0, H, ncw;
    int64_t pin, pout;       // row pitch of source and destination
    int64_t lane_off;
    uint32_t gpr, lg0, r, t;
    Key key;
    Lut K;
    __device__ __forceinline__ int wrap(int y) const { return y < 0 ? y + L : (y >= L ? y - L : y); }
    __device__ __forceinline__ int64_t off(int y) const { return (int64_t)wrap(y) * pin; }
    __device__ __forceinline__ int64_t off_out(int y) const { return (int64_t)wrap(y) * pout; }
};

// Caller's layout <-> split planes.  A row's 16C bytes x0 .. x0+16C-1 (x0 a
// multiple of 16C) hold its sites as int8 +-1; the split rows hold the even-x
// and the odd-x sites of that range as 0 (+1) / 1 (-1) bytes.  Plane p of row
// y holds the sites with x = 2k + ((y + p) & 1).
template <int C>
__device__ __forceinline__ void split_row(const Row<2 * C> &v, Row<C> &even, Row<C> &odd) {
    const uint32_t m = 0x01010101u;
#pragma unroll
    for (int i = 0; i < 2 * C; ++i) {
        const uint32_t b0 = (v.d[2 * i] >> 1) & m, b1 = (v.d[2 * i + 1] >> 1) & m;
        even.d[i] = perm(b1, b0, 0x06040200u);
        odd.d[i] = perm(b1, b0, 0x07050301u);
    }
}


// A lane writes 32 consecutive bytes of the row as two 16-byte stores, so
// one store instruction covers every other 16 bytes of a 2 KB span.  These
// stores go through the caches, which join the two halves of every line
// before it reaches memory: non-temporal stores wrote 1.38 times the row
// bytes (partial lines) and made the last sweep of a call 16 % slower.
template <int C>
__device__ __forceinline__ void store_joined_row(uint8_t *p, const Row<C> &even, const Row<C> &odd) {
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const uint32_t e0 = even.d[2 * i], o0 = odd.d[2 * i], e1 = even.d[2 * i + 1], o1 = odd.d[2 * i + 1];
        const v4 x = {bytes_pm1(perm(o0, e0, 0x05010400u)), bytes_pm1(perm(o0, e0, 0x07030602u)),
                      bytes_pm1(perm(o1, e1, 0x05010400u)), bytes_pm1(perm(o1, e1, 0x07030602u))};
        ((v4 *)p)[i] = x;
    }
}

// Loader waves: the feed of step s (plane-1 row s+1, plane-0 row s) goes to
// ring slot (s - Y0 + 1) % kSlots.  A feed is NF direct-load instructions,
// each moving 16 bytes per lane (1 KB per wave) of one plane row of L/2
// bytes (a 512-byte row, L = 1024, uses half the lanes); loader wave lw of
// NLW issues instructions lw, lw + NLW, ...
template <int NF>
struct LoaderShape {
    static constexpr int NLW = NF >= 4 ? 4 : NF;  // loader waves
    static constexpr int PER = NF / NLW;          // instructions per loader wave per feed
};

template <int C, int NF, int IO>
__device__ __forceinline__ void issue_feed(const Band<C> &B, int s, uint8_t *ring, int lw) {
    using SH = LoaderShape<NF>;
    const int slot = (s - B.Y0 + 1) % kSlots;
    const int lane = threadIdx.x & 63;
    constexpr int per_plane = NF / 2;
    const bool active = 16 * lane < B.half;
#pragma unroll
    for (int q = 0; q < SH::PER; ++q) {
        const int ins = lw + q * SH::NLW;  // instruction index within the feed
        if constexpr (IO & kAbiIn) {
            // the whole caller's row s+1 (L bytes) into slot `slot` (L bytes),
            // instruction ins moving bytes [seg * ins, seg * (ins + 1))
            const int seg = B.half < 1024 ? B.half : 1024;
            const uint8_t *src = B.S0 + B.off(s + 1) + (int64_t)seg * ins;
            uint8_t *dst = ring + (size_t)slot * (size_t)B.L + (size_t)seg * ins;
            if (active)
                __builtin_amdgcn_global_load_lds(src + 16 * lane, (lds_void_t *)(lds_u8_t *)dst, 16, 0, 0);
        } else {
            const int pl = ins / per_plane, k = ins % per_plane;
            const int row = pl == 0 ? s + 1 : s;  // pl 0: plane 1, pl 1: plane 0
            const uint8_t *src = (pl == 0 ? B.S1 : B.S0) + B.off(row);
            uint8_t *dst = ring + (size_t)(pl * kSlots + slot) * (size_t)B.half;
            if (active)
                __builtin_amdgcn_global_load_lds(src + 1024 * k + 16 * lane,
                                                 (lds_void_t *)(lds_u8_t *)(dst + 1024 * k), 16, 0, 0);
        }
    }
}

// Workgroup barrier without the memory fence of __syncthreads(): the fence
// would make the loaders drain all of their direct loads at every step.  The
// loaders order their LDS writes explicitly (wait_vmcnt before the barrier).
__device__ __forceinline__ void loader_barrier() { __builtin_amdgcn_s_barrier(); }

template <int C, int NF, int IO>
__device__ void loader_loop(const Band<C> &B, uint8_t *ring, int lw) {
    using SH = LoaderShape<NF>;
    const int first = B.Y0 - 1, last = B.Y0 + B.H;  // steps
    // prologue: feeds of steps first .. first+kDepth-1, then the first one must land
#pragma unroll
    for (int d = 0; d < kDepth; ++d) issue_feed<C, NF, IO>(B, first + d, ring, lw);
    wait_vmcnt<SH::PER *(kDepth - 1)>();
    loader_barrier();  // (1) prologue
    loader_barrier();  // (2) initial edge exchange of the compute waves
    for (int s = first; s < last; ++s) {
        // step s is running on the compute waves; bring in step s+kDepth, make s+1 land
        if (s + kDepth <= last) {
            issue_feed<C, NF, IO>(B, s + kDepth, ring, lw);
            wait_vmcnt<SH::PER *(kDepth - 1)>();
        } else {
            wait_vmcnt<0>();
        }
        loader_barrier();  // end of step s
    }
}

// Compute waves, step j: colour 0 of row j, colour 1 of row j-1, store row
// j-1, exchange the edge words of step j+1.  Row y of plane 1 is kept in
// p1[y & 3], new row y of plane 0 in n0[y & 3].
template <int C>
struct Pipe {
    Row<C> p1[4], n0[4];
    Row<C> next0;  // reading the caller's layout: plane-0 half of the row fed last step
    uint32_t e1, e0;
    uint32_t de_total, counted;
};

template <int C, int PH, int IO>
__device__ __forceinline__ void step(Pipe<C> &S, const Band<C> &B, int j, const uint8_t *ring, uint32_t *xch) {
    constexpr int a_m1 = (PH + 3) & 3, a_0 = PH & 3, a_p1 = (PH + 1) & 3, a_m2 = (PH + 2) & 3;
    constexpr int P = PH & 1;
    __builtin_amdgcn_sched_barrier(0);
    // new rows from the ring: plane-1 row j+1, plane-0 row j
    const int slot = (j - B.Y0 + 1) % kSlots;
    Row<C> own0;
    if constexpr (IO & kAbiIn) {
        // the caller's row j+1: plane 1 now, plane 0 at the next step (row
        // y = j+1 has parity (PH+1) & 1 since bands start at multiples of 4)
        const Row<2 * C> full = lds_row<2 * C>(ring + (size_t)slot * B.L + 2 * B.lane_off);
        Row<C> ev, od;
        split_row<C>(full, ev, od);
        own0 = S.next0;
        if constexpr (((PH + 1) & 1) == 1) {
            S.p1[a_p1] = ev;
            S.next0 = od;
        } else {
            S.p1[a_p1] = od;
            S.next0 = ev;
        }
    } else {
        S.p1[a_p1] = lds_row<C>(ring + (size_t)slot * B.half + B.lane_off);
        own0 = lds_row<C>(ring + (size_t)(kSlots + slot) * B.half + B.lane_off);
    }
    const int jw = j < 0 ? j + B.L : (j >= B.L ? j - B.L : j);
    const uint32_t row0 = (uint32_t)jw;
    const uint32_t row1 = jw == 0 ? (uint32_t)B.L - 1u : (uint32_t)jw - 1u;
    const uint32_t g0 = row0 * B.gpr + B.lg0, g1 = row1 * B.gpr + B.lg0;
    uint4 w[2 * C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
        w[q] = make_uint4(g0 + q, B.t, B.r, 2 * kTagHead + 0);
        w[C + q] = make_uint4(g1 + q, B.t, B.r, 2 * kTagHead + 1);
    }
    philox4x32_10_multi<2 * C>(w, B.key);
    uint4 w0[C], w1[C];
#pragma unroll
    for (int q = 0; q < C; ++q) {
        w0[q] = w[q];
        w1[q] = w[C + q];
    }
    // colour 0, row j
    const bool in0 = j >= B.Y0 && j < B.Y0 + B.H;
    apply_row<C>(own0, S.p1[a_m1], S.p1[a_p1], S.p1[a_0], S.e1, P, w0, g0, 0u, B.K, B.key, B.t, B.r, in0,
                 S.de_total);
    S.n0[a_0] = own0;
    S.counted += in0 ? 1u : 0u;
    if (j >= B.Y0 + 1) {
        // colour 1, row j-1, from the new colour-0 rows j-2, j-1, j
        apply_row<C>(S.p1[a_m1], S.n0[a_m2], S.n0[a_0], S.n0[a_m1], S.e0, P, w1, g1, 1u, B.K, B.key, B.t, B.r, true,
                     S.de_total);
        S.counted += 1u;
        if constexpr (IO & kAbiOut) {
            // row j-1 (parity (PH+1) & 1): even x in plane (y & 1), odd x in the other
            if constexpr (((PH + 1) & 1) == 1)
                store_joined_row<C>(B.D0 + B.off_out(j - 1) + 2 * B.lane_off, S.p1[a_m1], S.n0[a_m1]);
            else
                store_joined_row<C>(B.D0 + B.off_out(j - 1) + 2 * B.lane_off, S.n0[a_m1], S.p1[a_m1]);
        } else {
            store_row<C>(B.D0 + B.off_out(j - 1) + B.lane_off, S.n0[a_m1]);
            store_row<C>(B.D1 + B.off_out(j - 1) + B.lane_off, S.p1[a_m1]);
        }
    }
    if (j < B.Y0 + B.H) {
        // edges for step j+1: plane-1 old row j+1 and plane-0 new row j
        constexpr int D = (PH + 1) & 1;
        exchange2<D>(D ? S.p1[a_p1].d[0] : S.p1[a_p1].d[2 * C - 1], D ? S.n0[a_0].d[0] : S.n0[a_0].d[2 * C - 1], xch,
                     PH & 1, S.e1, S.e0, B.ncw);
    }
}

template <int C, int IO>
__device__ void compute_loop(const Band<C> &B, const uint8_t *ring, uint32_t *xch, int64_t *dE_part, bool first) {
    Pipe<C> S;
    const int Y0 = B.Y0;  // a multiple of 4: step Y0-1 has phase 3
    // rows Y0-2 and Y0-1 of plane 1 (all later rows come through the ring)
    if constexpr (IO & kAbiIn) {
        // caller's rows Y0-2 (even: plane 1 holds its odd x) and Y0-1 (odd:
        // plane 1 holds its even x, plane 0 its odd x, needed at step Y0-1)
        Row<C> ev, od;
        split_row<C>(load_row<2 * C>(B.S0 + B.off(Y0 - 2) + 2 * B.lane_off), ev, od);
        S.p1[2] = od;
        split_row<C>(load_row<2 * C>(B.S0 + B.off(Y0 - 1) + 2 * B.lane_off), ev, od);
        S.p1[3] = ev;
        S.next0 = od;
    } else {
        S.p1[2] = load_row<C>(B.S1 + B.off(Y0 - 2) + B.lane_off);
        S.p1[3] = load_row<C>(B.S1 + B.off(Y0 - 1) + B.lane_off);
    }
#pragma unroll
    for (int i = 0; i < 2 * C; ++i) S.n0[0].d[i] = S.n0[1].d[i] = S.n0[2].d[i] = S.n0[3].d[i] = 0u;
    S.de_total = 0;
    S.counted = 0;
    S.e0 = 0;
    __syncthreads();  // (1) prologue: the first feed has landed
    {
        // plane-1 row Y0-1 is odd: its colour-0 sites need the right neighbour word
        uint32_t dummy;
        exchange2<1>(S.p1[3].d[0], 0u, xch, 0, S.e1, dummy, B.ncw);  // (2)
    }
    step<C, 3, IO>(S, B, Y0 - 1, ring, xch);
    for (int j = Y0; j < Y0 + B.H; j += 4) {
        step<C, 0, IO>(S, B, j, ring, xch);
        step<C, 1, IO>(S, B, j + 1, ring, xch);
        step<C, 2, IO>(S, B, j + 2, ring, xch);
        step<C, 3, IO>(S, B, j + 3, ring, xch);
    }
    step<C, 0, IO>(S, B, Y0 + B.H, ring, xch);
    if (dE_part) {
        // sum over sites of (dE/4 + 2) minus 2 per counted site, into this
        // wave's own slot (no other wave touches it, so no atomics)
        long long v = ((long long)S.de_total - 2ll * (long long)S.counted * 8 * C) * 4;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) {
            int64_t *slot = dE_part + (int64_t)blockIdx.x * B.ncw + (threadIdx.x >> 6);
            *slot = first ? v : *slot + v;
        }
    }
}

// At least six waves per SIMD: two workgroups of eight compute and four
// loader waves per compute unit (at most 80 registers).
template <int C, int NF, int IO>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6))) void k_ising2d_split(Lattice2dArgs a) {
    // ring: [2 planes][kSlots][L/2] (split source) or [kSlots][L] (caller's rows), then the edge words
    extern __shared__ __align__(16) uint8_t smem[];
    const int ncw = (int)(blockDim.x >> 6) - LoaderShape<NF>::NLW;  // compute waves; the last NLW waves load
    uint8_t *ring = smem;
    uint32_t *xch = (uint32_t *)(smem + (size_t)2 * kSlots * (a.L >> 1));
    const int r = (int)(blockIdx.x / (uint32_t)a.bands);
    const int band = (int)(blockIdx.x % (uint32_t)a.bands);
    Band<C> B;
    B.L = a.L;
    B.half = a.L >> 1;
    B.H = band < a.nb1 ? a.H : a.H2;
    B.Y0 = band < a.nb1 ? band * a.H : a.nb1 * a.H + (band - a.nb1) * a.H2;
    B.pin = a.src_pitch;
    B.pout = a.dst_pitch;
    B.ncw = ncw;
    B.S0 = a.src + (int64_t)r * a.src_rep;
    B.S1 = B.S0 + B.pin * a.L;
    B.D0 = a.dst + (int64_t)r * a.dst_rep;
    B.D1 = B.D0 + B.pout * a.L;
    B.lane_off = (int64_t)threadIdx.x * 8 * C;
    B.gpr = (uint32_t)a.L >> 4;  // draw groups per row (8 sites each)
    B.lg0 = threadIdx.x * C;     // this lane's first group in a row
    B.r = (uint32_t)r;
    B.t = a.t;
    B.key = a.key;
    if ((int)(threadIdx.x >> 6) >= ncw) {
        loader_loop<C, NF, IO>(B, ring, (int)(threadIdx.x >> 6) - ncw);
    } else {
        B.K = make_lut<(IO & kAbiIn) != 0>(a.thr[r], a.one2);
        compute_loop<C, IO>(B, ring, xch, a.dE_part, a.dE_first != 0);
    }
}

// ----------------------------------------------------- layout conversion ----
// ABI row-major int8 +-1  <->  split planes of 0/1 bytes (x even -> plane
// (y&1), x odd -> plane ((y+1)&1), plane index x/2).
__global__ __launch_bounds__(256) void k_to_split(const int8_t *src, uint8_t *dst, int L, int64_t pitch,
                                                  int64_t chunks_per_rep, int64_t total) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const int64_t r = gid / chunks_per_rep, cidx = gid % chunks_per_rep;
    const int cpr = L >> 4;  // 16-site chunks per row
    const int y = (int)(cidx / cpr), xc = (int)(cidx % cpr);
    const int64_t N = (int64_t)L * L, P = (int64_t)L * pitch;  // sites, bytes per plane
    const uint4 v = *(const uint4 *)(src + r * N + (int64_t)y * L + 16 * xc);
    const uint32_t m = 0x01010101u;
    const uint32_t b0 = (v.x >> 1) & m, b1 = (v.y >> 1) & m, b2 = (v.z >> 1) & m, b3 = (v.w >> 1) & m;
    const uint2 ev = make_uint2(perm(b1, b0, 0x06040200u), perm(b3, b2, 0x06040200u));
    const uint2 od = make_uint2(perm(b1, b0, 0x07050301u), perm(b3, b2, 0x07050301u));
    uint8_t *base = dst + r * 2 * P;
    const int64_t off = (int64_t)y * pitch + 8 * xc;
    const int pe = y & 1, po = (y + 1) & 1;
    *(uint2 *)(base + pe * P + off) = ev;
    *(uint2 *)(base + po * P + off) = od;
}

__global__ __launch_bounds__(256) void k_from_split(const uint8_t *src, int8_t *dst, int L, int64_t pitch,
                                                    int64_t chunks_per_rep, int64_t total) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const int64_t r = gid / chunks_per_rep, cidx = gid % chunks_per_rep;
    const int cpr = L >> 4;
    const int y = (int)(cidx / cpr), xc = (int)(cidx % cpr);
    const int64_t N = (int64_t)L * L, P = (int64_t)L * pitch;
    const uint8_t *base = src + r * 2 * P;
    const int64_t off = (int64_t)y * pitch + 8 * xc;
    const int pe = y & 1, po = (y + 1) & 1;
    const uint2 ev = *(const uint2 *)(base + pe * P + off);
    const uint2 od = *(const uint2 *)(base + po * P + off);
    const uint32_t e0 = bytes_pm1(ev.x), e1 = bytes_pm1(ev.y), o0 = bytes_pm1(od.x), o1 = bytes_pm1(od.y);
    uint4 v;
    v.x = perm(o0, e0, 0x05010400u);
    v.y = perm(o0, e0, 0x07030602u);
    v.z = perm(o1, e1, 0x05010400u);
    v.w = perm(o1, e1, 0x07030602u);
    *(uint4 *)(dst + r * N + (int64_t)y * L + 16 * xc) = v;
}

// Energy changes of a call: replica r adds the partial sums of its
// workgroups' compute waves (slots [r * per_rep, (r + 1) * per_rep)).  One
// workgroup per replica, so the update of dE[r] needs no atomics.
// One workgroup per replica adds its per-wave slots (8192 at 16384^2 with
// 16-row bands).  1024 threads with their loads unrolled keep the few
// memory round trips in flight together: a serial loop of 32 dependent
// round trips per thread took 15 us per call.
__global__ __launch_bounds__(1024) void k_de_collect(const int64_t *part, int64_t *dE, int per_rep) {
    __shared__ long long red[16];
    const int r = (int)blockIdx.x;
    const int64_t *p = part + (int64_t)r * per_rep;
    long long v = 0;
#pragma unroll 8
    for (int i = (int)threadIdx.x; i < per_rep; i += 1024) v += p[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long tot = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) tot += red[w];
        dE[r] += tot;
    }
}

}  // namespace

// Launch shape: chunks of 16 x-positions per lane (one workgroup spans a
// whole row, at most 1024 lanes) and band height H (rows per workgroup).
// Results do not depend on either; SPINMC_L2D_CHUNKS / SPINMC_L2D_H override
// the defaults for tuning.
int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    return v && *v ? atoi(v) : dflt;
}

int lattice2d_chunks(int L) {
    // supported edges: 1024, 2048, 4096, 8192, 16384 (feeds of L/1024 direct loads)
    if (L < 1024 || L > 16384 || (L & (L - 1))) return 0;
    const int want = env_int("SPINMC_L2D_CHUNKS", 0);
    if (want == 2 && L >= 8192) return 2;
    if (want == 1 && L <= 8192) return 1;
    return L <= 4096 ? 1 : 2;  // at most 512 compute lanes per row
}

bool lattice2d_supported(int L) { return lattice2d_chunks(L) > 0; }

// 32 rows per band (16 at L = 16384, where the extra halo reads cost less
// than the shorter bands gain: 325 against 331 us per sweep of three
// lattices); a batch with fewer than two bands per compute unit (a single
// lattice of L <= 4096) takes lower bands, down to 4 rows, so that every
// compute unit has work (the halo rows then cost relatively more).
// SPINMC_L2D_H forces a height; a height smc_autotune measured for the edge
// and replica count comes next.
int lattice2d_band_height(int L, int n_rep) {
    int H = env_int("SPINMC_L2D_H", 0);
    Shape tuned;
    if ((H < 4 || H % 4 || L % H) && tuned_shape(kShapeBand2d, L, 0, n_rep, &tuned)) H = tuned.v[0];
    if (H < 4 || H % 4 || L % H) {
        int cus = 0, dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        H = L >= 16384 ? 16 : 32;
        while (H > 4 && cus > 0 && (int64_t)n_rep * (L / H) < 2 * (int64_t)cus) H >>= 1;
    }
    while (H > 4 && L % H) H >>= 1;
    return (L % H || H % 4) ? 0 : H;
}

// Row pitch of the split planes: L/2 bytes plus padding, so that the rows
// that concurrently running bands touch (H rows apart) do not all fall on
// the same memory channels.  SPINMC_L2D_PAD overrides the padding (bytes, a
// multiple of 16).
int64_t lattice2d_pitch(int L) {
    int pad = env_int("SPINMC_L2D_PAD", 256);
    if (pad < 0 || pad % 16) pad = 256;
    return (int64_t)(L / 2) + pad;
}

size_t lattice2d_split_bytes(int L) { return (size_t)(2 * (int64_t)L * lattice2d_pitch(L)); }

hipError_t launch_to_split(const int8_t *src, uint8_t *dst, int L, int n_rep, hipStream_t s) {
    const int64_t cpr = (int64_t)L * L / 16, total = cpr * n_rep;
    SMC_LAUNCH(k_to_split, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, L,
                       lattice2d_pitch(L), cpr, total);
    return hipGetLastError();
}

hipError_t launch_from_split(const uint8_t *src, int8_t *dst, int L, int n_rep, hipStream_t s) {
    const int64_t cpr = (int64_t)L * L / 16, total = cpr * n_rep;
    SMC_LAUNCH(k_from_split, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, L,
                       lattice2d_pitch(L), cpr, total);
    return hipGetLastError();
}

// Bands of one replica: nb1 of H rows, then bands - nb1 of H2 rows.
struct BandShape {
    int C, H, H2, nb1, bands, ncw;
};

static bool band_shape(int L, int n_rep, BandShape &g) {
    g.C = lattice2d_chunks(L);
    g.H = lattice2d_band_height(L, n_rep);
    if (g.C == 0 || g.H == 0) return false;
    g.H2 = g.H;
    g.bands = L / g.H;
    g.nb1 = g.bands;
    g.ncw = L / (16 * g.C) / 64;
    // With exactly two bands per compute unit (one replica), the workgroups
    // dispatched first (one per CU) win issue arbitration against the second
    // ones and finish far ahead of them; giving the first ones bands of
    // 9/8 H rows and the second ones 7/8 H lets both finish together.
    // SPINMC_L2D_H1 / SPINMC_L2D_H2 set the two heights (multiples of 4).
    {
        int cus = 0;
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        int h1 = 0, h2 = 0;
        if (n_rep == 1 && cus > 0 && L / g.H == 2 * cus && g.H % 32 == 0) {
            h1 = g.H + g.H / 8;
            h2 = g.H - g.H / 8;
        }
        h1 = env_int("SPINMC_L2D_H1", h1);
        h2 = env_int("SPINMC_L2D_H2", h2);
        if (h1 > 0 && h2 > 0 && h1 % 4 == 0 && h2 % 4 == 0 && L % (h1 + h2) == 0) {
            g.H = h1;
            g.H2 = h2;
            g.nb1 = L / (h1 + h2);
            g.bands = 2 * g.nb1;
        }
    }
    return true;
}

size_t lattice2d_de_slots(int L, int n_rep) {
    BandShape g;
    if (!band_shape(L, n_rep, g)) return 0;
    return (size_t)g.bands * (size_t)n_rep * (size_t)g.ncw;
}

hipError_t launch_lattice2d_de_collect(const int64_t *part, int64_t *dE, int L, int n_rep, hipStream_t s) {
    const size_t slots = lattice2d_de_slots(L, n_rep);
    if (slots == 0 || n_rep <= 0) return hipErrorInvalidValue;
    SMC_LAUNCH(k_de_collect, dim3((unsigned)n_rep), dim3(1024), 0, s, part, dE, (int)(slots / n_rep));
    return hipGetLastError();
}

hipError_t launch_ising2d_split(const void *src, bool src_rows, void *dst, bool dst_rows, int L, int n_rep,
                                const ThrRow *thr, int64_t *dE_part, bool dE_first, Key key, uint32_t t,
                                hipStream_t s) {
    BandShape g;
    if (!band_shape(L, n_rep, g)) return hipErrorInvalidValue;
    if (src == dst) return hipErrorInvalidValue;  // bands read only the source: never in place
    const int C = g.C;
    const int IO = (src_rows ? kAbiIn : 0) | (dst_rows ? kAbiOut : 0);
    Lattice2dArgs a;
    a.src = (const uint8_t *)src;
    a.dst = (uint8_t *)dst;
    const int64_t pitch = lattice2d_pitch(L);
    a.src_pitch = src_rows ? (int64_t)L : pitch;
    a.dst_pitch = dst_rows ? (int64_t)L : pitch;
    a.src_rep = src_rows ? (int64_t)L * L : 2 * (int64_t)L * pitch;
    a.dst_rep = dst_rows ? (int64_t)L * L : 2 * (int64_t)L * pitch;
    a.thr = thr;
    a.dE_part = dE_part;
    a.dE_first = dE_first ? 1 : 0;
    a.key = key;
    a.t = t;
    a.L = L;
    a.H = g.H;
    a.H2 = g.H2;
    a.bands = g.bands;
    a.nb1 = g.nb1;
    a.n_rep = n_rep;
    a.one2 = 0x00010001u;
    const unsigned compute_threads = (unsigned)(L / (16 * C));
    const unsigned blocks = (unsigned)(a.bands * n_rep);
    const size_t lds = (size_t)2 * kSlots * (L / 2) + 2 * 16 * 2 * sizeof(uint32_t);
    const int NF = L >= 2048 ? L / 1024 : 2;  // direct-load instructions per feed (two planes of L/2 bytes)
#define SMC_L2D_IO(CC, NFF, IOO)                                                                            \
    if (C == CC && NF == NFF && IO == IOO) {                                                                \
        (void)hipFuncSetAttribute((const void *)k_ising2d_split<CC, NFF, IOO>,                              \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                    \
        const unsigned threads = compute_threads + 64u * LoaderShape<NFF>::NLW;                            \
        SMC_LAUNCH((k_ising2d_split<CC, NFF, IOO>), dim3(blocks), dim3(threads), lds, s, a);                \
        return hipGetLastError();                                                                           \
    }
#define SMC_L2D(CC, NFF)     \
    SMC_L2D_IO(CC, NFF, 0)   \
    SMC_L2D_IO(CC, NFF, 1)   \
    SMC_L2D_IO(CC, NFF, 2)
    SMC_L2D(1, 2)
    SMC_L2D(1, 4)
    SMC_L2D(1, 8)
    SMC_L2D(2, 8)
    SMC_L2D(2, 16)
#undef SMC_L2D
#undef SMC_L2D_IO
    return hipErrorInvalidValue;
}

}  // namespace smc

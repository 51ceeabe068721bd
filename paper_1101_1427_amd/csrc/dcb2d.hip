// Double checkerboard sweeps with multi-hit updates (Sec. 3.2, Sec. 3.4) of
// 2D Ising and +-J EA lattices.  The lattice is cut into T x T tiles whose
// tile colour is (bx + by) & 1.  A sweep is two launches, one per tile
// colour; a workgroup loads its tile and a one-site halo into LDS, gives the
// tile k hits (colour-0 sites, then colour-1 sites, each a Metropolis
// attempt with the halo held fixed) and writes the tile back in place:
// tiles of one colour share no bond, so each launch reads only spins it
// does not write (a lattice of one tile refreshes its wrapped halo after
// every half-hit instead).  With the palindromic order, odd sweeps run both
// orders backwards.
//
// Random numbers: hit j of sweep t uses the plain sweep's draws of "sweep"
// t*k + j: the 16-bit head of in-colour site h is half h & 7 of the block
// (h/8, t*k + j, r, 6 + c); a head equal to the high half of the threshold
// takes the 16-bit tail of (h, t*k + j, r, 8 + c).  A thread handles the
// eight in-colour sites of one such block (16 consecutive columns of a tile
// row), so T is a multiple of 16.
#include "internal.hpp"
#include "intrin.hpp"

namespace smc {
namespace {

constexpr int kDcbMaxThreads = 1024;

struct DcbArgs {
    int8_t *spins;         // caller's spins, replica r at r * N (updated in place)
    const int8_t *coup;    // EA couplings [sample][2][N], replica r using sample r / rep_per_sample, or nullptr
    int rep_per_sample;
    const ThrRow *thr;     // per replica
    int64_t *dE_slots;     // [n_rep][2 * tiles_per_colour] partial sums, or nullptr
    Key key;
    uint32_t t;            // sweep index
    int k;                 // hits per tile
    int L, T, B;           // edge, tile edge, tiles per direction
    int tile_colour;
    int rev;               // 1: colour-1 sites first
    int tiles_per_colour;
};

__global__ __launch_bounds__(kDcbMaxThreads) void k_dcb2d(DcbArgs a) {
    extern __shared__ __align__(16) int8_t smem[];  // spins, bonds to +x, bonds to +y: (T+2)^2 each
    __shared__ long long red[kDcbMaxThreads / 64];
    const int L = a.L, T = a.T, W = T + 2;
    const int r = (int)blockIdx.x / a.tiles_per_colour;
    const int ti = (int)blockIdx.x % a.tiles_per_colour;
    // ti-th tile of the tile colour in row-major tile order
    int bx, by;
    if (a.B == 1) {
        bx = by = 0;
    } else {
        const int half = a.B / 2;  // tiles of one colour per tile row
        by = ti / half;
        bx = 2 * (ti % half) + ((by + a.tile_colour) & 1);
    }
    const int x0 = bx * T, y0 = by * T;
    const int64_t N = (int64_t)L * L;
    int8_t *S = a.spins + (int64_t)r * N;
    const int8_t *Jx = a.coup ? a.coup + (int64_t)(r / a.rep_per_sample) * 2 * N : nullptr;
    const int8_t *Jy = Jx ? Jx + N : nullptr;
    int8_t *ts = smem, *tx = smem + W * W, *ty = smem + 2 * W * W;
    // tile and halo: cell (u, v) of the staged square is site (x0 + u - 1, y0 + v - 1) mod L
    for (int q = threadIdx.x; q < W * W; q += blockDim.x) {
        const int v = q / W, u = q % W;
        const int x = (x0 + u - 1 + L) % L, y = (y0 + v - 1 + L) % L;
        const int64_t i = (int64_t)y * L + x;
        ts[q] = S[i];
        tx[q] = Jx ? Jx[i] : (int8_t)1;
        ty[q] = Jy ? Jy[i] : (int8_t)1;
    }
    const ThrRow th = a.thr[r];
    __syncthreads();

    const int segs = T / 16;
    const int v = (int)threadIdx.x / segs, seg = (int)threadIdx.x % segs;
    const int y = y0 + v;
    long long dE = 0;
    for (int j = 0; j < a.k; ++j) {
        const uint32_t tj = a.t * (uint32_t)a.k + (uint32_t)j;
        for (int ci = 0; ci < 2; ++ci) {
            const int c = a.rev ? 1 - ci : ci;
            // in-colour sites h0 .. h0+7: columns x0 + 16 seg + 2m + ((c + y) & 1)
            const uint32_t h0 = (uint32_t)(y * (L / 2) + x0 / 2 + 8 * seg);
            const uint4 w = philox4x32_10(make_uint4(h0 >> 3, tj, (uint32_t)r, 2 * kTagHead + (uint32_t)c), a.key);
            const int off = (c + y) & 1;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int u = 16 * seg + 2 * m + off;  // tile column
                const int q = (v + 1) * W + (u + 1);
                const int s = ts[q];
                const int hsum = tx[q] * ts[q + 1] + tx[q - 1] * ts[q - 1] + ty[q] * ts[q + W] + ty[q - W] * ts[q - W];
                const int d = 2 * s * hsum;
                bool flip = d <= 0;
                if (!flip) {
                    const uint32_t word = m < 2 ? w.x : m < 4 ? w.y : m < 6 ? w.z : w.w;
                    const uint32_t head = (m & 1) ? (word >> 16) : (word & 0xFFFFu);
                    flip = metropolis_accept(head, d == 8 ? th.m[2] : th.m[1], h0 + (uint32_t)m, tj, (uint32_t)r, (uint32_t)c,
                                             a.key);
                }
                if (flip) {
                    ts[q] = (int8_t)(-s);
                    dE += d;
                }
            }
            __syncthreads();
            if (a.B == 1) {
                // a single tile: its halo wraps onto its own sites, so the
                // halo copies take the values just updated
                for (int e = threadIdx.x; e < 4 * W; e += blockDim.x) {
                    const int side = e / W, p = e % W;
                    const int hv = side == 0 ? 0 : side == 1 ? W - 1 : p;
                    const int hu = side == 2 ? 0 : side == 3 ? W - 1 : p;
                    const int sv = (hv + T - 1) % T + 1, su = (hu + T - 1) % T + 1;
                    ts[hv * W + hu] = ts[sv * W + su];
                }
                __syncthreads();
            }
        }
    }
    // the tile back, in place
    for (int q = threadIdx.x; q < T * T; q += blockDim.x) {
        const int vv = q / T, u = q % T;
        S[(int64_t)(y0 + vv) * L + (x0 + u)] = ts[(vv + 1) * W + (u + 1)];
    }
    if (a.dE_slots) {
        long long tot = dE;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long sum = 0;
            for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) sum += red[w];
            // this workgroup's own slot (tile index and tile colour): no atomics
            int64_t *slot = a.dE_slots + (int64_t)r * 2 * a.tiles_per_colour + a.tile_colour * a.tiles_per_colour + ti;
            *slot += sum;
        }
    }
}

// ------------------------------------------------------------------ packed ----
// The same update with four sites per 32-bit word.  Inside the workgroup a
// tile row is held colour-split: plane c, row v, byte k is the site at
// column 2k + ((v + c) & 1) of the tile (0 = +1, 1 = -1); a colour-c site has
// its two vertical neighbours at the same byte of plane 1-c in rows v-1 and
// v+1 and its two horizontal ones at bytes (k-1, k) of plane 1-c in its own
// row when (v + c) is even, (k, k+1) when odd (y0 is even).  A thread owns a
// 16-column segment of one row, both colours, in registers for all k hits
// (and, for EA, the bond bytes of its sites as 0 = ferro, 1 = antiferro); the
// LDS copy of the planes (with the halo) serves the neighbours.  A
// half-hit per thread: two 8-byte LDS reads (rows above and below), one edge
// word (the neighbouring segment or the halo column), one Philox block, two
// four-site decisions, one 8-byte LDS write, one barrier.  The decision: the
// number n of unsatisfied bonds gives dE = 8 - 4n; the head is compared with
// the high half of thr(n) by packed 16-bit saturating subtraction; heads
// equal to it take the exact path with the 16-bit tail.

template <int T>
struct DcbGeom {
    static constexpr int SEGS = T / 16;                   // 16-column segments per tile row
    static constexpr int TPT = T * T / 16;                // threads per tile
    static constexpr int G = TPT >= 64 ? 1 : 64 / TPT;    // tiles per workgroup
    static constexpr int THREADS = G * TPT;
    static constexpr bool UNIFORM = TPT >= 128;           // every wave holds rows of one parity
    // LDS row: T/2 interior bytes, the left halo word (site in byte 3), the
    // right halo word (site in byte 0); the pitch spreads the 8-byte accesses
    // of a wave over the banks
    static constexpr int PITCH = T == 16 ? 16 : T == 32 ? 24 : T == 64 ? 48 : 96;
    static constexpr int PLANE = (T + 2) * PITCH;         // rows -1 .. T
    static constexpr int TILE = 2 * PLANE;
};

struct DcbLut {
    uint32_t tlo, thi;   // low / high bytes of the head thresholds T(n), n = 0, 1 (0xFF for n >= 2)
    uint32_t one2;
    uint2 thr1, thr2;    // exact thresholds of dE = 4 and dE = 8
};

// Flip flags (bit 0 of each byte) of four sites with unsatisfied counts n and
// heads wa (sites 0, 1), wb (sites 2, 3); eq collects head - T(n).
__device__ __forceinline__ uint32_t dcb_decide4(uint32_t n, uint32_t wa, uint32_t wb, const DcbLut &K,
                                                uint32_t &eq) {
    const uint32_t tl = perm(0xFFFFFFFFu, K.tlo, n);
    const uint32_t th = perm(0xFFFFFFFFu, K.thi, n);
    const uint32_t ta = perm(th, tl, 0x05010400u);
    const uint32_t tb = perm(th, tl, 0x07030602u);
    const uint32_t ra = min16(sub_sat16(ta, wa), K.one2);
    const uint32_t rb = min16(sub_sat16(tb, wb), K.one2);
    eq = min16(eq, min16(sub16(ta, wa), sub16(tb, wb)));
    return perm(rb, ra, 0x06040200u);
}

// Bytes 0, 2 (sel 0x06040200) or 1, 3 (sel 0x07050301) of two words.
__device__ __forceinline__ uint32_t dcb_pick(uint32_t hi, uint32_t lo, int odd) {
    return perm(hi, lo, odd ? 0x07050301u : 0x06040200u);
}
// +1 / -1 bytes to 0 / 1 bytes.
__device__ __forceinline__ uint32_t dcb_bits(uint32_t w) { return (w >> 7) & 0x01010101u; }

struct DcbPackedArgs {
    int8_t *spins;
    const int8_t *coup;
    int rep_per_sample;
    const ThrRow *thr;
    int64_t *dE_slots;
    Key key;
    uint32_t t;
    int k;
    int L, B;
    int tile_colour, rev, tiles_per_colour, total;  // total = n_rep * tiles_per_colour
    uint32_t one2;                                  // 0x00010001, opaque to the compiler
};

// Tile of a tile colour: the ti-th in row-major tile order.
__device__ __forceinline__ void dcb_tile_xy(int ti, int B, int tile_colour, int &bx, int &by) {
    if (B == 1) {
        bx = by = 0;
    } else {
        const int half = B / 2;
        by = ti / half;
        bx = 2 * (ti % half) + ((by + tile_colour) & 1);
    }
}

template <int T, bool EA>
__global__ __launch_bounds__(DcbGeom<T>::THREADS) void k_dcb2d_packed(DcbPackedArgs a) {
    using Gm = DcbGeom<T>;
    constexpr int SEGS = Gm::SEGS, PITCH = Gm::PITCH, PLANE = Gm::PLANE;
    __shared__ __align__(16) uint8_t lds[Gm::G * Gm::TILE];
    __shared__ long long red[(Gm::THREADS + 63) / 64];

    const int lt = (int)threadIdx.x;
    int g, v, seg;
    if constexpr (Gm::UNIFORM) {
        constexpr int RPW = 64 / SEGS;  // rows per wave
        const int w = lt >> 6, lane = lt & 63;
        g = 0;
        v = 2 * ((w >> 1) * RPW + lane / SEGS) + (w & 1);
        seg = lane % SEGS;
    } else {
        g = lt / Gm::TPT;
        const int l = lt % Gm::TPT;
        v = l / SEGS;
        seg = l % SEGS;
    }
    const int tile = (int)blockIdx.x * Gm::G + g;
    const bool active = tile < a.total;
    const int r = active ? tile / a.tiles_per_colour : 0;
    const int ti = active ? tile % a.tiles_per_colour : 0;
    int bx, by;
    dcb_tile_xy(ti, a.B, a.tile_colour, bx, by);
    const int L = a.L, x0 = bx * T, y0 = by * T, y = y0 + v, x = x0 + 16 * seg;
    const int64_t N = (int64_t)L * L;
    int8_t *S = a.spins + (int64_t)r * N;
    uint8_t *tl = lds + g * Gm::TILE;  // plane c at c * PLANE; row v of the tile at LDS row v + 1
    const int pe = v & 1;              // plane of the even columns of this row (x0, y0 even)

    // own spins: plane words sp0 (colour 0), sp1 (colour 1)
    uint32_t sp0[2] = {0u, 0u}, sp1[2] = {0u, 0u};
    if (active) {
        const uint4 q = *(const uint4 *)(S + (int64_t)y * L + x);
        const uint32_t b0 = dcb_bits(q.x), b1 = dcb_bits(q.y), b2 = dcb_bits(q.z), b3 = dcb_bits(q.w);
        const uint32_t e0 = dcb_pick(b1, b0, 0), e1 = dcb_pick(b3, b2, 0);
        const uint32_t o0 = dcb_pick(b1, b0, 1), o1 = dcb_pick(b3, b2, 1);
        sp0[0] = pe ? o0 : e0;
        sp0[1] = pe ? o1 : e1;
        sp1[0] = pe ? e0 : o0;
        sp1[1] = pe ? e1 : o1;
    }
    *(uint2 *)(tl + (v + 1) * PITCH + 8 * seg) = make_uint2(sp0[0], sp0[1]);
    *(uint2 *)(tl + PLANE + (v + 1) * PITCH + 8 * seg) = make_uint2(sp1[0], sp1[1]);
    // halo (fixed while the tile is updated); a single tile wraps onto itself instead
    if (active && a.B > 1) {
        auto halo_row = [&](int yy, int lrow) {
            const uint4 q = *(const uint4 *)(S + (int64_t)yy * L + x);
            const uint32_t b0 = dcb_bits(q.x), b1 = dcb_bits(q.y), b2 = dcb_bits(q.z), b3 = dcb_bits(q.w);
            const int pev = yy & 1;  // even columns of row yy are colour (yy & 1)
            *(uint2 *)(tl + pev * PLANE + lrow * PITCH + 8 * seg) = make_uint2(dcb_pick(b1, b0, 0), dcb_pick(b3, b2, 0));
            *(uint2 *)(tl + (1 - pev) * PLANE + lrow * PITCH + 8 * seg) =
                make_uint2(dcb_pick(b1, b0, 1), dcb_pick(b3, b2, 1));
        };
        if (v == 0) halo_row(y0 == 0 ? L - 1 : y0 - 1, 0);
        if (v == T - 1) halo_row(y0 + T == L ? 0 : y0 + T, T + 1);
        if (seg == 0) {
            const uint32_t b = ((uint32_t)(uint8_t)S[(int64_t)y * L + (x0 == 0 ? L - 1 : x0 - 1)] >> 7) & 1u;
            *(uint32_t *)(tl + (1 - pe) * PLANE + (v + 1) * PITCH + T / 2) = b << 24;
        }
        if (seg == SEGS - 1) {
            const uint32_t b = ((uint32_t)(uint8_t)S[(int64_t)y * L + (x0 + T == L ? 0 : x0 + T)] >> 7) & 1u;
            *(uint32_t *)(tl + pe * PLANE + (v + 1) * PITCH + T / 2 + 4) = b;
        }
    }

    // bonds of the own sites, per colour: jA to the same-byte horizontal
    // neighbour, jB to the shifted one, jU / jD to the rows above / below
    uint32_t jA[2][2] = {}, jB[2][2] = {}, jU[2][2] = {}, jD[2][2] = {};
    if constexpr (EA) {
        if (active) {
            const int8_t *Jx = a.coup + (int64_t)(r / a.rep_per_sample) * 2 * N;
            const int8_t *Jy = Jx + N;
            const int yu = y == 0 ? L - 1 : y - 1;
            const uint4 qx = *(const uint4 *)(Jx + (int64_t)y * L + x);
            const uint32_t prev = dcb_bits(*(const uint32_t *)(Jx + (int64_t)y * L + (x == 0 ? L - 4 : x - 4)));
            const uint4 qd = *(const uint4 *)(Jy + (int64_t)y * L + x);
            const uint4 qu = *(const uint4 *)(Jy + (int64_t)yu * L + x);
            const uint32_t x0b = dcb_bits(qx.x), x1b = dcb_bits(qx.y), x2b = dcb_bits(qx.z), x3b = dcb_bits(qx.w);
            const uint32_t d0 = dcb_bits(qd.x), d1 = dcb_bits(qd.y), d2 = dcb_bits(qd.z), d3 = dcb_bits(qd.w);
            const uint32_t u0 = dcb_bits(qu.x), u1 = dcb_bits(qu.y), u2 = dcb_bits(qu.z), u3 = dcb_bits(qu.w);
            const uint32_t xe[2] = {dcb_pick(x1b, x0b, 0), dcb_pick(x3b, x2b, 0)};
            const uint32_t xo[2] = {dcb_pick(x1b, x0b, 1), dcb_pick(x3b, x2b, 1)};
            // bonds to x - 1 of the even columns: bytes -1, 1, 3, ... of the +x bonds
            const uint32_t xl[2] = {alignbyte(xo[0], prev, 3), alignbyte(xo[1], xo[0], 3)};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int p = (v + c) & 1;  // own sites at odd columns of the segment
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    jA[c][i] = xe[i];  // p = 0: bond to x + 1; p = 1: bond to x - 1
                    jB[c][i] = p ? xo[i] : xl[i];
                    jD[c][i] = p ? dcb_pick(i ? d3 : d1, i ? d2 : d0, 1) : dcb_pick(i ? d3 : d1, i ? d2 : d0, 0);
                    jU[c][i] = p ? dcb_pick(i ? u3 : u1, i ? u2 : u0, 1) : dcb_pick(i ? u3 : u1, i ? u2 : u0, 0);
                }
            }
        }
    }

    const ThrRow th = a.thr[r];
    DcbLut K;
    K.tlo = (th.m[2].x & 0xFFu) | ((th.m[1].x & 0xFFu) << 8) | 0xFFFF0000u;
    K.thi = (th.m[2].x >> 8) | ((th.m[1].x >> 8) << 8) | 0xFFFF0000u;
    K.one2 = a.one2;
    K.thr1 = th.m[1];
    K.thr2 = th.m[2];

    // LDS offsets of the neighbour rows and edge words (a single tile wraps)
    const bool one = a.B == 1;
    const int up_off = (v == 0 ? (one ? T : 0) : v) * PITCH + 8 * seg;
    const int dn_off = (v == T - 1 ? (one ? 1 : T + 1) : v + 2) * PITCH + 8 * seg;
    const int row_off = (v + 1) * PITCH;
    const int le_off = row_off + (seg > 0 ? 8 * seg - 4 : (one ? T / 2 - 4 : T / 2));
    const int re_off = row_off + (seg < SEGS - 1 ? 8 * seg + 8 : (one ? 0 : T / 2 + 4));
    const uint32_t h0 = (uint32_t)(y * (L / 2) + x0 / 2 + 8 * seg);
    __syncthreads();

    uint32_t de_bytes = 0;
    long long de_total = 0;
    // Half-hit of colour C with the horizontal parity P (0, 1, or 2 = per lane).
    auto half = [&](auto cc, auto pp, uint32_t tj) {
        constexpr int C = decltype(cc)::value, P = decltype(pp)::value;
        uint32_t(&own)[2] = C ? sp1 : sp0;
        const uint32_t(&hz)[2] = C ? sp0 : sp1;
        const uint8_t *pl = tl + (1 - C) * PLANE;
        const int p = (v + C) & 1;
        const uint2 U = *(const uint2 *)(pl + up_off);
        const uint2 D = *(const uint2 *)(pl + dn_off);
        const uint32_t E = *(const uint32_t *)(pl + ((P == 2 ? p : P) ? re_off : le_off));
        uint32_t s0, s1;
        if constexpr (P == 0) {
            s0 = alignbyte(hz[0], E, 3);
            s1 = alignbyte(hz[1], hz[0], 3);
        } else if constexpr (P == 1) {
            s0 = alignbyte(hz[1], hz[0], 1);
            s1 = alignbyte(E, hz[1], 1);
        } else {
            s0 = p ? alignbyte(hz[1], hz[0], 1) : alignbyte(hz[0], E, 3);
            s1 = p ? alignbyte(E, hz[1], 1) : alignbyte(hz[1], hz[0], 3);
        }
        const uint32_t uu[2] = {U.x, U.y}, dd[2] = {D.x, D.y}, ss[2] = {s0, s1};
        uint32_t n[2], F[2];
        const uint4 w = philox4x32_10(make_uint4(h0 >> 3, tj, (uint32_t)r, 2 * kTagHead + (uint32_t)C), a.key);
        uint32_t eq = 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const uint32_t o = own[i];
            if constexpr (EA) {
                n[i] = ((o ^ uu[i] ^ jU[C][i]) + (o ^ dd[i] ^ jD[C][i])) +
                       ((o ^ hz[i] ^ jA[C][i]) + (o ^ ss[i] ^ jB[C][i]));
            } else {
                n[i] = ((o ^ uu[i]) + (o ^ dd[i])) + ((o ^ hz[i]) + (o ^ ss[i]));
            }
            F[i] = dcb_decide4(n[i], i ? w.z : w.x, i ? w.w : w.y, K, eq);
        }
        const bool tie = ((eq & 0xFFFFu) == 0u) || ((eq >> 16) == 0u);
        if (__builtin_expect(__any(tie), 0)) {
            // Exact decisions of the sites whose head equals the high half of
            // the threshold (probability 2^-16 each).  A wavefront that meets
            // one holds up the workgroup at the next barrier, so the path is
            // short: a mask of the tied sites, then one pass per tied site of
            // the lane with most of them (almost always one), each drawing the
            // single tail it needs.
            uint32_t tm = 0;  // bit 4 i + s4: site s4 of word i is tied
            if (tie) {
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const uint32_t tl = perm(0xFFFFFFFFu, K.tlo, n[i]), th = perm(0xFFFFFFFFu, K.thi, n[i]);
                    const uint32_t da = perm(th, tl, 0x05010400u) ^ (i ? w.z : w.x);
                    const uint32_t db = perm(th, tl, 0x07030602u) ^ (i ? w.w : w.y);
                    const uint32_t m4 = ((da & 0xFFFFu) == 0u ? 1u : 0u) | ((da >> 16) == 0u ? 2u : 0u) |
                                        ((db & 0xFFFFu) == 0u ? 4u : 0u) | ((db >> 16) == 0u ? 8u : 0u);
                    tm |= m4 << (4 * i);
                }
            }
            const uint32_t n0 = n[0], n1 = n[1], t2y = K.thr2.y, t1y = K.thr1.y;
            while (__any(tm != 0u)) {
                if (tm != 0u) {
                    const uint32_t s = __builtin_ctz(tm), b = 8u * (s & 3u);
                    tm &= tm - 1u;
                    const uint32_t ns = ((s < 4u ? n0 : n1) >> b) & 0xFFu;
                    uint32_t flip = 1u;  // a head of 0xFFFF at a site with Delta E <= 0
                    if (ns < 2u) {
                        // the head equals the threshold's high half: compare the tail
                        flip = tail16(h0 + s, tj, (uint32_t)r, (uint32_t)C, a.key) < (ns == 0u ? t2y : t1y) ? 1u : 0u;
                    }
                    const uint32_t keep = ~(0xFFu << b), set = flip << b;
                    if (s < 4u)
                        F[0] = (F[0] & keep) | set;
                    else
                        F[1] = (F[1] & keep) | set;
                }
            }
        }
        uint32_t de = 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            own[i] ^= F[i];
            // per site dE/4 + 2: 2 when kept, 4 - n when flipped (n >= 2 always flips)
            de += perm(0x01020304u, 0x02020202u, (F[i] << 2) + n[i]);
        }
        de_bytes = __builtin_amdgcn_sad_u8(de, 0u, de_bytes);
        *(uint2 *)(tl + C * PLANE + row_off + 8 * seg) = make_uint2(own[0], own[1]);
        __syncthreads();
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    auto half_c = [&](auto cc, uint32_t tj) {
        constexpr int C = decltype(cc)::value;
        if constexpr (Gm::UNIFORM) {
            if (__builtin_amdgcn_readfirstlane((v + C) & 1))
                half(cc, I1{}, tj);
            else
                half(cc, I0{}, tj);
        } else {
            half(cc, I2{}, tj);
        }
    };
    for (int j = 0; j < a.k; ++j) {
        const uint32_t tj = a.t * (uint32_t)a.k + (uint32_t)j;
        de_bytes = 0;
        if (a.rev) {
            half_c(I1{}, tj);
            half_c(I0{}, tj);
        } else {
            half_c(I0{}, tj);
            half_c(I1{}, tj);
        }
        de_total += (long long)de_bytes - 32;  // 16 sites at 2 each
    }

    // the segment back in lattice order, +1 / -1 bytes, in place
    if (active) {
        const uint32_t e0 = pe ? sp1[0] : sp0[0], e1 = pe ? sp1[1] : sp0[1];
        const uint32_t o0 = pe ? sp0[0] : sp1[0], o1 = pe ? sp0[1] : sp1[1];
        uint4 q;
        q.x = perm(0u, 0x0000FF01u, perm(o0, e0, 0x05010400u));
        q.y = perm(0u, 0x0000FF01u, perm(o0, e0, 0x07030602u));
        q.z = perm(0u, 0x0000FF01u, perm(o1, e1, 0x05010400u));
        q.w = perm(0u, 0x0000FF01u, perm(o1, e1, 0x07030602u));
        *(uint4 *)(S + (int64_t)y * L + x) = q;
    }
    if (a.dE_slots) {
        long long tot = active ? 4 * de_total : 0;
        if constexpr (Gm::TPT < 64) {
            // a tile is TPT consecutive lanes of the one wave
#pragma unroll
            for (int o = Gm::TPT / 2; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
            if (active && (lt % Gm::TPT) == 0)
                a.dE_slots[(int64_t)r * 2 * a.tiles_per_colour + a.tile_colour * a.tiles_per_colour + ti] += tot;
        } else {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
            if ((lt & 63) == 0) red[lt >> 6] = tot;
            __syncthreads();
            if (lt == 0 && active) {
                long long sum = 0;
                for (int w = 0; w < Gm::THREADS / 64; ++w) sum += red[w];
                a.dE_slots[(int64_t)r * 2 * a.tiles_per_colour + a.tile_colour * a.tiles_per_colour + ti] += sum;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_dcb_zero(int64_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// dE[r] = (assign) or += the sum of replica r's slots.
__global__ __launch_bounds__(256) void k_dcb_collect(const int64_t *slots, int64_t *dE, int per_rep, int assign) {
    __shared__ long long red[4];
    const int r = (int)blockIdx.x;
    long long v = 0;
    for (int i = (int)threadIdx.x; i < per_rep; i += 256) v += slots[(int64_t)r * per_rep + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long sum = red[0] + red[1] + red[2] + red[3];
        dE[r] = assign ? sum : dE[r] + sum;
    }
}

}  // namespace

bool dcb2d_supported(int L, int T) {
    if (T < 16 || T > 128 || T % 16 || L % T) return false;
    const int B = L / T;
    return B == 1 || B % 2 == 0;
}

int dcb2d_tiles_per_colour(int L, int T) {
    const int B = L / T;
    return B == 1 ? 1 : B * B / 2;
}

hipError_t launch_dcb_zero(int64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    SMC_LAUNCH(k_dcb_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_dcb_collect(const int64_t *slots, int64_t *dE, int n_rep, int per_rep, bool assign, hipStream_t s) {
    SMC_LAUNCH(k_dcb_collect, dim3((unsigned)n_rep), dim3(256), 0, s, slots, dE, per_rep, assign ? 1 : 0);
    return hipGetLastError();
}

template <int T>
hipError_t launch_packed(const DcbPackedArgs &a, bool ea, hipStream_t s) {
    using Gm = DcbGeom<T>;
    const unsigned blocks = (unsigned)((a.total + Gm::G - 1) / Gm::G);
    if (ea)
        SMC_LAUNCH((k_dcb2d_packed<T, true>), dim3(blocks), dim3(Gm::THREADS), 0, s, a);
    else
        SMC_LAUNCH((k_dcb2d_packed<T, false>), dim3(blocks), dim3(Gm::THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dcb2d(int8_t *spins, const int8_t *coup, int rep_per_sample, const ThrRow *thr, int64_t *dE_slots,
                        int n_rep, int L, int T, int k, Key key, uint32_t t, int tile_colour, bool rev, bool packed,
                        hipStream_t s) {
    if (!dcb2d_supported(L, T) || k < 1 || rep_per_sample < 1) return hipErrorInvalidValue;
    const int B = L / T;
    if (B == 1 && tile_colour == 1) return hipSuccess;  // one tile, of tile colour 0
    const int tpc = dcb2d_tiles_per_colour(L, T);
    if (packed) {
        DcbPackedArgs a;
        a.spins = spins;
        a.coup = coup;
        a.rep_per_sample = rep_per_sample;
        a.thr = thr;
        a.dE_slots = dE_slots;
        a.key = key;
        a.t = t;
        a.k = k;
        a.L = L;
        a.B = B;
        a.tile_colour = tile_colour;
        a.rev = rev ? 1 : 0;
        a.tiles_per_colour = tpc;
        a.total = n_rep * tpc;
        a.one2 = 0x00010001u;
        switch (T) {
            case 16: return launch_packed<16>(a, coup != nullptr, s);
            case 32: return launch_packed<32>(a, coup != nullptr, s);
            case 64: return launch_packed<64>(a, coup != nullptr, s);
            case 128: return launch_packed<128>(a, coup != nullptr, s);
            default: return hipErrorInvalidValue;
        }
    }
    DcbArgs a;
    a.spins = spins;
    a.coup = coup;
    a.rep_per_sample = rep_per_sample;
    a.thr = thr;
    a.dE_slots = dE_slots;
    a.key = key;
    a.t = t;
    a.k = k;
    a.L = L;
    a.T = T;
    a.B = B;
    a.tile_colour = tile_colour;
    a.rev = rev ? 1 : 0;
    a.tiles_per_colour = tpc;
    const unsigned threads = (unsigned)(T * T / 16);
    const size_t lds = (size_t)3 * (T + 2) * (T + 2);
    const unsigned blocks = (unsigned)(n_rep * tpc);
    SMC_LAUNCH(k_dcb2d, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

bool dcb2d_packed_supported(int L, int T) { return dcb2d_supported(L, T) && (T == 16 || T == 32 || T == 64 || T == 128); }

}  // namespace smc

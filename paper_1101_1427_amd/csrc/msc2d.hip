// Asynchronous multi-spin coding of the 2D +-J spin glass (Sec. 5): bit k of
// a 32-bit word holds replica 32g + k of word g, so one word operation
// updates the same site of 32 independent lattices, each with its own
// couplings.  The w = 32 or 64 replicas of a draw group share the
// Metropolis uniform of each site and sweep (the paper draws one random
// number per w-bit word); their counters carry the group index r / w where
// the single-replica sweep carries the replica index.  With w = 64 a thread
// updates the two words of a group with one draw.
//
// Decision for one site of the 32 replicas: with a_j = s ^ s_j ^ J_j the
// unsatisfied-bond bits of the four bonds, n = a_1 + .. + a_4 per replica
// and dE = 8 - 4n.  n >= 2 always flips; n = 1 flips iff u < thr(dE = 4);
// n = 0 iff u < thr(dE = 8).  Since thr(8) < thr(4), with the per-site
// booleans D1 = [u < thr(4)] and D2 = [u < thr(8)] the flip mask is
//   D2 ? all : D1 ? (n >= 1) : (n >= 2),
// computed with a bit-sliced adder on the four words.  u is compared in
// two 16-bit halves as in the other kernels: the head (one Philox block
// serves 8 sites) decides unless it equals the high half of a threshold.
//
// Gauge: a transformation s_i -> e_i s_i, J_ij -> e_i J_ij e_j (e_i = +-1
// per site and replica) leaves every unsatisfied-bond count, and so every
// decision, unchanged.  Before the sweeps each row is transformed so that
// its horizontal bonds are all +1 except the one that closes the periodic
// row (e runs as the prefix product of the row's bonds); afterwards the
// spins are transformed back.  The kernel then needs one horizontal bond
// word per row instead of one per site.
//
// Layout: a workgroup holds whole groups; each group's lattice of words
// lives in LDS (padded so that the lanes of a wave read 64 different banks)
// and in registers: a thread owns 16 consecutive sites of one row (8 of
// each colour, one Philox block per colour) with their spins and down
// bonds.  A half-sweep reads the neighbours' words and the up bonds from
// LDS, updates the owned words of one colour in registers and writes them
// back; one barrier per half-sweep.  All sweeps of a call run in
// one launch, so HBM is touched only at its start and end.
#include "internal.hpp"

namespace smc {
namespace {

constexpr int kMscBlock = 256;

// LDS geometry: word (group gw, row y, segment s, column xx) at
// gw*GS + y*RS + s*SS + xx.  The lanes of a wave share xx and differ in
// (group, row pair, segment); with these strides the 32 lanes of each half
// wave, which the LDS serves together, hit 32 different banks for every
// access of a half-sweep (rows y-1, y, y+1 and the neighbouring segments).
template <int SEG>
struct MscGeom;
template <>
struct MscGeom<1> {
    static constexpr int RS = 18, SS = 16, GS = 289;
};
template <>
struct MscGeom<2> {
    static constexpr int RS = 35, SS = 17, GS = 1120;
};
template <>
struct MscGeom<4> {
    static constexpr int RS = 70, SS = 17, GS = 4480;
};

struct Msc2dArgs {
    uint32_t *spins;       // packed, gauge-fixed [G][L*L] (bit k: replica 32g + k is -1)
    const uint32_t *coup;  // packed, gauge-fixed [G][2][L*L] (bit k: J = -1 for replica 32g + k);
                           // horizontal bonds are +1 except at x = L-1
    const ThrRow *thr;     // per group
    Key key;
    uint32_t t0;
    int n_sweeps;
    int G;
};

// Colour c of the thread's 16 sites, those at columns OFF, OFF+2, .., 14+OFF
// of its segment (OFF = (c + y) & 1 is uniform across a wave).
// Flip mask of the site in column xx (the 32 replicas of the word) for the
// decisions d1 = [u < thr(dE = 4)] and d2 = [u < thr(dE = 8)]: with a_j the
// unsatisfied-bond words of its four bonds, n >= 2 flips always, n = 1 iff
// d1, n = 0 iff d2 (d2 implies d1).
template <int OFF>
__device__ __forceinline__ uint32_t msc_flip_mask(const uint32_t (&S)[16], const uint32_t (&JD)[16], uint32_t JL,
                                                  uint32_t JR15, uint32_t bnd, const uint32_t *up, const uint32_t *dn,
                                                  const uint32_t *ju, int xx, bool d1, bool d2) {
    const uint32_t s = S[xx];
    const uint32_t left = xx == 0 ? bnd : S[xx == 0 ? 0 : xx - 1];
    const uint32_t right = xx == 15 ? bnd : S[xx == 15 ? 15 : xx + 1];
    const uint32_t a1 = xx == 0 ? s ^ left ^ JL : s ^ left;
    const uint32_t a2 = xx == 15 ? s ^ right ^ JR15 : s ^ right;
    const uint32_t a3 = s ^ up[xx] ^ ju[xx];
    const uint32_t a4 = s ^ dn[xx] ^ JD[xx];
    const uint32_t p = a1 ^ a2, q = a1 & a2, r = a3 ^ a4, u = a3 & a4;
    const uint32_t ge2 = q | u | (p & r);
    const uint32_t ge1 = a1 | a2 | a3 | a4;
    return d2 ? 0xFFFFFFFFu : (d1 ? ge1 : ge2);
}

// JL / JR15: the horizontal bonds into column 0 and out of column 15 of the
// segment (the row's closing bond at the lattice edge, +1 elsewhere after the
// gauge); JD: the bonds down from the owned sites; the bonds up from them are
// the row above's down bonds, read from the bond plane jd in LDS.  A thread
// updates NW words (1, or 2 for 64 replicas per draw) of the same sites with
// one Philox block per colour; g is the draw's group index.
template <int SEG, int OFF, int NW>
__device__ __forceinline__ void msc_half(uint32_t (&S)[NW][16], const uint32_t (&JD)[NW][16], const uint32_t (&JL)[NW],
                                         const uint32_t (&JR15)[NW], uint32_t *const (&lat)[NW],
                                         const uint32_t *const (&jd)[NW], int y, int seg, uint32_t g, uint32_t t,
                                         uint32_t c, const ThrRow &thr, Key key) {
    using GE = MscGeom<SEG>;
    constexpr int L = 16 * SEG;
    const int ru = ((y + L - 1) % L) * GE::RS + seg * GE::SS;
    const int rd = ((y + 1) % L) * GE::RS + seg * GE::SS;
    // the neighbour word outside the segment: column 15 of the segment to
    // the left (OFF = 0) or column 0 of the one to the right (OFF = 1)
    const int rb = OFF == 0 ? y * GE::RS + ((seg + SEG - 1) % SEG) * GE::SS + 15 : y * GE::RS + ((seg + 1) % SEG) * GE::SS;
    uint32_t bnd[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) bnd[w] = lat[w][rb];
    const uint32_t b = (uint32_t)(y * SEG + seg);  // Philox block: in-colour sites 8b .. 8b+7
    const uint4 wd = philox4x32_10(make_uint4(b, t, g, 2 * kTagHead + c), key);
    const uint32_t T1 = thr.m[1].x, T2 = thr.m[2].x;
    // Flip masks from the heads alone; a head equal to the high half of a
    // threshold (rare) marks its site for the exact path below, which then
    // replaces that site's masks.  Nothing is applied before both are done.
    uint32_t flip[NW][8];
    bool tie[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int xx = OFF + 2 * j;
        const uint32_t word = j < 2 ? wd.x : j < 4 ? wd.y : j < 6 ? wd.z : wd.w;
        const uint32_t head = (j & 1) ? (word >> 16) : (word & 0xFFFFu);
#pragma unroll
        for (int w = 0; w < NW; ++w)
            flip[w][j] = msc_flip_mask<OFF>(S[w], JD[w], JL[w], JR15[w], bnd[w], lat[w] + ru, lat[w] + rd, jd[w] + ru,
                                            xx, head < T1, head < T2);
        tie[j] = head == T1 || head == T2;
    }
    bool any = false;
#pragma unroll
    for (int j = 0; j < 8; ++j) any = any || tie[j];
    if (__builtin_expect(any, 0)) {
        // one tied site of this lane per pass (one tail draw at a time)
        uint32_t pending = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) pending |= tie[j] ? (1u << j) : 0u;
        while (pending) {
            const uint32_t jl = (uint32_t)__builtin_ctz(pending);
            pending &= pending - 1u;
            const uint32_t word = jl < 2u ? wd.x : jl < 4u ? wd.y : jl < 6u ? wd.z : wd.w;
            const uint32_t head = (jl & 1u) ? (word >> 16) : (word & 0xFFFFu);
            const uint32_t tail = tail16(8u * b + jl, t, g, c, key);
            const bool d1 = head < T1 || (head == T1 && tail < thr.m[1].y);
            const bool d2 = head < T2 || (head == T2 && tail < thr.m[2].y);
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (jl == (uint32_t)j) {
#pragma unroll
                    for (int w = 0; w < NW; ++w)
                        flip[w][j] = msc_flip_mask<OFF>(S[w], JD[w], JL[w], JR15[w], bnd[w], lat[w] + ru,
                                                        lat[w] + rd, jd[w] + ru, OFF + 2 * j, d1, d2);
                }
        }
    }
#pragma unroll
    for (int w = 0; w < NW; ++w) {
#pragma unroll
        for (int j = 0; j < 8; ++j) S[w][OFF + 2 * j] ^= flip[w][j];
        uint32_t *own = lat[w] + y * GE::RS + seg * GE::SS;
#pragma unroll
        for (int j = 0; j < 8; ++j) own[OFF + 2 * j] = S[w][OFF + 2 * j];
    }
}

// NW words per thread: 1 (32 replicas per draw) or 2 (64 replicas per draw,
// words 2h and 2h + 1 drawing as group h).
template <int SEG, int NW>
__global__ __launch_bounds__(kMscBlock) void k_msc2d(Msc2dArgs a) {
    using GE = MscGeom<SEG>;
    constexpr int L = 16 * SEG, N = L * L;
    constexpr int TPG = N / 16;           // threads per set of NW words
    constexpr int SPW = kMscBlock / TPG;  // thread sets per workgroup
    constexpr int WPW = SPW * NW;         // words per workgroup
    constexpr int PER = TPG / 2;          // threads per set and row parity
    __shared__ uint32_t lds[WPW * GE::GS];
    __shared__ uint32_t lds_jd[WPW * GE::GS];  // down bonds, same geometry
    // threads [0, 128) own even rows, [128, 256) odd rows, so that the
    // colour offset of a half-sweep is uniform across each wave
    const int par = (int)threadIdx.x / (kMscBlock / 2);
    const int q = (int)threadIdx.x % (kMscBlock / 2);
    const int set = q / PER, rem = q % PER;
    const int y = 2 * (rem / SEG) + par, seg = rem % SEG;
    const int g0 = (int)blockIdx.x * WPW + set * NW;  // first word (group of 32 replicas)
    const bool live = g0 < a.G;                        // (the G words come in whole sets)
    uint32_t *lat[NW];
    const uint32_t *jd[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        lat[w] = lds + (set * NW + w) * GE::GS;
        jd[w] = lds_jd + (set * NW + w) * GE::GS;
    }

    uint32_t S[NW][16], JD[NW][16], JL[NW], JR15[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (live) {
            const int g = g0 + w;
            const uint32_t *sp = a.spins + (size_t)g * N + (size_t)(y * L + 16 * seg);
            const uint32_t *cp = a.coup + 2 * (size_t)g * N;
#pragma unroll
            for (int xx = 0; xx < 16; ++xx) {
                S[w][xx] = sp[xx];
                JD[w][xx] = cp[N + y * L + 16 * seg + xx];
            }
            const uint32_t wrap = cp[y * L + L - 1];  // the row's closing bond (L-1 -> 0)
            JL[w] = seg == 0 ? wrap : 0u;
            JR15[w] = seg == SEG - 1 ? wrap : 0u;
        } else {
#pragma unroll
            for (int xx = 0; xx < 16; ++xx) S[w][xx] = JD[w][xx] = 0u;
            JL[w] = JR15[w] = 0u;
        }
        uint32_t *own = lat[w] + y * GE::RS + seg * GE::SS;
        uint32_t *ownj = (uint32_t *)jd[w] + y * GE::RS + seg * GE::SS;
#pragma unroll
        for (int xx = 0; xx < 16; ++xx) {
            own[xx] = S[w][xx];
            ownj[xx] = JD[w][xx];
        }
    }
    // the draws' group index: the word for 32 replicas per draw, the word pair for 64
    const uint32_t gdraw = (uint32_t)(NW == 2 ? g0 >> 1 : g0);
    const ThrRow thr = a.thr[live ? g0 : 0];
    __syncthreads();
    for (int k = 0; k < a.n_sweeps; ++k) {
        const uint32_t t = a.t0 + (uint32_t)k;
#pragma unroll
        for (uint32_t c = 0; c < 2; ++c) {
            if (((c + (uint32_t)par) & 1u) == 0u)
                msc_half<SEG, 0, NW>(S, JD, JL, JR15, lat, jd, y, seg, gdraw, t, c, thr, a.key);
            else
                msc_half<SEG, 1, NW>(S, JD, JL, JR15, lat, jd, y, seg, gdraw, t, c, thr, a.key);
            __syncthreads();
        }
    }
    if (live) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const size_t base = (size_t)(g0 + w) * N + (size_t)(y * L + 16 * seg);
#pragma unroll
            for (int xx = 0; xx < 16; ++xx) a.spins[base + xx] = S[w][xx];
        }
    }
}

// int8 +-1 values of replicas 32g .. 32g+31 (M values per replica, e.g. the
// spins or the d*N couplings) -> words (g, i); bit k set where replica
// 32g + k holds -1.  Four consecutive values per thread (M % 4 == 0);
// without a source (Ising couplings) every word is 0.
__global__ __launch_bounds__(256) void k_msc_pack(const int8_t *src, uint32_t *dst, int64_t M, int64_t quads) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= quads) return;
    const int64_t g = gid / (M / 4), i = 4 * (gid % (M / 4));
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    if (src) {
        const int8_t *p = src + 32 * g * M + i;
#pragma unroll 8
        for (int k = 0; k < 32; ++k) {
            const uint32_t v = *(const uint32_t *)(p + (int64_t)k * M);  // four values; the sign bit of each byte
            w0 |= ((v >> 7) & 1u) << k;
            w1 |= ((v >> 15) & 1u) << k;
            w2 |= ((v >> 23) & 1u) << k;
            w3 |= (v >> 31) << k;
        }
    }
    *(uint4 *)(dst + g * M + i) = make_uint4(w0, w1, w2, w3);
}

// Gauge fixing of 2D packed words, one thread per row (g, y): e(0) = 0,
// e(x+1) = e(x) ^ JR(x); spins ^= e; the row's horizontal bonds become 0
// (+1) except JR(L-1), which becomes the XOR of all of them (the row loop's
// sign).  e is kept for the way back.
__global__ __launch_bounds__(256) void k_msc_gauge_rows(uint32_t *spins, uint32_t *coup, uint32_t *gauge, int L,
                                                        int64_t rows) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= rows) return;
    const int64_t N = (int64_t)L * L, g = gid / L, y = gid % L;
    uint32_t *jr = coup + 2 * g * N + y * L;
    uint32_t *sp = spins + g * N + y * L;
    uint32_t *ep = gauge + g * N + y * L;
    uint32_t e = 0;
    for (int x = 0; x < L; ++x) {
        ep[x] = e;
        sp[x] ^= e;
        e ^= jr[x];
        jr[x] = x == L - 1 ? e : 0u;
    }
}

// Vertical bonds under the gauge: JD(x, y) ^= e(x, y) ^ e(x, y+1).
__global__ __launch_bounds__(256) void k_msc_gauge_vertical(uint32_t *coup, const uint32_t *gauge, int L,
                                                            int64_t words) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= words) return;
    const int64_t N = (int64_t)L * L, g = gid / N, i = gid % N;
    const int64_t y = i / L, x = i % L;
    const int64_t below = ((y + 1) % L) * L + x;
    coup[2 * g * N + N + i] ^= gauge[g * N + i] ^ gauge[g * N + below];
}

// Packed words (with gauge e, or none) -> int8 +-1 values of replicas 32g ..
// 32g+31, four sites per thread.
__global__ __launch_bounds__(256) void k_msc_unpack(const uint32_t *src, const uint32_t *gauge, int8_t *dst,
                                                    int64_t N, int64_t quads) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= quads) return;
    const int64_t g = gid / (N / 4), i = 4 * (gid % (N / 4));
    uint4 w = *(const uint4 *)(src + g * N + i);
    if (gauge) {
        const uint4 e = *(const uint4 *)(gauge + g * N + i);
        w.x ^= e.x;
        w.y ^= e.y;
        w.z ^= e.z;
        w.w ^= e.w;
    }
    int8_t *p = dst + 32 * g * N + i;
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
        // byte b = 0xFF (-1) where bit k of word b is set, else 0x01 (+1)
        const uint32_t bits = ((w.x >> k) & 1u) | (((w.y >> k) & 1u) << 8) | (((w.z >> k) & 1u) << 16) |
                              (((w.w >> k) & 1u) << 24);
        *(uint32_t *)(p + (int64_t)k * N) = (bits * 0xFEu) + 0x01010101u;
    }
}

// dE[r] += E1[r] - E0[r] (energies are exact integers in float64).
__global__ __launch_bounds__(256) void k_msc_energy_diff(const double *E0, const double *E1, int64_t *dE, int n) {
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r < n) dE[r] += (int64_t)E1[r] - (int64_t)E0[r];
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

bool msc2d_supported(int dim, int L) { return dim == 2 && (L == 16 || L == 32 || L == 64); }

hipError_t launch_msc_pack(const int8_t *spins, uint32_t *packed, int64_t N, int n_groups, hipStream_t s) {
    const int64_t quads = (int64_t)n_groups * N / 4;
    if (quads == 0 || N % 4) return quads == 0 ? hipSuccess : hipErrorInvalidValue;
    SMC_LAUNCH(k_msc_pack, dim3(blocks_for(quads)), dim3(256), 0, s, spins, packed, N, quads);
    return hipGetLastError();
}

hipError_t launch_msc_pack_coup(const int8_t *coup, uint32_t *packed, int64_t dN, int n_groups, hipStream_t s) {
    const int64_t quads = (int64_t)n_groups * dN / 4;
    if (quads == 0 || dN % 4) return quads == 0 ? hipSuccess : hipErrorInvalidValue;
    SMC_LAUNCH(k_msc_pack, dim3(blocks_for(quads)), dim3(256), 0, s, coup, packed, dN, quads);
    return hipGetLastError();
}

hipError_t launch_msc_unpack(const uint32_t *packed, const uint32_t *gauge, int8_t *spins, int64_t N, int n_groups,
                             hipStream_t s) {
    const int64_t quads = (int64_t)n_groups * N / 4;
    if (quads == 0 || N % 4) return quads == 0 ? hipSuccess : hipErrorInvalidValue;
    SMC_LAUNCH(k_msc_unpack, dim3(blocks_for(quads)), dim3(256), 0, s, packed, gauge, spins, N, quads);
    return hipGetLastError();
}

hipError_t launch_msc_gauge2d(uint32_t *spins, uint32_t *coup, uint32_t *gauge, int L, int n_groups, hipStream_t s) {
    const int64_t rows = (int64_t)n_groups * L, words = rows * L;
    if (rows == 0) return hipSuccess;
    SMC_LAUNCH(k_msc_gauge_rows, dim3(blocks_for(rows)), dim3(256), 0, s, spins, coup, gauge, L, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SMC_LAUNCH(k_msc_gauge_vertical, dim3(blocks_for(words)), dim3(256), 0, s, coup, gauge, L, words);
    return hipGetLastError();
}

hipError_t launch_msc_energy_diff(const double *E0, const double *E1, int64_t *dE, int n, hipStream_t s) {
    SMC_LAUNCH(k_msc_energy_diff, dim3(blocks_for(n)), dim3(256), 0, s, E0, E1, dE, n);
    return hipGetLastError();
}

template <int SEG>
hipError_t launch_msc2d_seg(const Msc2dArgs &a, int words_per_draw, hipStream_t s) {
    constexpr int tpg = 16 * SEG * 16 * SEG / 16;
    const int wpw = kMscBlock / tpg * words_per_draw;
    const unsigned blocks = (unsigned)((a.G + wpw - 1) / wpw);
    if (words_per_draw == 2)
        SMC_LAUNCH((k_msc2d<SEG, 2>), dim3(blocks), dim3(kMscBlock), 0, s, a);
    else
        SMC_LAUNCH((k_msc2d<SEG, 1>), dim3(blocks), dim3(kMscBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_msc2d(uint32_t *spins, const uint32_t *coup, const ThrRow *thr, int n_groups, int L, Key key,
                        uint32_t t0, int n_sweeps, int words_per_draw, hipStream_t s) {
    Msc2dArgs a;
    a.spins = spins;
    a.coup = coup;
    a.thr = thr;
    a.key = key;
    a.t0 = t0;
    a.n_sweeps = n_sweeps;
    a.G = n_groups;
    if (n_groups <= 0 || n_sweeps <= 0) return hipSuccess;
    if (words_per_draw != 1 && words_per_draw != 2) return hipErrorInvalidValue;
    if (n_groups % words_per_draw) return hipErrorInvalidValue;  // whole word pairs
    switch (L) {
        case 16: return launch_msc2d_seg<1>(a, words_per_draw, s);
        case 32: return launch_msc2d_seg<2>(a, words_per_draw, s);
        case 64: return launch_msc2d_seg<4>(a, words_per_draw, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace smc

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
// spin read once and written once (plus 4 halo rows per band from L2).
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

namespace smc {
namespace {

__device__ __forceinline__ uint32_t pk_sub_sat_u16(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_pk_sub_u16 %0, %1, %2 clamp" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ uint32_t pk_sub_u16(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_pk_sub_u16 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ uint32_t pk_min_u16(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}
__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t s) {
    return __builtin_amdgcn_alignbyte(hi, lo, s);
}

// Per-replica constants of the decision.
struct Lut {
    uint32_t tlo_lo, tlo_hi, thi_lo, thi_hi;  // T(n): low / high bytes, selectors n = 0..7
    uint32_t de_lo, de_hi;                    // dE/4 + 2 for index n + 4F
    uint32_t one2;                            // 0x00010001
    uint2 thr1, thr2;                         // exact thresholds of dE = 4 and dE = 8
};

__device__ __forceinline__ Lut make_lut(const ThrRow &row) {
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
    k.one2 = 0x00010001u;
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

template <int C>
__device__ __forceinline__ void store_row(uint8_t *p, const Row<C> &r) {
    if constexpr (C == 1) {
        *(uint2 *)p = make_uint2(r.d[0], r.d[1]);
    } else {
#pragma unroll
        for (int i = 0; i < C / 2; ++i)
            ((uint4 *)p)[i] = make_uint4(r.d[4 * i], r.d[4 * i + 1], r.d[4 * i + 2], r.d[4 * i + 3]);
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
    return ((own ^ va) + (own ^ vb)) + ((own ^ hz.d[i]) + (own ^ sh));
}

// Flip flags (bit 0 of each byte) of the four sites with counts n and heads
// in words wa (sites 0, 1) and wb (sites 2, 3); eq collects head - T.
__device__ __forceinline__ uint32_t decide4(uint32_t n, uint32_t wa, uint32_t wb, const Lut &K, uint32_t &eq) {
    const uint32_t tl = perm(K.tlo_hi, K.tlo_lo, n);
    const uint32_t th = perm(K.thi_hi, K.thi_lo, n);
    const uint32_t ta = perm(th, tl, 0x05010400u);
    const uint32_t tb = perm(th, tl, 0x07030602u);
    const uint32_t ra = pk_min_u16(pk_sub_sat_u16(ta, wa), K.one2);
    const uint32_t rb = pk_min_u16(pk_sub_sat_u16(tb, wb), K.one2);
    eq = pk_min_u16(eq, pk_min_u16(pk_sub_u16(ta, wa), pk_sub_u16(tb, wb)));
    return perm(rb, ra, 0x06040200u);
}

// Exact decision of site s (0..7) of a chunk: n its count, w the chunk's draw.
__device__ __noinline__ uint32_t exact_flip(uint32_t n, uint32_t head, const Lut &K, uint32_t h, uint32_t t,
                                            uint32_t r, uint32_t c, Key key) {
    if (n >= 2) return 1u;
    const uint2 th = n == 0 ? K.thr2 : K.thr1;
    return metropolis_accept(head, th, h, t, r, c, key) ? 1u : 0u;
}

struct Lattice2dArgs {
    const uint8_t *src;  // split planes of replica 0 (read)
    uint8_t *dst;        // split planes of replica 0 (written)
    int64_t rep_bytes;   // bytes per replica (L*L)
    const ThrRow *thr;   // per replica
    int64_t *dE;         // per replica or nullptr
    Key key;
    uint32_t t;
    int L, H, bands, n_rep;
};

// Update colour c of one lane-row: own (updated in place), vertical rows
// va/vb, horizontal row hz with edge word.  Returns the summed dE/4 + 2 per
// site via `de` (SWAR bytes) when counted.
template <int C>
__device__ __forceinline__ void update_row(Row<C> &own, const Row<C> &va, const Row<C> &vb, const Row<C> &hz,
                                           uint32_t edge, int p, uint32_t c, uint32_t row, uint32_t groups_per_row,
                                           uint32_t lane_group0, const Lut &K, Key key, uint32_t t, uint32_t r,
                                           bool count, uint32_t &de_total) {
    uint32_t n[2 * C], F[2 * C];
    uint4 w[C];
    uint32_t eq = 0xFFFFFFFFu;
#pragma unroll
    for (int q = 0; q < C; ++q) {
        const uint32_t g = row * groups_per_row + lane_group0 + q;
        w[q] = philox4x32_10(make_uint4(g, t, r, 2 * kTagHead + c), key);
    }
#pragma unroll
    for (int i = 0; i < 2 * C; ++i) {
        n[i] = count_anti<C>(own.d[i], va.d[i], vb.d[i], hz, i, edge, p);
        const uint4 &wq = w[i >> 1];
        const uint32_t wa = (i & 1) ? wq.z : wq.x;
        const uint32_t wb = (i & 1) ? wq.w : wq.y;
        F[i] = decide4(n[i], wa, wb, K, eq);
    }
    // a head equal to its threshold's high part: resolve those sites exactly
    const bool tie = ((eq & 0xFFFFu) == 0u) || ((eq >> 16) == 0u);
    if (__builtin_expect(__any(tie), 0)) {
        if (tie) {
#pragma unroll
            for (int i = 0; i < 2 * C; ++i) {
                const uint4 &wq = w[i >> 1];
                uint32_t f = 0;
                for (int s = 0; s < 4; ++s) {
                    const uint32_t k = 4 * (i & 1) + s;  // site within the chunk
                    const uint32_t word = word_of(wq, k >> 1);
                    const uint32_t head = (k & 1) ? (word >> 16) : (word & 0xFFFFu);
                    const uint32_t h = (row * groups_per_row + lane_group0 + (i >> 1)) * 8u + k;
                    f |= exact_flip((n[i] >> (8 * s)) & 0xFFu, head, K, h, t, r, c, key) << (8 * s);
                }
                F[i] = f;
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

// Neighbour-lane word exchange: every lane receives the last word of the
// lane to its left (dir 0) or the first word of the lane to its right
// (dir 1); the row wraps around through the workgroup.
__device__ __forceinline__ void exchange2(uint32_t v1, uint32_t v0, int dir, uint32_t *xch, int par,
                                          uint32_t &e1, uint32_t &e0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int send_lane = dir ? 0 : 63;
    if (lane == send_lane) {
        xch[(par * nw + wave) * 2] = v1;
        xch[(par * nw + wave) * 2 + 1] = v0;
    }
    __syncthreads();
    uint32_t s1 = dir ? __shfl_down(v1, 1) : __shfl_up(v1, 1);
    uint32_t s0 = dir ? __shfl_down(v0, 1) : __shfl_up(v0, 1);
    const int recv_lane = dir ? 63 : 0;
    if (lane == recv_lane) {
        const int other = dir ? (wave + 1 == nw ? 0 : wave + 1) : (wave == 0 ? nw - 1 : wave - 1);
        s1 = xch[(par * nw + other) * 2];
        s0 = xch[(par * nw + other) * 2 + 1];
    }
    e1 = s1;
    e0 = s0;
}

template <int C>
__global__ __launch_bounds__(1024) void k_ising2d_split(Lattice2dArgs a) {
    __shared__ uint32_t xch[2 * 16 * 2];
    // XCD-aware order: consecutive bands of a replica run on the same XCD.
    const uint32_t nblk = gridDim.x;
    const uint32_t xcd = blockIdx.x & 7u, slot = blockIdx.x >> 3;
    const uint32_t per_xcd = nblk >> 3;
    const uint32_t logical = (nblk & 7u) ? blockIdx.x : xcd * per_xcd + slot;
    const int r = (int)(logical / (uint32_t)a.bands);
    const int band = (int)(logical % (uint32_t)a.bands);
    const int L = a.L, H = a.H, half = L >> 1;
    const uint32_t gpr = (uint32_t)L >> 4;  // draw groups per row (8 sites each)
    const uint32_t lg0 = threadIdx.x * C;   // this lane's first group in a row
    const Lut K = make_lut(a.thr[r]);
    const uint8_t *S0 = a.src + (int64_t)r * a.rep_bytes;
    const uint8_t *S1 = S0 + (int64_t)half * L;
    uint8_t *D0 = a.dst + (int64_t)r * a.rep_bytes;
    uint8_t *D1 = D0 + (int64_t)half * L;
    const int64_t lane_off = (int64_t)threadIdx.x * 8 * C;
    auto rowp = [&](int y) { return (int64_t)((y % L + L) % L) * half + lane_off; };

    const int Y0 = band * H;
    // window for step j = Y0-1
    Row<C> q1m = load_row<C>(S1 + rowp(Y0 - 2));
    Row<C> q1c = load_row<C>(S1 + rowp(Y0 - 1));
    Row<C> q1p = load_row<C>(S1 + rowp(Y0));
    Row<C> q0c = load_row<C>(S0 + rowp(Y0 - 1));
    Row<C> pa1 = load_row<C>(S1 + rowp(Y0 + 1));  // plane 1 row j+2
    Row<C> pa0 = load_row<C>(S0 + rowp(Y0));      // plane 0 row j+1
    Row<C> n0m2, n0m1;
#pragma unroll
    for (int i = 0; i < 2 * C; ++i) n0m2.d[i] = n0m1.d[i] = 0u;
    uint32_t e1 = 0, e0 = 0;
    {
        const int dir = (Y0 - 1) & 1;
        exchange2(dir ? q1c.d[0] : q1c.d[2 * C - 1], 0u, dir, xch, 0, e1, e0);
    }
    uint32_t de_total = 0;
    uint32_t counted = 0;
    for (int j = Y0 - 1; j <= Y0 + H; ++j) {
        // prefetch the rows of step j+2
        Row<C> pb1, pb0;
#pragma unroll
        for (int i = 0; i < 2 * C; ++i) pb1.d[i] = pb0.d[i] = 0u;
        if (j + 3 <= Y0 + H + 1) pb1 = load_row<C>(S1 + rowp(j + 3));
        if (j + 2 <= Y0 + H) pb0 = load_row<C>(S0 + rowp(j + 2));
        const uint32_t jm = (uint32_t)((j % L + L) % L);
        const int p = j & 1;
        // colour 0 of row j
        const bool in0 = j >= Y0 && j < Y0 + H;
        Row<C> n0c = q0c;
        update_row<C>(n0c, q1m, q1p, q1c, e1, p, 0u, jm, gpr, lg0, K, a.key, a.t, (uint32_t)r, in0, de_total);
        counted += in0 ? 1u : 0u;
        if (j >= Y0 + 1) {
            // colour 1 of row j-1 from the new colour-0 rows j-2, j-1, j
            const uint32_t jm1 = jm == 0 ? (uint32_t)L - 1u : jm - 1u;
            update_row<C>(q1m, n0m2, n0c, n0m1, e0, p, 1u, jm1, gpr, lg0, K, a.key, a.t, (uint32_t)r, true,
                          de_total);
            counted += 1u;
            store_row<C>(D0 + rowp(j - 1), n0m1);
            store_row<C>(D1 + rowp(j - 1), q1m);
        }
        // rotate the window
        n0m2 = n0m1;
        n0m1 = n0c;
        q1m = q1c;
        q1c = q1p;
        q1p = pa1;
        q0c = pa0;
        pa1 = pb1;
        pa0 = pb0;
        if (j < Y0 + H) {
            const int dir = (j + 1) & 1;
            exchange2(dir ? q1c.d[0] : q1c.d[2 * C - 1], dir ? n0m1.d[0] : n0m1.d[2 * C - 1], dir, xch, j & 1,
                      e1, e0);
        }
    }
    if (a.dE) {
        // sum over sites of (dE/4 + 2) minus 2 per counted site
        long long v = ((long long)de_total - 2ll * (long long)counted * 8 * C) * 4;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0 && v != 0) atomicAdd((unsigned long long *)&a.dE[r], (unsigned long long)v);
    }
}

// ----------------------------------------------------- layout conversion ----
// ABI row-major int8 +-1  <->  split planes of 0/1 bytes (x even -> plane
// (y&1), x odd -> plane ((y+1)&1), plane index x/2).
__global__ __launch_bounds__(256) void k_to_split(const int8_t *src, uint8_t *dst, int L, int64_t chunks_per_rep,
                                                  int64_t total) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const int64_t r = gid / chunks_per_rep, cidx = gid % chunks_per_rep;
    const int cpr = L >> 4;  // 16-site chunks per row
    const int y = (int)(cidx / cpr), xc = (int)(cidx % cpr);
    const int64_t N = (int64_t)L * L;
    const uint4 v = *(const uint4 *)(src + r * N + (int64_t)y * L + 16 * xc);
    const uint32_t m = 0x01010101u;
    const uint32_t b0 = (v.x >> 1) & m, b1 = (v.y >> 1) & m, b2 = (v.z >> 1) & m, b3 = (v.w >> 1) & m;
    const uint2 ev = make_uint2(perm(b1, b0, 0x06040200u), perm(b3, b2, 0x06040200u));
    const uint2 od = make_uint2(perm(b1, b0, 0x07050301u), perm(b3, b2, 0x07050301u));
    uint8_t *base = dst + r * N;
    const int64_t off = (int64_t)y * (L >> 1) + 8 * xc;
    const int pe = y & 1, po = (y + 1) & 1;
    *(uint2 *)(base + (int64_t)pe * (N >> 1) + off) = ev;
    *(uint2 *)(base + (int64_t)po * (N >> 1) + off) = od;
}

__device__ __forceinline__ uint32_t pm1(uint32_t b) { return ((b << 8) - b) | 0x01010101u; }

__global__ __launch_bounds__(256) void k_from_split(const uint8_t *src, int8_t *dst, int L, int64_t chunks_per_rep,
                                                    int64_t total) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= total) return;
    const int64_t r = gid / chunks_per_rep, cidx = gid % chunks_per_rep;
    const int cpr = L >> 4;
    const int y = (int)(cidx / cpr), xc = (int)(cidx % cpr);
    const int64_t N = (int64_t)L * L;
    const uint8_t *base = src + r * N;
    const int64_t off = (int64_t)y * (L >> 1) + 8 * xc;
    const int pe = y & 1, po = (y + 1) & 1;
    const uint2 ev = *(const uint2 *)(base + (int64_t)pe * (N >> 1) + off);
    const uint2 od = *(const uint2 *)(base + (int64_t)po * (N >> 1) + off);
    const uint32_t e0 = pm1(ev.x), e1 = pm1(ev.y), o0 = pm1(od.x), o1 = pm1(od.y);
    uint4 v;
    v.x = perm(o0, e0, 0x05010400u);
    v.y = perm(o0, e0, 0x07030602u);
    v.z = perm(o1, e1, 0x05010400u);
    v.w = perm(o1, e1, 0x07030602u);
    *(uint4 *)(dst + r * N + (int64_t)y * L + 16 * xc) = v;
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
    if (L % 1024 != 0 || L < 1024) return 0;
    const int lanes16 = L / 16;  // lanes at one chunk each
    const int want = env_int("SPINMC_L2D_CHUNKS", 0);
    if (want == 1 || want == 2 || want == 4)
        if (lanes16 / want <= 1024 && lanes16 % (want * 64) == 0) return want;
    for (int C = 1; C <= 4; C *= 2)
        if (lanes16 / C <= 1024 && lanes16 % (C * 64) == 0) return C;
    return 0;
}

bool lattice2d_supported(int L) { return lattice2d_chunks(L) > 0; }

int lattice2d_band_height(int L, int n_rep) {
    (void)n_rep;
    int H = env_int("SPINMC_L2D_H", 64);
    if (H < 2 || H % 2 || L % H) H = 64;
    while (H > 2 && L % H) H >>= 1;
    return L % H ? 0 : H;
}

hipError_t launch_to_split(const int8_t *src, uint8_t *dst, int L, int n_rep, hipStream_t s) {
    const int64_t cpr = (int64_t)L * L / 16, total = cpr * n_rep;
    hipLaunchKernelGGL(k_to_split, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, L, cpr, total);
    return hipGetLastError();
}

hipError_t launch_from_split(const uint8_t *src, int8_t *dst, int L, int n_rep, hipStream_t s) {
    const int64_t cpr = (int64_t)L * L / 16, total = cpr * n_rep;
    hipLaunchKernelGGL(k_from_split, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, dst, L, cpr, total);
    return hipGetLastError();
}

hipError_t launch_ising2d_split(const uint8_t *src, uint8_t *dst, int L, int n_rep, const ThrRow *thr, int64_t *dE,
                                Key key, uint32_t t, hipStream_t s) {
    const int C = lattice2d_chunks(L);
    const int H = lattice2d_band_height(L, n_rep);
    if (C == 0 || H == 0) return hipErrorInvalidValue;
    Lattice2dArgs a;
    a.src = src;
    a.dst = dst;
    a.rep_bytes = (int64_t)L * L;
    a.thr = thr;
    a.dE = dE;
    a.key = key;
    a.t = t;
    a.L = L;
    a.H = H;
    a.bands = L / H;
    a.n_rep = n_rep;
    const unsigned threads = (unsigned)(L / (16 * C));
    const unsigned blocks = (unsigned)(a.bands * n_rep);
    switch (C) {
        case 1: hipLaunchKernelGGL(k_ising2d_split<1>, dim3(blocks), dim3(threads), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_ising2d_split<2>, dim3(blocks), dim3(threads), 0, s, a); break;
        case 4: hipLaunchKernelGGL(k_ising2d_split<4>, dim3(blocks), dim3(threads), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace smc

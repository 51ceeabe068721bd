// Parallel tempering of 3D Ising / +-J Edwards-Anderson lattices of edge 16
// with every step of a call inside one launch (Sec. 6, Eq. 12).
//
// One workgroup runs one chain: the n_temps replicas of the chain and the
// coupling sample they share stay in LDS for all n_steps steps (m sweeps of
// every replica, sweep indices t*m .. t*m + m - 1, then the exchange round
// of step t), and go back to HBM
// once at the end.  Results are those of the sweep and exchange kernels of
// the generic path step for step: colour 0 then colour 1 per sweep, the same
// Philox streams keyed by (seed, step, replica storage index, site), the
// same integer thresholds, the same FP64 exchange test.
//
// LDS layout of a replica (4 KiB): row rho = z*16 + y holds 16 bytes, the
// eight sites with even x (array E, x = 2i) and the eight with odd x (array
// O, x = 2i+1), one byte per site with value (1 - s)/2.  The E sites of row
// (y, z) have colour (y + z) & 1, the O sites the other colour.  A colour-c
// pass updates, in every row, the array of colour c: its x neighbours are the
// other array of the same row (shifted by one byte with wrap-around), its y
// and z neighbours the same array of the four adjacent rows.
#include "internal.hpp"
#include "intrin.hpp"

namespace smc {
namespace {

constexpr int kEdge = 16;
constexpr int kRowsPerRep = kEdge * kEdge;      // (z, y) rows
constexpr int kRepWords = kRowsPerRep * 4;      // 16 bytes per row
constexpr int kSites = kEdge * kEdge * kEdge;   // 4096
constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxTemps = 2 * kWaves;           // two replicas per wave
constexpr int kCoupWords = kRowsPerRep * 2 * 6 * 2;  // [row][array][direction][2 words]

struct Pt3dArgs {
    int8_t *spins;            // [n_rep][4096] int8 +-1; chain q owns replicas q*n_temps ...
    const int8_t *coup;       // EA: [sample][3][4096] int8 +-1; Ising: nullptr
    int rep_per_sample;
    int n_chains, n_temps, beta_per_chain;
    const double *beta;       // [rows][n_temps]
    const ThrRow *thr;        // [rows][n_temps]
    int32_t *slot_of_temp;    // [n_chains][n_temps]
    double *energy;           // [n_rep]
    unsigned long long *acc;  // [n_chains][n_temps - 1] or nullptr
    Key key;
    uint32_t t0;
    int n_steps;
    int m;          // sweeps per step
    uint32_t one2;  // 0x00010001 (opaque to the compiler, keeps the packed 16-bit ops)
};


// Threshold table of one temperature for the byte-parallel decision: the
// high 16 bits of the threshold for n unsatisfied bonds (n = 0, 1, 2 give
// Delta E = 12, 8, 4), 0xFFFF for n >= 3 (Delta E <= 0, always accepted; a
// head of 0xFFFF goes through the exact path), split into low and high bytes
// indexed by n.
struct TempLut {
    uint32_t lo, hi;
};

__device__ __forceinline__ TempLut temp_lut(const ThrRow &row) {
    const uint32_t t3 = row.m[3].x, t2 = row.m[2].x, t1 = row.m[1].x;  // <= 0xFFFF (checked on the host)
    TempLut k;
    k.lo = (t3 & 0xFFu) | ((t2 & 0xFFu) << 8) | ((t1 & 0xFFu) << 16) | 0xFF000000u;
    k.hi = (t3 >> 8) | ((t2 >> 8) << 8) | ((t1 >> 8) << 16) | 0xFF000000u;
    return k;
}

// Flip flags (0/1 bytes) of four sites with unsatisfied-bond counts n (bytes
// 0..6) and heads in wa (sites 0, 1) and wb (sites 2, 3).  eq collects the
// 16-bit differences threshold - head; a zero marks a head equal to the high
// half of its threshold, which needs the exact decision.
__device__ __forceinline__ uint32_t decide4(uint32_t n, uint32_t wa, uint32_t wb, TempLut k, uint32_t one2,
                                            uint32_t &eq) {
    const uint32_t tl = perm(0xFFFFFFFFu, k.lo, n);
    const uint32_t th = perm(0xFFFFFFFFu, k.hi, n);
    const uint32_t ta = perm(th, tl, 0x05010400u);  // sites 0, 1 as 16-bit lanes
    const uint32_t tb = perm(th, tl, 0x07030602u);  // sites 2, 3
    const uint32_t ra = min16(sub_sat16(ta, wa), one2);
    const uint32_t rb = min16(sub_sat16(tb, wb), one2);
    eq = min16(eq, min16(sub16(ta, wa), sub16(tb, wb)));
    return perm(rb, ra, 0x06040200u);
}

// Shared state of the chain besides the lattices.
struct ChainState {
    ThrRow thr[kMaxTemps];
    double beta[kMaxTemps];
    int E[kMaxTemps];           // energy of replica slot s
    int temp_of_slot[kMaxTemps];
    int slot_of_temp[kMaxTemps];
    unsigned acc[kMaxTemps];
    int bad;
};

// Row of pass index idx (0..127) among the rows with (y + z) & 1 == P.
__device__ __forceinline__ int row_of(int idx, int P) {
    const int z = idx >> 3, j = idx & 7;
    return z * kEdge + 2 * j + ((z + P) & 1);
}

// One colour-c pass of rows whose own array is a (0: E, 1: O) for the
// replicas s0 and s1 = s0 + kWaves (s1 only if < n).  Accumulates per
// replica the number of flips (cnt) and the sum of n over flips (nsum).
template <bool EA>
__device__ __forceinline__ void half_pass(uint32_t *S, const uint32_t *Cb, const ChainState &cs, int a, int P, int c,
                                          int s0, int n, uint32_t rbase, uint32_t t, Key key, uint32_t one2,
                                          uint32_t (&cnt)[2], uint32_t (&nsum)[2]) {
    const int lane = threadIdx.x & 63;
    const bool has1 = s0 + kWaves < n;
    const int s1 = has1 ? s0 + kWaves : s0;
    const TempLut k0 = temp_lut(cs.thr[cs.temp_of_slot[s0]]);
    const TempLut k1 = temp_lut(cs.thr[cs.temp_of_slot[s1]]);
#pragma unroll 1
    for (int rr = 0; rr < 2; ++rr) {
        const int row = row_of(lane + 64 * rr, P);
        const int z = row >> 4, y = row & 15;
        const int rym = z * kEdge + ((y + 15) & 15), ryp = z * kEdge + ((y + 1) & 15);
        const int rzm = ((z + 15) & 15) * kEdge + y, rzp = ((z + 1) & 15) * kEdge + y;
        // coupling bytes of the row: (x-, x+), (y-, y+), (z-, z+), two words each
        uint4 cx = make_uint4(0u, 0u, 0u, 0u), cy = cx, cz = cx;
        if constexpr (EA) {
            const uint4 *cp = (const uint4 *)(Cb + (row * 2 + a) * 12);
            cx = cp[0];
            cy = cp[1];
            cz = cp[2];
        }
        uint4 w[2];
        w[0] = make_uint4((uint32_t)row, t, rbase + (uint32_t)s0, 2 * kTagHead + (uint32_t)c);
        w[1] = make_uint4((uint32_t)row, t, rbase + (uint32_t)s1, 2 * kTagHead + (uint32_t)c);
        philox4x32_10_multi<2>(w, key);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (q == 1 && !has1) break;
            const int s = q ? s1 : s0;
            uint32_t *R = S + s * kRepWords;
            const uint2 own = *(const uint2 *)(R + row * 4 + 2 * a);
            const uint2 oth = *(const uint2 *)(R + row * 4 + 2 * (1 - a));
            const uint2 ym = *(const uint2 *)(R + rym * 4 + 2 * a);
            const uint2 yp = *(const uint2 *)(R + ryp * 4 + 2 * a);
            const uint2 zm = *(const uint2 *)(R + rzm * 4 + 2 * a);
            const uint2 zp = *(const uint2 *)(R + rzp * 4 + 2 * a);
            // x neighbours: E site 2i has O[i-1], O[i]; O site 2i+1 has E[i], E[i+1]
            uint32_t xl0, xl1, xr0, xr1;
            if (a == 0) {
                xl0 = alignbyte(oth.x, oth.y, 3);
                xl1 = alignbyte(oth.y, oth.x, 3);
                xr0 = oth.x;
                xr1 = oth.y;
            } else {
                xl0 = oth.x;
                xl1 = oth.y;
                xr0 = alignbyte(oth.y, oth.x, 1);
                xr1 = alignbyte(oth.x, oth.y, 1);
            }
            uint32_t n0, n1;
            if constexpr (EA) {
                n0 = ((own.x ^ xl0 ^ cx.x) + (own.x ^ xr0 ^ cx.z)) + ((own.x ^ ym.x ^ cy.x) + (own.x ^ yp.x ^ cy.z)) +
                     ((own.x ^ zm.x ^ cz.x) + (own.x ^ zp.x ^ cz.z));
                n1 = ((own.y ^ xl1 ^ cx.y) + (own.y ^ xr1 ^ cx.w)) + ((own.y ^ ym.y ^ cy.y) + (own.y ^ yp.y ^ cy.w)) +
                     ((own.y ^ zm.y ^ cz.y) + (own.y ^ zp.y ^ cz.w));
            } else {
                n0 = ((own.x ^ xl0) + (own.x ^ xr0)) + ((own.x ^ ym.x) + (own.x ^ yp.x)) +
                     ((own.x ^ zm.x) + (own.x ^ zp.x));
                n1 = ((own.y ^ xl1) + (own.y ^ xr1)) + ((own.y ^ ym.y) + (own.y ^ yp.y)) +
                     ((own.y ^ zm.y) + (own.y ^ zp.y));
            }
            const TempLut K = q ? k1 : k0;
            uint32_t eq = 0xFFFFFFFFu;
            uint32_t F0 = decide4(n0, w[q].x, w[q].y, K, one2, eq);
            uint32_t F1 = decide4(n1, w[q].z, w[q].w, K, one2, eq);
            const bool tie = ((eq & 0xFFFFu) == 0u) || ((eq >> 16) == 0u);
            if (__builtin_expect(__any(tie), 0)) {
                // Exact decisions of the sites whose head equals the high half
                // of the threshold (probability 2^-16 each).  A wavefront that
                // meets one holds up the workgroup at the next barrier, so the
                // path is short: a mask of the tied sites, then one pass per
                // tied site of the lane with most of them (almost always one),
                // each drawing the single tail it needs.
                uint32_t tm = 0;  // bit i: site i (0 .. 7) is tied
                if (tie) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t nn = h ? n1 : n0;
                        const uint32_t tl = perm(0xFFFFFFFFu, K.lo, nn), thh = perm(0xFFFFFFFFu, K.hi, nn);
                        const uint32_t da = perm(thh, tl, 0x05010400u) ^ (h ? w[q].z : w[q].x);
                        const uint32_t db = perm(thh, tl, 0x07030602u) ^ (h ? w[q].w : w[q].y);
                        const uint32_t m4 = ((da & 0xFFFFu) == 0u ? 1u : 0u) | ((da >> 16) == 0u ? 2u : 0u) |
                                            ((db & 0xFFFFu) == 0u ? 4u : 0u) | ((db >> 16) == 0u ? 8u : 0u);
                        tm |= m4 << (4 * h);
                    }
                }
                const ThrRow &th = cs.thr[cs.temp_of_slot[s]];
                while (__any(tm != 0u)) {
                    if (tm != 0u) {
                        const uint32_t i = __builtin_ctz(tm), b = 8u * (i & 3u);
                        tm &= tm - 1u;
                        const uint32_t ns = ((i < 4u ? n0 : n1) >> b) & 0xFFu;
                        uint32_t flip = 1u;  // a head of 0xFFFF at a site with Delta E <= 0
                        if (ns < 3u) {
                            // the head equals the threshold's high half: compare the tail
                            const uint32_t h = (uint32_t)row * 8u + i;
                            flip = tail16(h, t, rbase + (uint32_t)s, (uint32_t)c, key) < th.m[3u - ns].y ? 1u : 0u;
                        }
                        const uint32_t keep = ~(0xFFu << b), set = flip << b;
                        if (i < 4u)
                            F0 = (F0 & keep) | set;
                        else
                            F1 = (F1 & keep) | set;
                    }
                }
            }
            *(uint2 *)(R + row * 4 + 2 * a) = make_uint2(own.x ^ F0, own.y ^ F1);
            // Delta E of a flip with n unsatisfied bonds is 4 (3 - n)
            const uint32_t m0 = bytes_ff(F0), m1 = bytes_ff(F1);  // 0xFF where flipped
            cnt[q] = __builtin_amdgcn_sad_u8(F0, 0u, __builtin_amdgcn_sad_u8(F1, 0u, cnt[q]));
            nsum[q] = __builtin_amdgcn_sad_u8(n0 & m0, 0u, __builtin_amdgcn_sad_u8(n1 & m1, 0u, nsum[q]));
        }
    }
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool EA>
__global__ __launch_bounds__(kThreads) void k_pt3d_chain(Pt3dArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];  // [n][1024] lattices, then the EA coupling table
    __shared__ ChainState cs;
    const int q = blockIdx.x;
    const int n = a.n_temps;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    uint32_t *S = lds;
    uint32_t *Cb = lds + n * kRepWords;
    const uint32_t rbase = (uint32_t)(q * n);
    const int trow = a.beta_per_chain ? q * n : 0;

    // ---- chain state: the permutation must be one, else the chain is left as it is
    if (tid == 0) cs.bad = 0;
    __syncthreads();
    if (tid < n) {
        const int s = a.slot_of_temp[(int64_t)q * n + tid];
        cs.slot_of_temp[tid] = s;
        cs.thr[tid] = a.thr[trow + tid];
        cs.beta[tid] = a.beta[trow + tid];
        cs.acc[tid] = 0u;
        cs.E[tid] = (int)a.energy[(int64_t)q * n + tid];
        if ((unsigned)s >= (unsigned)n) atomicOr(&cs.bad, 1);
    }
    __syncthreads();
    if (tid < n) {
        int seen = 0;
        for (int k = 0; k < n; ++k) seen += cs.slot_of_temp[k] == tid ? 1 : 0;
        if (seen != 1) atomicOr(&cs.bad, 1);
        if (cs.bad == 0) cs.temp_of_slot[cs.slot_of_temp[tid]] = tid;
    }
    __syncthreads();
    if (cs.bad) return;

    // ---- lattices into LDS
    const int8_t *gsp = a.spins + (int64_t)q * n * kSites;
    for (int i = tid; i < n * kRowsPerRep; i += kThreads) {
        const uint4 v = *(const uint4 *)(gsp + (int64_t)i * 16);
        const uint32_t m = 0x01010101u;
        const uint32_t b0 = (v.x >> 1) & m, b1 = (v.y >> 1) & m, b2 = (v.z >> 1) & m, b3 = (v.w >> 1) & m;
        *(uint4 *)(S + i * 4) = make_uint4(perm(b1, b0, 0x06040200u), perm(b3, b2, 0x06040200u),
                                           perm(b1, b0, 0x07050301u), perm(b3, b2, 0x07050301u));
    }
    // ---- coupling table: byte = 1 where J = -1, per (row, array, direction)
    if constexpr (EA) {
        const int sample = (int)(rbase / (uint32_t)a.rep_per_sample);
        const int8_t *J = a.coup + (int64_t)sample * 3 * kSites;
        for (int u = tid; u < kRowsPerRep * 2 * 6; u += kThreads) {
            const int d = u % 6, ra = u / 6, arr = ra & 1, row = ra >> 1;
            const int z = row >> 4, y = row & 15;
            uint32_t word[2] = {0u, 0u};
            for (int i = 0; i < 8; ++i) {
                const int x = 2 * i + arr;
                int xs = x, ys = y, zs = z, mu;
                switch (d) {
                    case 0: xs = (x + 15) & 15; mu = 0; break;  // x-: bond of the left neighbour
                    case 1: mu = 0; break;                      // x+
                    case 2: ys = (y + 15) & 15; mu = 1; break;  // y-
                    case 3: mu = 1; break;                      // y+
                    case 4: zs = (z + 15) & 15; mu = 2; break;  // z-
                    default: mu = 2; break;                     // z+
                }
                const int site = (zs * kEdge + ys) * kEdge + xs;
                const uint32_t cbit = J[(int64_t)mu * kSites + site] < 0 ? 1u : 0u;
                word[i >> 2] |= cbit << (8 * (i & 3));
            }
            *(uint2 *)(Cb + u * 2) = make_uint2(word[0], word[1]);
        }
    }
    __syncthreads();

    // ---- the steps
    const int s0 = wave;
    const bool active = s0 < n;
    for (int step = 0; step < a.n_steps; ++step) {
        const uint32_t t = a.t0 + (uint32_t)step;
        for (int j = 0; j < a.m; ++j) {
            const uint32_t ts = t * (uint32_t)a.m + (uint32_t)j;  // sweep index
            uint32_t cnt[2] = {0u, 0u}, nsum[2] = {0u, 0u};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (active) {
                    // rows with (y+z)&1 == c update array E, the others array O
                    half_pass<EA>(S, Cb, cs, 0, c, c, s0, n, rbase, ts, a.key, a.one2, cnt, nsum);
                    half_pass<EA>(S, Cb, cs, 1, 1 - c, c, s0, n, rbase, ts, a.key, a.one2, cnt, nsum);
                }
                __syncthreads();
            }
            if (active) {
                const int d0 = wave_sum(3 * (int)cnt[0] - (int)nsum[0]);
                const int d1 = wave_sum(3 * (int)cnt[1] - (int)nsum[1]);
                if (lane == 0) {
                    cs.E[s0] += 4 * d0;
                    if (s0 + kWaves < n) cs.E[s0 + kWaves] += 4 * d1;
                }
            }
            __syncthreads();
        }
        // exchange round: pairs (k, k+1) with k = t mod 2, one thread each
        if (tid < n - 1 && (((uint32_t)tid ^ t) & 1u) == 0u) {
#pragma clang fp contract(off)
            const int k = tid;
            const int A = cs.slot_of_temp[k], B = cs.slot_of_temp[k + 1];
            const double x = (cs.beta[k + 1] - cs.beta[k]) * (double)(cs.E[B] - cs.E[A]);
            bool accept = x >= 0.0;
            if (!accept) {
                const uint4 w = philox4x32_10(make_uint4((uint32_t)k, t, (uint32_t)q, 2 * kTagSwap), a.key);
                accept = unit53(w.x, w.y) < exp(x);
            }
            if (accept) {
                cs.slot_of_temp[k] = B;
                cs.slot_of_temp[k + 1] = A;
                cs.temp_of_slot[B] = k;
                cs.temp_of_slot[A] = k + 1;
                cs.acc[k] += 1u;
            }
        }
        __syncthreads();
    }

    // ---- back to HBM
    int8_t *osp = a.spins + (int64_t)q * n * kSites;
    for (int i = tid; i < n * kRowsPerRep; i += kThreads) {
        const uint4 v = *(const uint4 *)(S + i * 4);  // E0..3, E4..7, O0..3, O4..7
        const uint32_t b0 = perm(v.z, v.x, 0x05010400u), b1 = perm(v.z, v.x, 0x07030602u);
        const uint32_t b2 = perm(v.w, v.y, 0x05010400u), b3 = perm(v.w, v.y, 0x07030602u);
        *(uint4 *)(osp + (int64_t)i * 16) = make_uint4(bytes_pm1(b0), bytes_pm1(b1), bytes_pm1(b2), bytes_pm1(b3));
    }
    if (tid < n) {
        a.slot_of_temp[(int64_t)q * n + tid] = cs.slot_of_temp[tid];
        a.energy[(int64_t)q * n + tid] = (double)cs.E[tid];
        if (a.acc && tid < n - 1) a.acc[(int64_t)q * (n - 1) + tid] += (unsigned long long)cs.acc[tid];
    }
}

}  // namespace

bool pt3d_supported(const smc_desc *d, int n_temps) {
    if (d->model != SMC_ISING && d->model != SMC_EA) return false;
    if (d->dim != 3 || d->L != kEdge) return false;
    if (n_temps < 2 || n_temps > kMaxTemps) return false;
    if (d->model == SMC_EA && d->rep_per_sample % n_temps) return false;
    return true;
}

size_t pt3d_lds_bytes(int model, int n_temps) {
    return (size_t)n_temps * kRepWords * 4 + (model == SMC_EA ? (size_t)kCoupWords * 4 : 0);
}

hipError_t launch_pt3d(int model, int8_t *spins, const int8_t *coup, int rep_per_sample, int n_chains, int n_temps,
                       int beta_per_chain, const double *beta, const ThrRow *thr, int32_t *slot_of_temp,
                       double *energy, unsigned long long *acc, Key key, uint32_t t0, int n_steps, int m,
                       hipStream_t s) {
    Pt3dArgs a;
    a.spins = spins;
    a.coup = coup;
    a.rep_per_sample = rep_per_sample;
    a.n_chains = n_chains;
    a.n_temps = n_temps;
    a.beta_per_chain = beta_per_chain;
    a.beta = beta;
    a.thr = thr;
    a.slot_of_temp = slot_of_temp;
    a.energy = energy;
    a.acc = acc;
    a.key = key;
    a.t0 = t0;
    a.n_steps = n_steps;
    a.m = m;
    a.one2 = 0x00010001u;
    const size_t lds = pt3d_lds_bytes(model, n_temps);
    if (model == SMC_EA) {
        (void)hipFuncSetAttribute((const void *)k_pt3d_chain<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        SMC_LAUNCH(k_pt3d_chain<true>, dim3(n_chains), dim3(kThreads), lds, s, a);
    } else {
        (void)hipFuncSetAttribute((const void *)k_pt3d_chain<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        SMC_LAUNCH(k_pt3d_chain<false>, dim3(n_chains), dim3(kThreads), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace smc

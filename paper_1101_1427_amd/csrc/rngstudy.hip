// The random-number study of Sec. 3.3 (Table 1): the double checkerboard of
// 2D Ising / +-J EA lattices driven by the paper's generators instead of the
// counter-based Philox streams, so that their effect on the sampled
// distribution can be measured.
//
// Generators (Sec. 3.3): LCG32 x' = 1664525 x + 1013904223 mod 2^32 and
// LCG64 x' = 2862933555777941757 x + 1442695040888963407 mod 2^64 (uniform:
// its top 32 bits), either all streams reading one global sequence with
// skip-ahead (stream j delivers x_j, x_{j+M}, ...: the step is the M-th
// power of the map, Eqs. 4-5) or every stream seeded independently and
// stepped by the map itself; and the lagged Fibonacci generator x_n =
// x_{n-r} + x_{n-s} mod 2^32 with (r, s) = (521, 353) or (1279, 861),
// one per tile, whose ring buffer of r words sits in LDS while the tile is
// updated (Sec. 3.3 shares it among the threads of a block).
//
// Layout of the update: one workgroup per tile of the current tile colour,
// T^2/2 threads; thread p owns in-colour position p of the tile (site
// (u, v) with v = p / (T/2), u = 2 (p mod T/2) + ((c + v) & 1) for colour c)
// and the stream j = q T^2/2 + p of the tile's index q among its tile colour
// (q = by (B/2) + bx/2).  A hit updates colour 0, then colour 1, every
// thread drawing one number per colour (also where Delta E <= 0 decides
// alone); the tile and a one-site halo sit in LDS for all k hits.  The
// acceptance is the integer test u < floor(2^32 exp(-beta Delta E)) of the
// Philox sweeps.
#include "internal.hpp"

namespace smc {
namespace {

constexpr int kFamLcg32 = 0, kFamLcg64 = 1, kFamFib = 2;

struct StudyArgs {
    int8_t *spins;        // replica r at r * L^2
    const int8_t *coup;   // EA: [sample][2][L^2], or nullptr
    int rep_per_sample;
    const ThrRow *thr;    // per replica
    void *state;          // generator state, replica-major
    int64_t state_words;  // 32- or 64-bit words of one replica's state
    unsigned long long *dE;  // per replica, or nullptr
    uint64_t A, C;        // LCG step (skip-ahead: the M-th power of the map)
    int L, T, B, k, tc;   // edge, tile, tiles per direction, hits, tile colour of this launch
    int r_lag, s_lag;     // Fibonacci lags
};

__device__ __forceinline__ int wrapi(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

template <int FAM>
__global__ __launch_bounds__(512) void k_dcb_rng(StudyArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];  // (T+2)^2 spins, then the Fibonacci ring (r + 1 words)
    const int T = a.T, W = T + 2, P = T * T / 2, L = a.L;
    const int tiles = a.B * a.B / 2;
    const int rep = (int)blockIdx.x / tiles, q = (int)blockIdx.x % tiles;
    const int by = q / (a.B / 2), bx = 2 * (q % (a.B / 2)) + ((by + a.tc) & 1);
    const int p = (int)threadIdx.x;
    const int64_t N = (int64_t)L * L;
    int8_t *S = a.spins + (int64_t)rep * N;
    int8_t *tile = (int8_t *)smem;
    uint32_t *ring = (uint32_t *)(smem + ((W * W + 15) & ~15));
    // tile and halo into LDS
    for (int cell = p; cell < W * W; cell += P) {
        const int cu = cell % W, cv = cell / W;
        const int x = wrapi(bx * T + cu - 1, L), y = wrapi(by * T + cv - 1, L);
        tile[cell] = S[(int64_t)y * L + x];
    }
    // generator state of this thread / tile
    uint32_t x32 = 0u;
    uint64_t x64 = 0u;
    uint32_t n0 = 0u;
    const int64_t j = (int64_t)q * P + p;
    if constexpr (FAM == kFamLcg32) x32 = ((const uint32_t *)a.state)[(int64_t)rep * a.state_words + j];
    if constexpr (FAM == kFamLcg64) x64 = ((const uint64_t *)a.state)[(int64_t)rep * a.state_words + j];
    const uint32_t *gring = nullptr;
    if constexpr (FAM == kFamFib) {
        gring = (const uint32_t *)a.state + (int64_t)rep * a.state_words + (int64_t)q * (a.r_lag + 1);
        for (int w = p; w <= a.r_lag; w += P) ring[w] = gring[w];
    }
    __syncthreads();
    if constexpr (FAM == kFamFib) n0 = ring[a.r_lag];
    // the thread's two sites (colour 0 and colour 1 at position p) and their bonds
    const int v = p / (T / 2);
    int cell_of[2], ix[2];
    int jr[2] = {1, 1}, jl[2] = {1, 1}, ju[2] = {1, 1}, jd[2] = {1, 1};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int u = 2 * (p % (T / 2)) + ((c + v) & 1);
        cell_of[c] = (v + 1) * W + (u + 1);
        const int x = bx * T + u, y = by * T + v;
        ix[c] = y * L + x;
        if (a.coup) {
            const int8_t *J = a.coup + (int64_t)(rep / a.rep_per_sample) * 2 * N;
            jr[c] = J[(int64_t)y * L + x];
            jl[c] = J[(int64_t)y * L + wrapi(x - 1, L)];
            ju[c] = J[N + (int64_t)y * L + x];
            jd[c] = J[N + (int64_t)wrapi(y - 1, L) * L + x];
        }
    }
    const ThrRow th = a.thr[rep];
    long long dE = 0;
    for (int hit = 0; hit < a.k; ++hit) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            uint32_t uu;
            if constexpr (FAM == kFamLcg32) {
                uu = x32;
                x32 = (uint32_t)a.A * x32 + (uint32_t)a.C;
            } else if constexpr (FAM == kFamLcg64) {
                uu = (uint32_t)(x64 >> 32);
                x64 = a.A * x64 + a.C;
            } else {
                // position p of this round takes number n0 + p: x_{n-r} sits in
                // its own slot, x_{n-s} in a slot no thread writes this round
                const uint32_t sn = (n0 + (uint32_t)p) % (uint32_t)a.r_lag;
                const uint32_t sb = (n0 + (uint32_t)p + (uint32_t)(a.r_lag - a.s_lag)) % (uint32_t)a.r_lag;
                uu = ring[sn] + ring[sb];
                ring[sn] = uu;
                n0 = (n0 + (uint32_t)P) % (uint32_t)a.r_lag;
            }
            const int cc = cell_of[c];
            const int s0 = tile[cc];
            const int h = jr[c] * tile[cc + 1] + jl[c] * tile[cc - 1] + ju[c] * tile[cc + W] + jd[c] * tile[cc - W];
            const int d = 2 * s0 * h;
            bool accept = d <= 0;
            if (!accept) {
                const uint2 t2 = th.m[d >> 2];
                accept = (uint64_t)uu < (((uint64_t)t2.x << 16) | t2.y);
            }
            if (accept) {
                tile[cc] = (int8_t)(-s0);
                dE += d;
            }
            __syncthreads();
        }
    }
    // tile interior back, generator state back
#pragma unroll
    for (int c = 0; c < 2; ++c) S[ix[c]] = tile[cell_of[c]];
    if constexpr (FAM == kFamLcg32) ((uint32_t *)a.state)[(int64_t)rep * a.state_words + j] = x32;
    if constexpr (FAM == kFamLcg64) ((uint64_t *)a.state)[(int64_t)rep * a.state_words + j] = x64;
    if constexpr (FAM == kFamFib) {
        uint32_t *out = (uint32_t *)a.state + (int64_t)rep * a.state_words + (int64_t)q * (a.r_lag + 1);
        for (int w = p; w < a.r_lag; w += P) out[w] = ring[w];
        if (p == 0) out[a.r_lag] = n0;
    }
    if (a.dE) {
        __shared__ long long red[8];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dE += __shfl_xor(dE, o, 64);
        if ((p & 63) == 0) red[p >> 6] = dE;
        __syncthreads();
        if (p == 0) {
            long long tot = 0;
            for (int w = 0; w < (P + 63) / 64; ++w) tot += red[w];
            if (tot != 0) atomicAdd(&a.dE[rep], (unsigned long long)tot);
        }
    }
}

// Initial state.  Skip-ahead LCGs: stream j holds x_j of the replica's global
// sequence, x_j = f^j(x_0) for the map f, by binary powers of f; x_0 and the
// independent stream seeds come from Philox draws with counter word 3 = 16:
// (0, 0, r, 16) for x_0, (j, 1, r, 16) for stream j, (q r_lag + i, 2, r, 16)
// for word i of tile q's Fibonacci ring (word 0, or words 0 and 1 as the
// low and high half of a 64-bit value).
template <int FAM>
__global__ __launch_bounds__(256) void k_rng_init(void *state, int64_t words, int n_rep, int skip, uint64_t a,
                                                  uint64_t c, int r_lag, Key key) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= words * n_rep) return;
    const int rep = (int)(g / words);
    const int64_t w = g - (int64_t)rep * words;
    constexpr uint32_t kTagSeed = 16u;
    if constexpr (FAM == kFamFib) {
        const int64_t q = w / (r_lag + 1), i = w % (r_lag + 1);
        uint32_t v = 0u;  // the last word of a tile: the count n mod r
        if (i < r_lag)
            v = philox4x32_10(make_uint4((uint32_t)(q * r_lag + i), 2u, (uint32_t)rep, kTagSeed), key).x;
        ((uint32_t *)state)[g] = v;
        return;
    }
    uint64_t x;
    if (skip) {
        const uint4 s0 = philox4x32_10(make_uint4(0u, 0u, (uint32_t)rep, kTagSeed), key);
        x = FAM == kFamLcg32 ? (uint64_t)s0.x : (((uint64_t)s0.y << 32) | s0.x);
        // apply f^w: square-and-multiply on the affine map x -> a x + c
        uint64_t pa = a, pc = c;
        for (uint64_t e = (uint64_t)w; e; e >>= 1) {
            if (e & 1u) x = pa * x + pc;
            pc = pa * pc + pc;
            pa = pa * pa;
            if (FAM == kFamLcg32) {
                x &= 0xFFFFFFFFull;
                pa &= 0xFFFFFFFFull;
                pc &= 0xFFFFFFFFull;
            }
        }
    } else {
        const uint4 s1 = philox4x32_10(make_uint4((uint32_t)w, 1u, (uint32_t)rep, kTagSeed), key);
        x = FAM == kFamLcg32 ? (uint64_t)s1.x : (((uint64_t)s1.y << 32) | s1.x);
    }
    if (FAM == kFamLcg32)
        ((uint32_t *)state)[g] = (uint32_t)x;
    else
        ((uint64_t *)state)[g] = x;
}

int family_of(int gen) {
    switch (gen) {
        case SMC_RNG_LCG32:
        case SMC_RNG_LCG32_RANDOM: return kFamLcg32;
        case SMC_RNG_LCG64:
        case SMC_RNG_LCG64_RANDOM: return kFamLcg64;
        default: return kFamFib;
    }
}

// x -> a x + c applied m times, as one affine map (mod 2^32 for LCG32).
void affine_power(int fam, uint64_t a, uint64_t c, uint64_t m, uint64_t *A, uint64_t *C) {
    uint64_t ra = 1, rc = 0, pa = a, pc = c;
    for (; m; m >>= 1) {
        if (m & 1u) {
            rc = pa * rc + pc;
            ra = pa * ra;
        }
        pc = pa * pc + pc;
        pa = pa * pa;
        if (fam == kFamLcg32) {
            ra &= 0xFFFFFFFFull;
            rc &= 0xFFFFFFFFull;
            pa &= 0xFFFFFFFFull;
            pc &= 0xFFFFFFFFull;
        }
    }
    *A = ra;
    *C = rc;
}

}  // namespace

bool rng_study_lags(int gen, int *r, int *s) {
    if (gen == SMC_RNG_FIB521) {
        *r = 521;
        *s = 353;
        return true;
    }
    if (gen == SMC_RNG_FIB1279) {
        *r = 1279;
        *s = 861;
        return true;
    }
    return false;
}

int64_t rng_study_state_bytes(int gen, int L, int T) {
    const int64_t M = (int64_t)L * L / 4, Q = (int64_t)(L / T) * (L / T) / 2;
    int r, s;
    if (gen == SMC_RNG_LCG32 || gen == SMC_RNG_LCG32_RANDOM) return 4 * M;
    if (gen == SMC_RNG_LCG64 || gen == SMC_RNG_LCG64_RANDOM) return 8 * M;
    if (rng_study_lags(gen, &r, &s)) return 4 * Q * (r + 1);
    return 0;
}

static void lcg_constants(int gen, uint64_t *a, uint64_t *c) {
    if (gen == SMC_RNG_LCG32 || gen == SMC_RNG_LCG32_RANDOM) {
        *a = 1664525u;
        *c = 1013904223u;
    } else {
        *a = 2862933555777941757ull;
        *c = 1442695040888963407ull;
    }
}

hipError_t launch_rng_init(int gen, int L, int T, int n_rep, void *state, Key key, hipStream_t s) {
    const int fam = family_of(gen);
    const int64_t words = rng_study_state_bytes(gen, L, T) / (fam == kFamLcg64 ? 8 : 4);
    const int64_t total = words * n_rep;
    int r = 0, sl = 0;
    rng_study_lags(gen, &r, &sl);
    uint64_t a = 0, c = 0;
    lcg_constants(gen, &a, &c);
    const int skip = gen == SMC_RNG_LCG32 || gen == SMC_RNG_LCG64;
    const dim3 grid((unsigned)((total + 255) / 256));
    if (fam == kFamLcg32)
        SMC_LAUNCH(k_rng_init<kFamLcg32>, grid, dim3(256), 0, s, state, words, n_rep, skip, a, c, r, key);
    else if (fam == kFamLcg64)
        SMC_LAUNCH(k_rng_init<kFamLcg64>, grid, dim3(256), 0, s, state, words, n_rep, skip, a, c, r, key);
    else
        SMC_LAUNCH(k_rng_init<kFamFib>, grid, dim3(256), 0, s, state, words, n_rep, skip, a, c, r, key);
    return hipGetLastError();
}

hipError_t launch_dcb_rng(int gen, int8_t *spins, const int8_t *coup, int rep_per_sample, const ThrRow *thr,
                          void *state, int64_t *dE, int n_rep, int L, int T, int k, int tile_colour, hipStream_t s) {
    const int fam = family_of(gen);
    StudyArgs a;
    a.spins = spins;
    a.coup = coup;
    a.rep_per_sample = rep_per_sample;
    a.thr = thr;
    a.state = state;
    a.state_words = rng_study_state_bytes(gen, L, T) / (fam == kFamLcg64 ? 8 : 4);
    a.dE = (unsigned long long *)dE;
    a.L = L;
    a.T = T;
    a.B = L / T;
    a.k = k;
    a.tc = tile_colour;
    a.r_lag = 0;
    a.s_lag = 0;
    rng_study_lags(gen, &a.r_lag, &a.s_lag);
    uint64_t la = 0, lc = 0;
    lcg_constants(gen, &la, &lc);
    const bool skip = gen == SMC_RNG_LCG32 || gen == SMC_RNG_LCG64;
    affine_power(fam, la, lc, skip ? (uint64_t)L * L / 4 : 1u, &a.A, &a.C);
    const int W = T + 2;
    const size_t lds = (size_t)((W * W + 15) & ~15) + (fam == kFamFib ? 4u * (size_t)(a.r_lag + 1) : 0u);
    const dim3 grid((unsigned)((int64_t)n_rep * a.B * a.B / 2)), block((unsigned)(T * T / 2));
    if (fam == kFamLcg32)
        SMC_LAUNCH(k_dcb_rng<kFamLcg32>, grid, block, lds, s, a);
    else if (fam == kFamLcg64)
        SMC_LAUNCH(k_dcb_rng<kFamLcg64>, grid, block, lds, s, a);
    else
        SMC_LAUNCH(k_dcb_rng<kFamFib>, grid, block, lds, s, a);
    return hipGetLastError();
}

}  // namespace smc

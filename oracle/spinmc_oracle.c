/*
 * spinmc_oracle.c -- plain, serial, obviously-correct CPU reference for the
 * checkerboard Metropolis / parallel-tempering hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it; the product library never links, calls or falls back
 * to it.  It shares no code with the HIP sources (its own Philox, indexing,
 * thresholds and energies).
 *
 * Method (M. Weigel, "Performance potential for simulating spin models on
 * GPU", J. Comput. Phys. 231 (2012)):
 *   - Ising Hamiltonian, Sec. 3.1 Eq. (1); Metropolis acceptance Eq. (2) with
 *     Delta E = 2 s_i sum_nn J s_j;
 *   - two-colour checkerboard sweep: all sites of one sub-lattice are
 *     independent and are updated, then the other sub-lattice (Sec. 3.2);
 *   - tabulated Boltzmann factors for discrete energy changes (Sec. 3.5);
 *   - O(n) / Heisenberg Hamiltonian Eq. (10) with uniform re-orientation
 *     proposals (Sec. 4);
 *   - +-J Edwards-Anderson spin glass Eq. (11), bimodal couplings (Sec. 5);
 *   - parallel tempering, exchange probability Eq. (12), temperatures (not
 *     configurations) are exchanged (Sec. 6);
 *   - energies tracked incrementally from accepted flips (Sec. 3.5, Sec. 6).
 *
 * Readings where the paper leaves a choice open (the random-number contract,
 * the sweep order, the threshold arithmetic, the swap schedule) are fixed
 * here and listed in the design notes; each function states the one it uses.
 *
 * Everything is plain loops over sites in storage order.  Floating point is
 * FP64; the file is compiled with -ffp-contract=off so that a*b+c is never
 * fused.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  One round maps (x0,x1,x2,x3) with key (k0,k1): */
/*   (hi0,lo0) = M0*x0,  (hi1,lo1) = M1*x2                                  */
/*   x' = (hi1^x1^k0, lo1, hi0^x3^k1, lo0)                                  */
/* and the key is advanced by the Weyl constants between rounds.            */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

EXPORT void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream tags: counter word 3 is (tag * 2 + colour). */
enum { TAG_INIT = 1, TAG_COUP = 2, TAG_HEAD = 3, TAG_TAIL = 4, TAG_HEIS = 5, TAG_SWAP = 6 };

static void draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* The 32-bit Metropolis uniform of the colour-c site with in-colour index h
 * at sweep t in replica r.  Its high 16 bits are half (h mod 8) of the draw
 * (h/8, t, r, HEAD) (halves numbered low half of word 0 first), its low 16
 * bits are the low half of word 0 of the draw (h, t, r, TAIL). */
EXPORT uint32_t orc_metropolis_u32(uint64_t seed, uint32_t t, uint32_t r, int c, uint64_t h)
{
    uint32_t w[4], v[4];
    draw(seed, (uint32_t)(h >> 3), t, r, (uint32_t)(TAG_HEAD * 2 + c), w);
    uint32_t word = w[(h & 7) >> 1];
    uint32_t head = (h & 1) ? (word >> 16) : (word & 0xFFFFu);
    draw(seed, (uint32_t)h, t, r, (uint32_t)(TAG_TAIL * 2 + c), v);
    uint32_t tail = v[0] & 0xFFFFu;
    return (head << 16) | tail;
}

/* Uniform in (0,1) from the top 23 bits of a word: (k + 1/2) 2^-23.
 * Every such value is exact in binary32 and in binary64. */
static double unit23(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* 53-bit uniform in [0,1) from two words (swap stream). */
static double unit53(uint32_t w0, uint32_t w1)
{
    return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6)) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry.  Periodic simple-cubic lattice of edge L (even), d = 2  */
/* or 3, N = L^d sites in row-major order with x fastest:                    */
/*   2D: i = y L + x;  3D: i = (z L + y) L + x.                              */
/* Colour c(i) = (x + y [+ z]) mod 2; the in-colour index h(i) = i / 2       */
/* (equal to (row index) * L/2 + x/2 because L is even).                     */
/* ------------------------------------------------------------------------ */
static void coords(int dim, int L, int64_t i, int x[3])
{
    x[0] = (int)(i % L);
    x[1] = (int)((i / L) % L);
    x[2] = dim == 3 ? (int)(i / ((int64_t)L * L)) : 0;
}

static int64_t index_of(int dim, int L, const int x[3])
{
    int64_t i = x[0] + (int64_t)L * x[1];
    if (dim == 3) i += (int64_t)L * L * x[2];
    return i;
}

static int colour_of(int dim, const int x[3])
{
    int s = x[0] + x[1] + (dim == 3 ? x[2] : 0);
    return s & 1;
}

/* Neighbour of site x in direction mu, step +1 or -1, periodic. */
static int64_t neighbour(int dim, int L, const int x[3], int mu, int step)
{
    int y[3] = {x[0], x[1], x[2]};
    y[mu] = (y[mu] + step + L) % L;
    return index_of(dim, L, y);
}

static int64_t n_sites(int dim, int L)
{
    return dim == 3 ? (int64_t)L * L * L : (int64_t)L * L;
}

/* ------------------------------------------------------------------------ */
/* Initial state.                                                            */
/* ------------------------------------------------------------------------ */

/* Random start for Ising / EA spins of replica r: site i takes word (i mod 4)
 * of the draw (i/4, 0, r, INIT); the spin is +1 iff that word's top bit is 0. */
EXPORT void orc_init_spins(int dim, int L, uint64_t seed, uint32_t r, int8_t *s)
{
    int64_t N = n_sites(dim, L);
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w[4];
        draw(seed, (uint32_t)(i >> 2), 0, r, TAG_INIT * 2, w);
        s[i] = (w[i & 3] >> 31) ? -1 : +1;
    }
}

/* Bimodal couplings of disorder sample q (Sec. 5: J = +-1 with probability
 * 1/2 each).  Bond (i, mu) joins i and i + e_mu; its draw is word (b mod 4)
 * of (b/4, 0, q, COUP) with b = i d + mu; J = +1 iff the top bit is 0.
 * Storage J[mu * N + i]. */
EXPORT void orc_init_couplings(int dim, int L, uint64_t seed, uint32_t q, int8_t *J)
{
    int64_t N = n_sites(dim, L);
    for (int64_t i = 0; i < N; ++i) {
        for (int mu = 0; mu < dim; ++mu) {
            uint64_t b = (uint64_t)i * dim + mu;
            uint32_t w[4];
            draw(seed, (uint32_t)(b >> 2), 0, q, TAG_COUP * 2, w);
            J[(int64_t)mu * N + i] = (w[b & 3] >> 31) ? -1 : +1;
        }
    }
}

/* Uniform point on the unit sphere from two uniforms (Archimedes: z is
 * uniform on [-1,1], the azimuth uniform on [0, 2 pi)). */
static void sphere_point(double u0, double u1, double out[3])
{
    double z = 2.0 * u0 - 1.0;
    double phi = TWO_PI * u1;
    double rho = sqrt(1.0 - z * z);
    out[0] = rho * cos(phi);
    out[1] = rho * sin(phi);
    out[2] = z;
}

/* Random start for Heisenberg spins of replica r: words 0, 1 of (i, 0, r, INIT). */
EXPORT void orc_init_heis(int dim, int L, uint64_t seed, uint32_t r, double *s)
{
    int64_t N = n_sites(dim, L);
    for (int64_t i = 0; i < N; ++i) {
        uint32_t w[4];
        draw(seed, (uint32_t)i, 0, r, TAG_INIT * 2, w);
        sphere_point(unit23(w[0]), unit23(w[1]), &s[3 * i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds for discrete energy changes Delta E = 4m > 0        */
/* (Sec. 3.5: tabulate exp(-beta Delta E)).  thr[m] = floor(2^32 e^{-4 m b}) */
/* in FP64 with libm exp; a flip with Delta E = 4m > 0 is accepted iff the   */
/* 32-bit uniform u satisfies u < thr[m]; thr[m] = 2^32 means always.        */
/* ------------------------------------------------------------------------ */
EXPORT void orc_thresholds(double beta, int dim, uint64_t *thr /* [dim+1] */)
{
    thr[0] = 4294967296ull;
    for (int m = 1; m <= dim; ++m) {
        double p = exp(-beta * (4.0 * m));
        double v = floor(4294967296.0 * p);
        thr[m] = (uint64_t)v;
    }
}

/* Local field h_i = sum_mu [ J(i,mu) s(i+e_mu) + J(i-e_mu,mu) s(i-e_mu) ]
 * (J == NULL: ferromagnet, all couplings +1). */
static int local_field(int dim, int L, const int8_t *J, const int8_t *s, int64_t i)
{
    int64_t N = n_sites(dim, L);
    int x[3];
    coords(dim, L, i, x);
    int h = 0;
    for (int mu = 0; mu < dim; ++mu) {
        int64_t up = neighbour(dim, L, x, mu, +1);
        int64_t dn = neighbour(dim, L, x, mu, -1);
        int j_up = J ? J[(int64_t)mu * N + i] : 1;
        int j_dn = J ? J[(int64_t)mu * N + dn] : 1;
        h += j_up * s[up] + j_dn * s[dn];
    }
    return h;
}

/* One half-sweep: a Metropolis attempt (Eq. 2) at every site of colour c.
 * Sites of one colour only neighbour sites of the other colour, so their
 * updates are independent and the visiting order is irrelevant.
 * Returns the sum of Delta E over accepted flips. */
EXPORT int64_t orc_half_sweep(int dim, int L, const int8_t *J, int8_t *s, double beta,
                              uint64_t seed, uint32_t r, uint32_t t, int c)
{
    uint64_t thr[4];
    orc_thresholds(beta, dim, thr);
    int64_t N = n_sites(dim, L);
    int64_t dE_sum = 0;
    for (int64_t i = 0; i < N; ++i) {
        int x[3];
        coords(dim, L, i, x);
        if (colour_of(dim, x) != c) continue;
        int h = local_field(dim, L, J, s, i);
        int dE = 2 * s[i] * h;
        int accept;
        if (dE <= 0) {
            accept = 1;
        } else {
            uint32_t u = orc_metropolis_u32(seed, t, r, c, (uint64_t)(i >> 1));
            accept = (uint64_t)u < thr[dE / 4];
        }
        if (accept) {
            s[i] = (int8_t)(-s[i]);
            dE_sum += dE;
        }
    }
    return dE_sum;
}

/* Sweep t: colour 0, then colour 1. */
EXPORT int64_t orc_sweep(int dim, int L, const int8_t *J, int8_t *s, double beta,
                         uint64_t seed, uint32_t r, uint32_t t)
{
    int64_t dE = orc_half_sweep(dim, L, J, s, beta, seed, r, t, 0);
    dE += orc_half_sweep(dim, L, J, s, beta, seed, r, t, 1);
    return dE;
}

/* n sweeps t0 .. t0+n-1. */
EXPORT int64_t orc_run(int dim, int L, const int8_t *J, int8_t *s, double beta,
                       uint64_t seed, uint32_t r, uint32_t t0, int n)
{
    int64_t dE = 0;
    for (int k = 0; k < n; ++k) dE += orc_sweep(dim, L, J, s, beta, seed, r, t0 + (uint32_t)k);
    return dE;
}

/* Double checkerboard sweeps with multi-hit updates of a 2D lattice
 * (Sec. 3.2 steps 1-7; Sec. 3.4 for k hits and the palindromic order).
 * The lattice of edge L is cut into T x T tiles, B = L / T per direction
 * (B even, or B = 1); tile (bx, by) has tile colour (bx + by) & 1.  Sweep t
 * treats the tiles of tile colour 0, then those of tile colour 1; each tile
 * gets k hits, a hit being a Metropolis attempt (Eq. 2) at every colour-0
 * site of the tile followed by one at every colour-1 site, with the
 * neighbours outside the tile (tiles of the other tile colour) held fixed.
 * Tiles of one tile colour share no bond, so their order is irrelevant.
 * With palindromic != 0, odd sweeps run both orders backwards (tile colour
 * 1 first, colour-1 sites first), so that two consecutive sweeps form a
 * palindrome of single-colour updates.  Hit j of sweep t draws the uniform
 * of "sweep" t*k + j of the plain checkerboard (orc_metropolis_u32); with
 * T = L and k = 1 the sweep is exactly orc_sweep.  Returns the summed
 * Delta E of accepted flips. */
EXPORT int64_t orc_dcb_run(int L, int T, int k, const int8_t *J, int8_t *s, double beta, uint64_t seed,
                           uint32_t r, uint32_t t0, int n, int palindromic)
{
    uint64_t thr[4];
    orc_thresholds(beta, 2, thr);
    const int B = L / T;
    int64_t dE_sum = 0;
    for (int m = 0; m < n; ++m) {
        const uint32_t t = t0 + (uint32_t)m;
        const int rev = palindromic && (t & 1u);
        for (int ci = 0; ci < 2; ++ci) {
            const int tile_colour = rev ? 1 - ci : ci;
            for (int by = 0; by < B; ++by) {
                for (int bx = 0; bx < B; ++bx) {
                    if (((bx + by) & 1) != tile_colour) continue;
                    for (int j = 0; j < k; ++j) {
                        const uint32_t th = t * (uint32_t)k + (uint32_t)j;
                        for (int si = 0; si < 2; ++si) {
                            const int c = rev ? 1 - si : si;
                            for (int v = 0; v < T; ++v) {
                                for (int u = 0; u < T; ++u) {
                                    const int x = bx * T + u, y = by * T + v;
                                    if (((x + y) & 1) != c) continue;
                                    const int64_t i = (int64_t)y * L + x;
                                    const int h = local_field(2, L, J, s, i);
                                    const int dE = 2 * s[i] * h;
                                    int accept = 1;
                                    if (dE > 0) {
                                        uint32_t uu = orc_metropolis_u32(seed, th, r, c, (uint64_t)(i >> 1));
                                        accept = (uint64_t)uu < thr[dE / 4];
                                    }
                                    if (accept) {
                                        s[i] = (int8_t)(-s[i]);
                                        dE_sum += dE;
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    return dE_sum;
}

/* ------------------------------------------------------------------------ */
/* The generators of the paper's random-number study (Sec. 3.3, Table 1),    */
/* driving the double checkerboard of orc_dcb_run (tile colour 0 then 1, k   */
/* hits, colour 0 then colour 1 sites, no palindrome):                       */
/*   LCG32: x' = (1664525 x + 1013904223) mod 2^32 (Eq. 3, m = 2^32);        */
/*   LCG64: x' = (2862933555777941757 x + 1442695040888963407) mod 2^64,     */
/*          the uniform being its top 32 bits;                               */
/*   lagged Fibonacci: x_n = x_{n-r} + x_{n-s} mod 2^32 (Eq. 6 with unit     */
/*          multipliers, i.e. Eq. 7 on 32-bit fixed point), (r, s) =         */
/*          (521, 353) or (1279, 861).                                       */
/* Streams.  With tiles of edge T (B = L / T per direction), the tiles of one */
/* tile colour are numbered q = by (B/2) + bx/2 and the colour-c sites of a  */
/* tile p = v (T/2) + u/2 (site (u, v) of the tile), so that (q, p) runs     */
/* over L^2/4 positions, the threads of the paper's GPU code.  An LCG stream */
/* j = q T^2/2 + p serves position (q, p) of both tile colours and both site */
/* colours, one number per attempt, in the order of the sweep: per sweep     */
/* tile colour 0 (k hits, each colour 0 then 1), then tile colour 1.  With   */
/* skip-ahead (Eqs. 4, 5) stream j delivers x_j, x_{j+M}, x_{j+2M}, ... of   */
/* one global sequence (M = L^2/4 streams); the "random" variants instead   */
/* start each stream at an independent seed and step it by Eq. 3 itself.     */
/* A lagged-Fibonacci generator serves tile q (both tile colours): each      */
/* round of a tile (one colour of one hit) consumes T^2/2 consecutive        */
/* numbers, position p taking the p-th.  Every attempt consumes its number,  */
/* also when Delta E <= 0 accepts without it.                                */
/* Seeds come from Philox draws with counter word 3 = 16: the start x_0 of   */
/* the global sequence of replica r from (0, 0, r, 16) (word 0, LCG64: words */
/* 0 and 1 as low and high half), stream j's seed from (j, 1, r, 16), word   */
/* i of Fibonacci generator q's initial ring from word 0 of                  */
/* (q r_lag + i, 2, r, 16).                                                  */
/* ------------------------------------------------------------------------ */
enum { GEN_LCG32 = 1, GEN_LCG32_RANDOM = 2, GEN_LCG64 = 3, GEN_LCG64_RANDOM = 4, GEN_FIB521 = 5, GEN_FIB1279 = 6 };
static const uint32_t LCG32_A = 1664525u, LCG32_C = 1013904223u;
static const uint64_t LCG64_A = 2862933555777941757ull, LCG64_C = 1442695040888963407ull;
enum { TAG_GEN = 8 };

static int fib_lags(int gen, int *r, int *s)
{
    if (gen == GEN_FIB521) { *r = 521; *s = 353; return 1; }
    if (gen == GEN_FIB1279) { *r = 1279; *s = 861; return 1; }
    return 0;
}

/* uint64 words of the state of one replica: the M stream values (LCG), or
 * per tile q its r ring words followed by the count n mod r (Fibonacci);
 * 0 for an unknown generator. */
EXPORT int64_t orc_rng_state_words(int gen, int L, int T)
{
    int64_t M = (int64_t)L * L / 4, Q = (int64_t)(L / T) * (L / T) / 2;
    int r, sl;
    if (gen >= GEN_LCG32 && gen <= GEN_LCG64_RANDOM) return M;
    if (fib_lags(gen, &r, &sl)) return Q * (r + 1);
    return 0;
}

EXPORT void orc_rng_init(int gen, int L, int T, uint64_t seed, uint32_t rep, uint64_t *state)
{
    int64_t M = (int64_t)L * L / 4, Q = (int64_t)(L / T) * (L / T) / 2;
    uint32_t w[4];
    int r, sl;
    if (gen == GEN_LCG32 || gen == GEN_LCG64) {
        /* x_0 .. x_{M-1} of the global sequence, by plain iteration */
        draw(seed, 0, 0, rep, TAG_GEN * 2, w);
        uint64_t x = gen == GEN_LCG32 ? (uint64_t)w[0] : ((uint64_t)w[1] << 32 | w[0]);
        for (int64_t j = 0; j < M; ++j) {
            state[j] = x;
            x = gen == GEN_LCG32 ? (uint64_t)(uint32_t)(LCG32_A * (uint32_t)x + LCG32_C) : LCG64_A * x + LCG64_C;
        }
    } else if (gen == GEN_LCG32_RANDOM || gen == GEN_LCG64_RANDOM) {
        for (int64_t j = 0; j < M; ++j) {
            draw(seed, (uint32_t)j, 1, rep, TAG_GEN * 2, w);
            state[j] = gen == GEN_LCG32_RANDOM ? (uint64_t)w[0] : ((uint64_t)w[1] << 32 | w[0]);
        }
    } else if (fib_lags(gen, &r, &sl)) {
        for (int64_t q = 0; q < Q; ++q) {
            for (int i = 0; i < r; ++i) {
                draw(seed, (uint32_t)(q * r + i), 2, rep, TAG_GEN * 2, w);
                state[q * (r + 1) + i] = w[0];
            }
            state[q * (r + 1) + r] = 0;  /* x_n is written to ring word n mod r */
        }
    }
}

/* The step that moves a skip-ahead stream on by M numbers of the global
 * sequence, x -> A x + C, composed from M plain steps (Eqs. 4, 5). */
static void lcg_power(int gen, int64_t M, uint64_t *A, uint64_t *C)
{
    uint64_t a = 1, c = 0;
    for (int64_t i = 0; i < M; ++i) {
        if (gen == GEN_LCG32) {
            a = (uint32_t)(LCG32_A * (uint32_t)a);
            c = (uint32_t)(LCG32_A * (uint32_t)c + LCG32_C);
        } else {
            a = LCG64_A * a;
            c = LCG64_A * c + LCG64_C;
        }
    }
    *A = a;
    *C = c;
}

/* n double-checkerboard sweeps of a 2D Ising / EA lattice with the
 * uniforms taken from the study's generators (layout above); the state
 * advances.  Tiles T x T with B = L / T even; the Fibonacci generators need
 * T^2/2 <= min(s, r - s) (a round then reads no number of its own round).
 * Returns the summed Delta E of accepted flips. */
EXPORT int64_t orc_dcb_run_rng(int L, int T, int k, const int8_t *J, int8_t *s, double beta, int gen,
                               uint64_t *state, int n)
{
    uint64_t thr[4];
    orc_thresholds(beta, 2, thr);
    const int B = L / T, P = T * T / 2;
    const int64_t M = (int64_t)L * L / 4;
    uint64_t A = 1, C = 0;
    int r = 0, sl = 0;
    const int fib = fib_lags(gen, &r, &sl);
    if (gen == GEN_LCG32 || gen == GEN_LCG64) lcg_power(gen, M, &A, &C);
    if (gen == GEN_LCG32_RANDOM) { A = LCG32_A; C = LCG32_C; }
    if (gen == GEN_LCG64_RANDOM) { A = LCG64_A; C = LCG64_C; }
    int64_t dE_sum = 0;
    for (int m = 0; m < n; ++m) {
        for (int tile_colour = 0; tile_colour < 2; ++tile_colour) {
            for (int by = 0; by < B; ++by) {
                for (int bx = 0; bx < B; ++bx) {
                    if (((bx + by) & 1) != tile_colour) continue;
                    const int64_t q = (int64_t)by * (B / 2) + bx / 2;
                    for (int j = 0; j < k; ++j) {
                        for (int c = 0; c < 2; ++c) {
                            for (int v = 0; v < T; ++v) {
                                for (int u = 0; u < T; ++u) {
                                    const int x = bx * T + u, y = by * T + v;
                                    if (((x + y) & 1) != c) continue;
                                    const int64_t p = (int64_t)v * (T / 2) + u / 2;
                                    uint32_t uu;
                                    if (fib) {
                                        uint64_t *ring = state + q * (r + 1);
                                        const uint64_t nn = ring[r];
                                        const uint64_t back = (nn + (uint64_t)r - (uint64_t)sl) % (uint64_t)r;
                                        uu = (uint32_t)(ring[nn] + ring[back]);
                                        ring[nn] = uu;
                                        ring[r] = (nn + 1) % (uint64_t)r;
                                    } else {
                                        uint64_t *xs = &state[q * P + p];
                                        uu = (gen == GEN_LCG32 || gen == GEN_LCG32_RANDOM) ? (uint32_t)*xs
                                                                                            : (uint32_t)(*xs >> 32);
                                        *xs = (gen == GEN_LCG32 || gen == GEN_LCG32_RANDOM)
                                                  ? (uint64_t)(uint32_t)((uint32_t)A * (uint32_t)*xs + (uint32_t)C)
                                                  : A * *xs + C;
                                    }
                                    const int64_t i = (int64_t)y * L + x;
                                    const int h = local_field(2, L, J, s, i);
                                    const int dE = 2 * s[i] * h;
                                    const int accept = dE <= 0 || (uint64_t)uu < thr[dE / 4];
                                    if (accept) {
                                        s[i] = (int8_t)(-s[i]);
                                        dE_sum += dE;
                                    }
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    return dE_sum;
}

/* The same in three dimensions (the paper carries the tiled update over to
 * 3D): T x T x T tiles, tile colour (bx + by + bz) & 1, tile colour 0 first,
 * colour-0 sites (x + y + z even) of a tile before its colour-1 sites, the
 * sites outside the tile held fixed; hit j of sweep t draws as plain sweep
 * t*k + j, so T = L and k = 1 is orc_sweep in 3D. */
EXPORT int64_t orc_dcb_run3(int L, int T, int k, const int8_t *J, int8_t *s, double beta, uint64_t seed,
                            uint32_t r, uint32_t t0, int n, int palindromic)
{
    uint64_t thr[4];
    orc_thresholds(beta, 3, thr);
    const int B = L / T;
    int64_t dE_sum = 0;
    for (int m = 0; m < n; ++m) {
        const uint32_t t = t0 + (uint32_t)m;
        const int rev = palindromic && (t & 1u);
        for (int ci = 0; ci < 2; ++ci) {
            const int tile_colour = rev ? 1 - ci : ci;
            for (int bz = 0; bz < B; ++bz)
                for (int by = 0; by < B; ++by)
                    for (int bx = 0; bx < B; ++bx) {
                        if (((bx + by + bz) & 1) != tile_colour) continue;
                        for (int j = 0; j < k; ++j) {
                            const uint32_t th = t * (uint32_t)k + (uint32_t)j;
                            for (int si = 0; si < 2; ++si) {
                                const int c = rev ? 1 - si : si;
                                for (int w = 0; w < T; ++w)
                                    for (int v = 0; v < T; ++v)
                                        for (int u = 0; u < T; ++u) {
                                            const int x = bx * T + u, y = by * T + v, z = bz * T + w;
                                            if (((x + y + z) & 1) != c) continue;
                                            const int64_t i = ((int64_t)z * L + y) * L + x;
                                            const int h = local_field(3, L, J, s, i);
                                            const int dE = 2 * s[i] * h;
                                            int accept = 1;
                                            if (dE > 0) {
                                                uint32_t uu = orc_metropolis_u32(seed, th, r, c, (uint64_t)(i >> 1));
                                                accept = (uint64_t)uu < thr[dE / 4];
                                            }
                                            if (accept) {
                                                s[i] = (int8_t)(-s[i]);
                                                dE_sum += dE;
                                            }
                                        }
                            }
                        }
                    }
        }
    }
    return dE_sum;
}

/* n sweeps t0 .. t0+n-1 of a W x W window of a 2D Ising lattice of edge L
 * (no couplings), for checking sampled sites of lattices too large to sweep
 * here.  win[v*W + u] is the site (x0 + u, y0 + v) mod L; every interior
 * window site is updated exactly as in orc_sweep (same colour order, same
 * uniform keyed by the site's index in the whole lattice), the outermost ring
 * of the window is held fixed.  A wrong value can only enter from that ring
 * and moves at most two sites per sweep (colour 0 then colour 1), so after
 * n sweeps every site at distance > 2n from the ring equals the full
 * lattice's. */
EXPORT void orc_window_run(int L, int W, int x0, int y0, int8_t *win, double beta, uint64_t seed,
                           uint32_t r, uint32_t t0, int n)
{
    uint64_t thr[4];
    orc_thresholds(beta, 2, thr);
    for (int k = 0; k < n; ++k) {
        uint32_t t = t0 + (uint32_t)k;
        for (int c = 0; c < 2; ++c) {
            for (int v = 1; v < W - 1; ++v) {
                for (int u = 1; u < W - 1; ++u) {
                    int gx = (x0 + u) % L, gy = (y0 + v) % L;
                    if (((gx + gy) & 1) != c) continue;
                    int8_t *si = &win[v * W + u];
                    int h = win[v * W + u + 1] + win[v * W + u - 1] + win[(v + 1) * W + u] + win[(v - 1) * W + u];
                    int dE = 2 * (*si) * h;
                    int accept = 1;
                    if (dE > 0) {
                        int64_t i = (int64_t)gy * L + gx;
                        uint32_t uu = orc_metropolis_u32(seed, t, r, c, (uint64_t)(i >> 1));
                        accept = (uint64_t)uu < thr[dE / 4];
                    }
                    if (accept) *si = (int8_t)(-(*si));
                }
            }
        }
    }
}

/* E = -sum_i sum_mu J(i,mu) s_i s_{i+e_mu} (Eqs. 1 and 11), each bond once. */
EXPORT int64_t orc_energy(int dim, int L, const int8_t *J, const int8_t *s)
{
    int64_t N = n_sites(dim, L);
    int64_t E = 0;
    for (int64_t i = 0; i < N; ++i) {
        int x[3];
        coords(dim, L, i, x);
        for (int mu = 0; mu < dim; ++mu) {
            int64_t up = neighbour(dim, L, x, mu, +1);
            int j = J ? J[(int64_t)mu * N + i] : 1;
            E -= (int64_t)j * s[i] * s[up];
        }
    }
    return E;
}

EXPORT int64_t orc_magnetisation(int dim, int L, const int8_t *s)
{
    int64_t N = n_sites(dim, L);
    int64_t M = 0;
    for (int64_t i = 0; i < N; ++i) M += s[i];
    return M;
}

/* n sweeps t0 .. t0+n-1 recording E and M after every sweep (for the
 * statistical checks against exact results). */
EXPORT void orc_run_series(int dim, int L, const int8_t *J, int8_t *s, double beta,
                           uint64_t seed, uint32_t r, uint32_t t0, int n,
                           int64_t *E_series, int64_t *M_series)
{
    for (int k = 0; k < n; ++k) {
        orc_sweep(dim, L, J, s, beta, seed, r, t0 + (uint32_t)k);
        E_series[k] = orc_energy(dim, L, J, s);
        M_series[k] = orc_magnetisation(dim, L, s);
    }
}

/* ------------------------------------------------------------------------ */
/* Heisenberg (O(3)) model, Eq. (10), FP64.                                  */
/* ------------------------------------------------------------------------ */

/* Small-step proposal (Sec. 4 suggests small changes instead of uniform
 * re-orientations for low temperatures): s' uniform on the spherical cap
 * {s' : 1 - a.s' <= cap} around a = s/|s|, cap in (0, 2], so that the
 * proposal density is symmetric in s and s'.  From two uniforms: w = cap u0,
 * the cosine of the angle 1 - w, the radius sqrt(w (2 - w)), the azimuth
 * 2 pi u1 in the frame (e1, e2): e1 a unit vector perpendicular to a (in the
 * x-y plane when |a_x| > |a_z|, else in the y-z plane), e2 = a x e1. */
static void cap_point(const double *s, double cap, double u0, double u1, double out[3])
{
    double n = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    double a[3] = {s[0] / n, s[1] / n, s[2] / n};
    double e1[3];
    if (fabs(a[0]) > fabs(a[2])) {
        double m = sqrt(a[0] * a[0] + a[1] * a[1]);
        e1[0] = -a[1] / m;
        e1[1] = a[0] / m;
        e1[2] = 0.0;
    } else {
        double m = sqrt(a[1] * a[1] + a[2] * a[2]);
        e1[0] = 0.0;
        e1[1] = -a[2] / m;
        e1[2] = a[1] / m;
    }
    double e2[3] = {a[1] * e1[2] - a[2] * e1[1], a[2] * e1[0] - a[0] * e1[2], a[0] * e1[1] - a[1] * e1[0]};
    double w = cap * u0;
    double zc = 1.0 - w;
    double rc = sqrt(w * (2.0 - w));
    double phi = TWO_PI * u1;
    double cs = cos(phi), sn = sin(phi);
    for (int k = 0; k < 3; ++k) out[k] = zc * a[k] + rc * (cs * e1[k] + sn * e2[k]);
}

/* The Metropolis move at site i of colour c in sweep t: propose a fresh
 * uniform direction s' (independent of s, Sec. 4; cap == 0) or a point of
 * the cap of size cap around s (0 < cap <= 2) from words 0, 1 of
 * (i >> 1, t, r, HEIS+c) and accept iff Delta E = -(s' - s).h <= 0 or
 * u < exp(-beta Delta E), u from word 2.  Returns 1 if accepted. */
static int heis_site_move_gap(int dim, int L, double *s, double beta, uint64_t seed, uint32_t r, uint32_t t, int c,
                              int64_t i, double cap, double *gap)
{
    int x[3];
    coords(dim, L, i, x);
    double h[3] = {0.0, 0.0, 0.0};
    for (int mu = 0; mu < dim; ++mu) {
        int64_t up = neighbour(dim, L, x, mu, +1);
        int64_t dn = neighbour(dim, L, x, mu, -1);
        for (int a = 0; a < 3; ++a) h[a] += s[3 * up + a] + s[3 * dn + a];
    }
    uint32_t w[4];
    draw(seed, (uint32_t)(i >> 1), t, r, (uint32_t)(TAG_HEIS * 2 + c), w);
    double sp[3];
    if (cap > 0.0)
        cap_point(&s[3 * i], cap, unit23(w[0]), unit23(w[1]), sp);
    else
        sphere_point(unit23(w[0]), unit23(w[1]), sp);
    double dE = 0.0;
    for (int a = 0; a < 3; ++a) dE -= (sp[a] - s[3 * i + a]) * h[a];
    int accept = (dE <= 0.0) || (unit23(w[2]) < exp(-beta * dE));
    if (gap) *gap = dE <= 0.0 ? INFINITY : unit23(w[2]) - exp(-beta * dE);
    if (accept)
        for (int a = 0; a < 3; ++a) s[3 * i + a] = sp[a];
    return accept;
}

static int heis_site_move_cap(int dim, int L, double *s, double beta, uint64_t seed, uint32_t r, uint32_t t, int c,
                              int64_t i, double cap)
{
    return heis_site_move_gap(dim, L, s, beta, seed, r, t, c, i, cap, NULL);
}

static int heis_site_move(int dim, int L, double *s, double beta, uint64_t seed, uint32_t r, uint32_t t, int c,
                          int64_t i)
{
    return heis_site_move_cap(dim, L, s, beta, seed, r, t, c, i, 0.0);
}

/* One half-sweep of colour c: the move above at every site of colour c.
 * Returns the number of accepted moves. */
EXPORT int64_t orc_heis_half_sweep(int dim, int L, double *s, double beta,
                                   uint64_t seed, uint32_t r, uint32_t t, int c)
{
    int64_t N = n_sites(dim, L);
    int64_t n_acc = 0;
    for (int64_t i = 0; i < N; ++i) {
        int x[3];
        coords(dim, L, i, x);
        if (colour_of(dim, x) != c) continue;
        n_acc += heis_site_move(dim, L, s, beta, seed, r, t, c, i);
    }
    return n_acc;
}

/* orc_heis_half_sweep that also reports, for every site i of colour c, the
 * margin of its acceptance test: gap[i] = u - exp(-beta Delta E), or +inf
 * where Delta E <= 0 decides alone (other entries untouched).  An
 * implementation that evaluates the move in lower precision can only take
 * the other decision where |gap| lies within its rounding (test
 * infrastructure: the same moves as orc_heis_half_sweep). */
EXPORT int64_t orc_heis_half_sweep_gaps(int dim, int L, double *s, double beta, uint64_t seed, uint32_t r,
                                        uint32_t t, int c, double *gap)
{
    int64_t N = n_sites(dim, L);
    int64_t n_acc = 0;
    for (int64_t i = 0; i < N; ++i) {
        int x[3];
        coords(dim, L, i, x);
        if (colour_of(dim, x) != c) continue;
        n_acc += heis_site_move_gap(dim, L, s, beta, seed, r, t, c, i, 0.0, &gap[i]);
    }
    return n_acc;
}

EXPORT void orc_heis_renormalise(int dim, int L, double *s)
{
    int64_t N = n_sites(dim, L);
    for (int64_t i = 0; i < N; ++i) {
        double n = sqrt(s[3 * i] * s[3 * i] + s[3 * i + 1] * s[3 * i + 1] + s[3 * i + 2] * s[3 * i + 2]);
        for (int a = 0; a < 3; ++a) s[3 * i + a] /= n;
    }
}

/* Sweep t (colour 0 then colour 1); spins are renormalised after the sweep
 * when renorm_every > 0 and (t + 1) is a multiple of renorm_every. */
EXPORT int64_t orc_heis_sweep(int dim, int L, double *s, double beta, uint64_t seed,
                              uint32_t r, uint32_t t, int renorm_every)
{
    int64_t n = orc_heis_half_sweep(dim, L, s, beta, seed, r, t, 0);
    n += orc_heis_half_sweep(dim, L, s, beta, seed, r, t, 1);
    if (renorm_every > 0 && ((uint64_t)t + 1) % (uint64_t)renorm_every == 0)
        orc_heis_renormalise(dim, L, s);
    return n;
}

EXPORT int64_t orc_heis_run(int dim, int L, double *s, double beta, uint64_t seed,
                            uint32_t r, uint32_t t0, int n, int renorm_every)
{
    int64_t acc = 0;
    for (int k = 0; k < n; ++k) acc += orc_heis_sweep(dim, L, s, beta, seed, r, t0 + (uint32_t)k, renorm_every);
    return acc;
}

/* Double checkerboard with multi-hit updates (Sec. 3.2, Sec. 3.4) for the
 * 2D Heisenberg model, in the order of orc_dcb_run: sweep t treats the
 * tiles of tile colour 0, then those of colour 1 (both reversed on odd
 * sweeps when palindromic != 0); a tile gets k hits, each a move at every
 * colour-0 site of the tile, then at every colour-1 site, the spins outside
 * the tile held fixed.  Hit j of sweep t draws as plain sweep t*k + j, so
 * T = L, k = 1 and cap = 0 is orc_heis_sweep.  cap > 0 takes the small-step
 * proposal of heis_site_move_cap.  Spins are renormalised after sweep t
 * when renorm_every > 0 and (t + 1) is a multiple of it.  Returns the
 * number of accepted moves. */
EXPORT int64_t orc_heis_dcb_run(int L, int T, int k, double *s, double beta, uint64_t seed, uint32_t r,
                                uint32_t t0, int n, int palindromic, int renorm_every, double cap)
{
    const int B = L / T;
    int64_t n_acc = 0;
    for (int m = 0; m < n; ++m) {
        const uint32_t t = t0 + (uint32_t)m;
        const int rev = palindromic && (t & 1u);
        for (int ci = 0; ci < 2; ++ci) {
            const int tile_colour = rev ? 1 - ci : ci;
            for (int by = 0; by < B; ++by) {
                for (int bx = 0; bx < B; ++bx) {
                    if (((bx + by) & 1) != tile_colour) continue;
                    for (int j = 0; j < k; ++j) {
                        const uint32_t th = t * (uint32_t)k + (uint32_t)j;
                        for (int si = 0; si < 2; ++si) {
                            const int c = rev ? 1 - si : si;
                            for (int v = 0; v < T; ++v) {
                                for (int u = 0; u < T; ++u) {
                                    const int x = bx * T + u, y = by * T + v;
                                    if (((x + y) & 1) != c) continue;
                                    n_acc += heis_site_move_cap(2, L, s, beta, seed, r, th, c,
                                                                (int64_t)y * L + x, cap);
                                }
                            }
                        }
                    }
                }
            }
        }
        if (renorm_every > 0 && ((uint64_t)t + 1) % (uint64_t)renorm_every == 0) orc_heis_renormalise(2, L, s);
    }
    return n_acc;
}

/* Kahan-compensated FP64 sums of E = -sum_bonds s_i . s_j and of M. */
EXPORT double orc_heis_energy(int dim, int L, const double *s)
{
    int64_t N = n_sites(dim, L);
    double sum = 0.0, comp = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        int x[3];
        coords(dim, L, i, x);
        for (int mu = 0; mu < dim; ++mu) {
            int64_t up = neighbour(dim, L, x, mu, +1);
            double term = -(s[3 * i] * s[3 * up] + s[3 * i + 1] * s[3 * up + 1] + s[3 * i + 2] * s[3 * up + 2]);
            double y = term - comp;
            double tt = sum + y;
            comp = (tt - sum) - y;
            sum = tt;
        }
    }
    return sum;
}

EXPORT void orc_heis_magnetisation(int dim, int L, const double *s, double m[3])
{
    int64_t N = n_sites(dim, L);
    for (int a = 0; a < 3; ++a) {
        double sum = 0.0, comp = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double y = s[3 * i + a] - comp;
            double tt = sum + y;
            comp = (tt - sum) - y;
            sum = tt;
        }
        m[a] = sum;
    }
}

/* ------------------------------------------------------------------------ */
/* Parallel tempering (Sec. 6).                                              */
/* A chain q holds n_temps replicas (storage slots 0..n_temps-1, replica     */
/* index r = r0 + slot) that share the couplings J.  slot_of_temp[k] is the  */
/* slot currently simulated at inverse temperature beta[k]; beta[0] is the   */
/* coldest end of the ladder by convention.  E[slot] is the energy of the    */
/* configuration in that slot.                                               */
/*                                                                           */
/* Step t: m sweeps (indices t*m .. t*m + m - 1; Sec. 6 attempts exchanges  */
/* once per m sweeps) of every slot at its current temperature, tracking E;  */
/* then for every k with k = t (mod 2), k <= n_temps - 2, the                */
/* exchange of temperatures k and k+1 is attempted with Eq. (12):            */
/*   x = (beta[k+1] - beta[k]) (E[B] - E[A]),  A = slot at k, B = at k+1,    */
/*   accept iff x >= 0 or u < exp(x), u the 53-bit uniform of (k, t, q, SWAP)*/
/* and on acceptance the two slots exchange temperatures.                    */
/* ------------------------------------------------------------------------ */
/* Near-tie audit of the exchange decisions (test infrastructure): the
 * device evaluates exp(x) with its own float64 exp, which may differ from
 * libm by an ulp, so a decision is only shared when u is not within such a
 * distance of exp(x).  Every attempt with x < 0 is counted, with those whose
 * |u - exp(x)| < 2^-40 and the smallest gap seen.  Not thread-safe. */
static uint64_t audit_attempts = 0, audit_near_ties = 0;
static double audit_min_gap = 1.0;

EXPORT void orc_pt_audit(uint64_t counts[2], double *min_gap, int reset)
{
    counts[0] = audit_attempts;
    counts[1] = audit_near_ties;
    *min_gap = audit_min_gap;
    if (reset) {
        audit_attempts = 0;
        audit_near_ties = 0;
        audit_min_gap = 1.0;
    }
}

EXPORT void orc_pt_step(int dim, int L, const int8_t *J, int8_t *spins /* [n_temps][N] */,
                        int n_temps, const double *beta, int32_t *slot_of_temp, int64_t *E,
                        uint64_t seed, uint32_t q, uint32_t r0, uint32_t t, int m, uint64_t *swap_acc)
{
    int64_t N = n_sites(dim, L);
    for (int k = 0; k < n_temps; ++k) {
        int slot = slot_of_temp[k];
        for (int j = 0; j < m; ++j)
            E[slot] += orc_sweep(dim, L, J, spins + (int64_t)slot * N, beta[k], seed, r0 + (uint32_t)slot,
                                 t * (uint32_t)m + (uint32_t)j);
    }
    for (int k = (int)(t & 1u); k + 1 < n_temps; k += 2) {
        int A = slot_of_temp[k], B = slot_of_temp[k + 1];
        double x = (beta[k + 1] - beta[k]) * (double)(E[B] - E[A]);
        uint32_t w[4];
        draw(seed, (uint32_t)k, t, q, TAG_SWAP * 2, w);
        int accept = 1;
        if (!(x >= 0.0)) {
            double u = unit53(w[0], w[1]), p = exp(x);
            double gap = fabs(u - p);
            audit_attempts += 1;
            if (gap < 0x1p-40) audit_near_ties += 1;
            if (gap < audit_min_gap) audit_min_gap = gap;
            accept = u < p;
        }
        if (accept) {
            slot_of_temp[k] = B;
            slot_of_temp[k + 1] = A;
            if (swap_acc) swap_acc[k] += 1;
        }
    }
}

EXPORT void orc_pt_run(int dim, int L, const int8_t *J, int8_t *spins, int n_temps,
                       const double *beta, int32_t *slot_of_temp, int64_t *E, uint64_t seed,
                       uint32_t q, uint32_t r0, uint32_t t0, int n_steps, int m, uint64_t *swap_acc)
{
    for (int k = 0; k < n_steps; ++k)
        orc_pt_step(dim, L, J, spins, n_temps, beta, slot_of_temp, E, seed, q, r0, t0 + (uint32_t)k, m, swap_acc);
}

/* The swap uniform itself, exposed for the near-tie audit of exp(x). */
EXPORT double orc_swap_u53(uint64_t seed, uint32_t k, uint32_t t, uint32_t q)
{
    uint32_t w[4];
    draw(seed, k, t, q, TAG_SWAP * 2, w);
    return unit53(w[0], w[1]);
}

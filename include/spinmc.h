/*
 * spinmc.h -- C ABI of the MI355X checkerboard Metropolis / parallel-tempering
 * library (libspinmc.so).
 *
 * Method: M. Weigel, "Performance potential for simulating spin models on
 * GPU" (arXiv:1101.1427).  Models: Ising ferromagnet (Sec. 3.1, Eq. 1),
 * +-J Edwards-Anderson spin glass (Sec. 5, Eq. 11), O(3) Heisenberg model
 * with uniform re-orientation proposals (Sec. 4, Eq. 10).  Update:
 * single-spin-flip Metropolis (Eq. 2) on the two-colour checkerboard
 * (Sec. 3.2): one sweep updates every colour-0 site (x+y[+z] even), then
 * every colour-1 site.  Parallel tempering exchanges temperatures of
 * neighbouring replicas with Eq. (12) (Sec. 6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments marked DEVICE are device pointers owned by the caller
 *   (e.g. torch tensors on the current HIP device); arrays marked HOST are
 *   read during the call only.  The library never frees caller memory.  It
 *   keeps internal device scratch (threshold tables, ping-pong buffers),
 *   allocated on first use and grown as needed; SMC_ENOMEM if that fails.
 * - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *   asynchronous with respect to the host on that stream; its results are
 *   valid once the stream has reached the call.
 * - Arguments are validated on the host before anything is launched; on an
 *   argument error nothing is launched and nothing is modified.  Every kernel
 *   launch configuration is checked on the host as well (at least one
 *   workgroup, at most 2^31 - 1; 1 .. 1024 work-items per workgroup; dynamic
 *   LDS within 160 KiB; fewer than 2^32 work-items): a configuration outside
 *   these limits is not issued and the call returns SMC_EHIP with the
 *   kernel and the broken limit in smc_last_error().
 * - Calls on a stream that is capturing a graph return SMC_EINVAL and issue
 *   nothing: they stage host tables through pinned buffers, may grow their
 *   scratch and build graphs of their own, none of which can be recorded into
 *   a caller's capture.
 * - Inverse temperatures and uneven-batch tables are HOST arrays: the
 *   acceptance thresholds floor(2^32 exp(-beta Delta E)) are computed from
 *   them on the host in float64 with the C library's exp, so that every
 *   integer decision is reproducible off the device.
 * - Results are a pure function of (inputs, seed, sweep/step index): they
 *   do not depend on launch shapes, streams or the device.  Every random
 *   number is a Philox4x32-10 draw keyed by the seed with a counter made of
 *   (site or pair index, sweep index, replica or chain index, stream tag).
 * - Lattices are periodic simple (hyper)cubic, d = 2 or 3, edge L even and
 *   >= 4, N = L^d sites in row-major order with x fastest:
 *     2D: i = y*L + x,  3D: i = (z*L + y)*L + x.
 * - Ising / EA spins are int8 +1/-1.  Heisenberg spins are float32 triples
 *   (x, y, z) per site.  Couplings are int8 +1/-1 laid out [sample][mu][N]:
 *   entry (mu, i) is the bond joining i and i + e_mu.
 * - A batch holds n_rep replicas.  Uniform batch (desc.L > 0): replica r's
 *   spins start at element r*N (r*N*3 floats for Heisenberg) and an EA
 *   replica r uses sample r / rep_per_sample, whose couplings start at
 *   element (r / rep_per_sample) * d * N.  Uneven batch (desc.L == 0): the
 *   HOST table desc.inst[n_rep] gives each replica's edge, sample and offsets.
 * - Return value: SMC_OK (0) or a negative smc_status.
 * - Execution paths.  Uniform 2D Ising batches with L a power of two in
 *   [1024, 16384] sweep on a colour-split copy of the lattice in one launch
 *   per sweep (tempering too); uniform 2D Ising / EA batches of edge 16 ..
 *   128 (or 256 with at least 2^19 sites) keep each replica in one
 *   workgroup's LDS for up to 256 sweeps per launch; 3D edge-16 tempering
 *   runs all steps of a call in one launch; 2D tempering with edges in
 *   {16, 32, ..., 256} runs one workgroup per replica per step (a graph of
 *   steps); uniform 3D Ising / EA batches with L a multiple of 16 sweep
 *   16-site row segments per thread: for L in [512, 1024] in one launch per
 *   sweep that alternates between the caller's lattice and a library-held
 *   second lattice of the same size (an odd sweep count ends with one
 *   device copy back), below in two launches per sweep, in place;
 *   everything else takes generic per-site kernels.  All paths give
 *   identical results.  Environment variables for comparisons and tuning
 *   (read at each call): SPINMC_PT3D=0, SPINMC_UNEVEN2D=0 and
 *   SPINMC_PT_SPLIT2D=0 send tempering to the generic kernels,
 *   SPINMC_SWEEP_LDS2D=0 small 2D sweeps, SPINMC_SWEEP3D=0 3D Ising / EA
 *   sweeps; SPINMC_SWEEP3D_PASS=0 keeps the two launches per sweep for
 *   every edge, =1 takes the one launch from edge 32 (SPINMC_PASS3D_TY,
 *   _SEGS and _D set its rows per strip, segments per thread and planes
 *   per z segment; SPINMC_SWEEP3D_Z = 1 .. 16 rows per thread and
 *   SPINMC_SWEEP3D_NT=0, plain stores, the two-launch shape);
 *   SPINMC_L2D_CHUNKS (1 or 2),
 *   SPINMC_L2D_H (band height, a multiple of 4), SPINMC_L2D_H1 /
 *   SPINMC_L2D_H2 (heights of the bands of the first and second half of
 *   the grid) and SPINMC_L2D_PAD (row padding in bytes) set the launch
 *   shape of the 2D Ising sweep.  SPINMC_HEIS3D=0 sends uniform 3D
 *   Heisenberg batches to the generic kernel.
 */
#ifndef SPINMC_H
#define SPINMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SMC_OK = 0,
    SMC_EINVAL = -1,       /* invalid argument (message in smc_last_error()) */
    SMC_EUNSUPPORTED = -2, /* valid but not supported combination           */
    SMC_EHIP = -3,         /* a HIP runtime call failed                      */
    SMC_ENOMEM = -4        /* internal scratch could not be allocated        */
} smc_status;

typedef enum {
    SMC_ISING = 0,       /* ferromagnet, all couplings +1 (Eq. 1)              */
    SMC_EA = 1,          /* +-J Edwards-Anderson spin glass (Eq. 11)           */
    SMC_HEISENBERG = 2   /* O(3) unit vectors, ferromagnetic (Eq. 10)          */
} smc_model;

/* Arithmetic of the Heisenberg double checkerboard (Sec. 4 compares them). */
typedef enum {
    SMC_HEIS_FLOAT = 0,  /* float32 spins, accurate library sin/cos/exp, IEEE sqrt */
    SMC_HEIS_FAST = 1,   /* float32 spins, hardware sin/cos/exp/sqrt (the move of
                            smc_metropolis_sweep's Heisenberg kernels)           */
    SMC_HEIS_DOUBLE = 2  /* float64 spins and arithmetic                          */
} smc_heis_precision;

/* Generators of the random-number study (Sec. 3.3, Table 1). */
typedef enum {
    SMC_RNG_LCG32 = 1,         /* x' = 1664525 x + 1013904223 mod 2^32, one global
                                  sequence shared by all streams with skip-ahead */
    SMC_RNG_LCG32_RANDOM = 2,  /* the same map, every stream seeded independently */
    SMC_RNG_LCG64 = 3,         /* x' = 2862933555777941757 x + 1442695040888963407
                                  mod 2^64 (top 32 bits used), skip-ahead          */
    SMC_RNG_LCG64_RANDOM = 4,  /* the same map, independent stream seeds          */
    SMC_RNG_FIB521 = 5,        /* lagged Fibonacci x_n = x_{n-521} + x_{n-353}
                                  mod 2^32, one generator per tile                 */
    SMC_RNG_FIB1279 = 6        /* lagged Fibonacci with lags 1279 and 861          */
} smc_rng_generator;

/* One replica of an uneven batch. */
typedef struct smc_inst {
    int32_t L;        /* even edge length >= 4                                  */
    int32_t sample;   /* coupling sample (keys the coupling draws; EA only)     */
    int64_t spin_off; /* first spin of the replica, in spins (x3 floats: Heis.) */
    int64_t coup_off; /* first coupling of its sample, in int8 elements (EA)    */
} smc_inst;

typedef struct smc_desc {
    int32_t model;          /* smc_model                                          */
    int32_t dim;            /* 2 or 3                                             */
    int32_t L;              /* > 0: uniform batch of edge L; 0: use inst[]        */
    int32_t n_rep;          /* replicas in the batch, >= 1                        */
    int32_t rep_per_sample; /* uniform EA batch: replicas per coupling sample     */
    int32_t renorm_every;   /* Heisenberg: renormalise every spin after sweeps t
                               with (t+1) % renorm_every == 0; 0 = never          */
    uint64_t seed;          /* Philox key                                         */
    const smc_inst *inst;   /* HOST [n_rep] when L == 0, otherwise NULL           */
    int64_t spins_len;      /* elements in the caller's spin buffer (int8 spins or
                               floats, 3 per Heisenberg site); every replica must
                               lie inside it, else SMC_EINVAL                     */
    int64_t coup_len;       /* int8 elements in the coupling buffer (EA), else 0  */
} smc_desc;

/* Parallel-tempering layout: replica r = chain * n_temps + slot. */
typedef struct smc_pt_desc {
    int32_t n_chains;       /* independent chains                                 */
    int32_t n_temps;        /* temperatures (= replicas) per chain, >= 2          */
    int32_t beta_per_chain; /* 0: beta is [n_temps]; 1: beta is [n_chains][n_temps] */
    int32_t sweeps_per_step; /* m: sweeps between exchange rounds (0 or 1: one)  */
    const double *beta;     /* HOST inverse temperatures of the ladder, index k   */
} smc_pt_desc;

/*
 * Random initial state (scope row "spin_init").
 *  Ising/EA: spin i of replica r is +1 iff the top bit of word (i mod 4) of
 *  the draw (i/4, 0, r, 2) is 0.  Heisenberg: a uniform point on the sphere
 *  from words 0, 1 of (i, 0, r, 2).  EA couplings (Sec. 5, bimodal, p = 1/2):
 *  bond b = i*d + mu of sample q is +1 iff the top bit of word (b mod 4) of
 *  (b/4, 0, q, 4) is 0.
 *  spins:     DEVICE, int8 [.. N] or float32 [.. N][3], written.
 *  couplings: DEVICE int8, written for every sample used by the batch when
 *             model == SMC_EA and couplings != NULL; ignored otherwise.
 */
int smc_spin_init(const smc_desc *desc, void *spins, int8_t *couplings, void *stream);

/*
 * n_sweeps checkerboard Metropolis sweeps with global sweep indices
 * sweep0 .. sweep0 + n_sweeps - 1 (Eq. 2; Sec. 3.2; rows "half-sweep
 * colour 0 / colour 1", "Heisenberg sweep", "Delta E tracking").
 *  beta:     HOST [n_rep] inverse temperature of each replica (>= 0, finite).
 *  Ising/EA: a flip with Delta E = 4m > 0 is accepted iff the 32-bit uniform
 *            u < floor(2^32 exp(-4 m beta)); Delta E <= 0 is always accepted.
 *  Heisenberg: proposal uniform on the sphere, accepted iff Delta E <= 0 or
 *            u < exp(-beta Delta E) in float32; renormalisation per desc.
 *  couplings: DEVICE int8 (EA), NULL otherwise.
 *  dE_accum: DEVICE int64 [n_rep] or NULL.  Ising/EA: += the sum of Delta E
 *            over accepted flips (so E + dE_accum is the new energy).
 *            Heisenberg: += the number of accepted moves.
 *  Constraint: sweep0 + n_sweeps <= 2^32 (the sweep index is 32 bits).
 */
int smc_metropolis_sweep(const smc_desc *desc, void *spins, const int8_t *couplings,
                         const double *beta, uint64_t sweep0, int32_t n_sweeps,
                         int64_t *dE_accum, void *stream);

/*
 * n_steps parallel-tempering steps with indices step0 .. step0+n_steps-1
 * (Sec. 6, Eq. 12).  Step t: m = pt.sweeps_per_step sweeps (sweep indices
 * t*m .. t*m + m - 1; m = 1 when the field is 0) of every replica at its
 * current temperature, energies tracked from the accepted flips; then
 * for every pair (k, k+1) with k = t (mod 2), k <= n_temps-2, in every
 * chain q: A = slot_of_temp[q][k], B = slot_of_temp[q][k+1],
 * x = (beta_{k+1} - beta_k) * (E_B - E_A) in float64, accepted iff x >= 0 or
 * u53 < exp(x) with u53 the 53-bit uniform of the draw (k, t, q, 12); on
 * acceptance the two slots exchange temperatures.
 *  Models: Ising and EA (the EA replicas of one chain must share a sample).
 *  desc.n_rep must equal n_chains * n_temps.
 *  slot_of_temp: DEVICE int32 [n_chains][n_temps], in/out (a permutation of
 *                0..n_temps-1 per chain; a chain whose row is not one is
 *                left unchanged: spins, energies, slots and counts).
 *  energy:       DEVICE float64 [n_rep], in/out: energy of the configuration
 *                stored in each replica (exact integers; e.g. from
 *                smc_measure_energy_magnetisation).
 *  swap_accepts: DEVICE uint64 [n_chains][n_temps-1] or NULL; += accepted
 *                exchanges of pair k.
 *  Constraint: (step0 + n_steps) * m <= 2^32.
 */
int smc_pt_sweep_swap(const smc_desc *desc, const smc_pt_desc *pt, void *spins,
                      const int8_t *couplings, int32_t *slot_of_temp, double *energy,
                      uint64_t step0, int32_t n_steps, uint64_t *swap_accepts, void *stream);

/*
 * Energy and magnetisation of every replica (Sec. 3.5: energies as sums over
 * bonds, tracked incrementally during sweeps and recomputed here; Sec. 4:
 * measurements accumulated in double precision; Eqs. 1, 10, 11):
 *  E = -sum_i sum_mu J(i,mu) s_i . s_{i+e_mu},  M = sum_i s_i.
 *  energy:        DEVICE float64 [n_rep] (exact integers for Ising/EA).
 *  magnetisation: DEVICE float64 [n_rep] (Ising/EA) or [n_rep][3]
 *                 (Heisenberg), or NULL.
 *  Heisenberg sums are accumulated in float64 in a fixed order (the result
 *  is reproducible run to run).
 */
int smc_measure_energy_magnetisation(const smc_desc *desc, const void *spins,
                                     const int8_t *couplings, double *energy,
                                     double *magnetisation, void *stream);

/*
 * The same measurement for callers that cannot allocate device memory (code
 * running under a stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc / hipFree and stages nothing from the
 * host.  Its partial sums live in one fixed device array of the library
 * (16 MiB on each GPU it runs on, held until the process ends) instead of the
 * per-stream scratch; arguments, results and kernels are those of
 * smc_measure_energy_magnetisation, so the results are identical.
 *  desc:  a uniform batch (L > 0); SMC_EUNSUPPORTED for an uneven one.
 *         The partial sums take 32 bytes x n_rep x min(2048, ceil(N / 4096));
 *         a batch needing more than 16 MiB is refused with SMC_EINVAL before
 *         anything is issued (e.g. up to 256 replicas of 16384^2, or 524288
 *         replicas of up to 4096 sites).
 *  spins, couplings, energy, magnetisation, stream: as above.
 * Every call on one GPU shares that GPU's array, which keeps the previous
 * call's contents (every entry a call reads it writes first): calls that
 * overlap on one GPU (different streams, or host threads) race and must be
 * ordered by the caller.
 */
int smc_measure_energy_magnetisation_noalloc(const smc_desc *desc, const void *spins,
                                             const int8_t *couplings, double *energy,
                                             double *magnetisation, void *stream);

/*
 * Autotuning of launch shapes; it never changes results.  It measures, on
 * scratch lattices of the batch's shape with random spins, and keeps for
 * later calls in the process on this device:
 *  - 2D Ising / EA: the workgroup size of the LDS-resident 2D kernel
 *    (small lattices, uneven tempering) for every edge of the batch that
 *    this kernel takes (calls that meet an edge first measure it
 *    themselves, on copies of their own replicas);
 *  - uniform 2D Ising with L a power of two in [1024, 16384]: the band
 *    height of the one-pass sweep (rows per workgroup, 4 .. 128), per edge
 *    and replica count;
 *  - uniform 3D Ising / EA with L a multiple of 16: the strip shape of the
 *    one-pass sweep (rows per strip, segments per thread, planes per z
 *    segment) where that sweep is taken, else the rows per thread of the
 *    half-sweeps, per edge, model and replica count.
 * Each candidate is timed over about 5 ms after an untimed round; a shape
 * other than the default is kept only if it is more than 2 % faster.
 * Environment overrides of a shape (SPINMC_L2D_H, SPINMC_PASS3D_*,
 * SPINMC_SWEEP3D_Z, SPINMC_U2D_THREADS) take precedence, and that shape is
 * then not measured.  The double checkerboard's tile is an argument of
 * smc_dcb_sweep (it changes the chain), never a tuned shape.  Other batches
 * have nothing to tune (SMC_OK, no device work).
 *  cache_path: NULL, or a text file read first (choices recorded for this
 *              device, identified by its architecture name and compute
 *              units, are not measured again) and written afterwards (lines
 *              of other devices are kept).  SMC_EINVAL if it cannot be
 *              written.
 * Synchronous with respect to the host; not allowed under stream capture.
 */
int smc_autotune(const smc_desc *desc, const char *cache_path, void *stream);

/*
 * How smc_metropolis_sweep will execute this batch: the number of kernel
 * launches per sweep and the name of the sweep kernel (a static string).
 * Used by benchmarks to attribute per-launch time; no device work.
 */
int smc_sweep_plan(const smc_desc *desc, int32_t *launches_per_sweep, const char **kernel_name);

/*
 * Profiling aid.  While enabled (enable != 0), smc_metropolis_sweep records a
 * pair of HIP events on the call's stream around the sweep kernels of each
 * call (the layout conversions of the 2D Ising path are outside the pair).
 * smc_kernel_timing_read waits for the recorded events, returns the summed
 * elapsed milliseconds and the number of sweep-kernel launches they cover,
 * and forgets them.  Disabling also forgets unread events.  Returns
 * SMC_EHIP if an event call fails.
 */
int smc_kernel_timing_enable(int enable);
int smc_kernel_timing_read(double *elapsed_ms, int64_t *launches);

/*
 * How smc_pt_sweep_swap will execute: the number of kernel launches for a
 * call of n_steps steps and the name of the sweep kernel (a static string).
 * 3D lattices of edge 16 with n_temps <= 32 (EA: rep_per_sample a multiple
 * of n_temps) run all steps of a call in one launch, one workgroup per chain
 * with the chain resident in LDS; other shapes take three launches per step
 * (two half-sweeps and the exchange round) plus two.  No device work.
 */
int smc_pt_plan(const smc_desc *desc, const smc_pt_desc *pt, int32_t n_steps, int32_t *launches,
                const char **kernel_name);

/*
 * Asynchronous multi-spin coding (Sec. 5): the same sweeps as
 * smc_metropolis_sweep for a uniform Ising or EA batch whose replicas come
 * in groups of w = word_bits (32 or 64; replicas wg .. wg+w-1 form group g)
 * that share their Metropolis random numbers: the draws of every site of
 * replica r are made with the group index r / w in the place of the
 * replica index (counters (h/8, t, r/w, 6 + c) and (h, t, r/w, 8 + c)), as
 * the paper uses one random number per site for all replicas coded in one
 * w-bit word.  Each replica keeps its own spins and couplings (EA:
 * rep_per_sample must be 1).
 *  desc:     uniform batch (L > 0), model SMC_ISING or SMC_EA, n_rep a
 *            multiple of w.
 *  spins, couplings, sweep0, n_sweeps, dE_accum, stream: as for
 *            smc_metropolis_sweep (dE_accum: DEVICE int64 [n_rep], += the
 *            energy change of each replica).
 *  beta:     HOST [n_rep]; equal within each group of w, else SMC_EINVAL.
 *  word_bits: 32 or 64, else SMC_EINVAL.
 * 2D batches of edge 16, 32 or 64 (spins and couplings 4-byte aligned) run
 * with 32 replicas packed per 32-bit word (w = 64: a thread updates the two
 * words of a group with one draw), every sweep of the call in one
 * launch, the lattices held on chip
 * (SPINMC_MSC2D=0 sends them to the generic kernels); other shapes take the
 * generic kernels.  Results are identical either way.  SMC_EUNSUPPORTED for
 * the Heisenberg model.
 */
int smc_msc_sweep(const smc_desc *desc, void *spins, const int8_t *couplings, const double *beta, uint64_t sweep0,
                  int32_t n_sweeps, int32_t word_bits, int64_t *dE_accum, void *stream);

/*
 * How smc_msc_sweep will execute: the number of sweep-kernel launches for a
 * call of n_sweeps sweeps and the sweep kernel's name (a static string),
 * for aligned buffers.  The same argument checks as smc_msc_sweep on desc
 * and word_bits; no device work.
 */
int smc_msc_plan(const smc_desc *desc, int32_t n_sweeps, int32_t word_bits, int32_t *launches,
                 const char **kernel_name);

/*
 * Double checkerboard sweeps with multi-hit updates (Sec. 3.2, Sec. 3.4): a
 * different Markov chain from smc_metropolis_sweep, whose order depends on
 * the tiling.  The lattice is cut into tiles of edge `tile`, B = L / tile
 * per direction; tile (bx, by) has tile colour (bx + by) & 1.  Sweep t treats every tile of tile colour 0, then every
 * tile of colour 1; each tile gets `hits` hits, a hit being a Metropolis
 * attempt (Eq. 2) at each colour-0 site of the tile, then at each colour-1
 * site, with the sites outside the tile held fixed.  With palindromic != 0
 * odd sweeps run both orders backwards (tile colour 1 first, colour-1 sites
 * first; two sweeps then form a palindrome of single-colour updates, Sec.
 * 3.4).  Hit j of sweep t draws the uniforms smc_metropolis_sweep draws in
 * sweep t*hits + j; with tile = L and hits = 1 the two calls agree.
 *  desc:      uniform 2D or 3D batch (L > 0), model SMC_ISING or SMC_EA.
 *             In 3D the tiles are cubes and tile colour is (bx + by + bz) & 1.
 *  tile:      2D: a multiple of 16 in [16, 128] with L / tile even or 1;
 *             3D: 16, with L / 16 even or 1 (spins and couplings 16-byte
 *             aligned).
 *  hits:      >= 1; (sweep0 + n_sweeps) * hits must not exceed 2^32.
 *  spins, couplings, beta (HOST [n_rep]), sweep0, n_sweeps, dE_accum,
 *  stream: as for smc_metropolis_sweep; every replica is updated in place.
 *  dE_trace:  device int64 [n_sweeps][n_rep] or NULL: row m receives each
 *             replica's energy change from the start of the call through
 *             sweep m (a measurement after every sweep, as in the
 *             autocorrelation study of Sec. 3.4); written, not added to.
 * SMC_EUNSUPPORTED for Heisenberg batches (see smc_heis_dcb_sweep),
 * SMC_EINVAL for a tile or hit count outside these limits.
 */
int smc_dcb_sweep(const smc_desc *desc, void *spins, const int8_t *couplings, const double *beta, uint64_t sweep0,
                  int32_t n_sweeps, int32_t tile, int32_t hits, int32_t palindromic, int64_t *dE_accum,
                  int64_t *dE_trace, void *stream);

/*
 * Double checkerboard sweeps with multi-hit updates of the 2D Heisenberg
 * model (Sec. 3.2, Sec. 3.4, Sec. 4): the order of smc_dcb_sweep (tile
 * colour 0, then 1; k = hits hits per tile, each a move at every colour-0
 * site of the tile, then at every colour-1 site, with the sites outside the
 * tile held fixed; palindromic != 0 reverses both orders on odd sweeps).
 * The move at a site is that of smc_metropolis_sweep (uniform proposal from
 * words 0, 1 and acceptance from word 2 of the Heisenberg draw) with the
 * draws of sweep t*hits + j for hit j of sweep t, so tile = L, hits = 1 and
 * precision = SMC_HEIS_FAST reproduce smc_metropolis_sweep.  After sweep t
 * every spin is renormalised when desc.renorm_every > 0 divides t + 1.
 *  desc:      uniform 2D batch (L > 0), model SMC_HEISENBERG; spins_len in
 *             elements (3 per site).
 *  spins:     DEVICE, 16-byte aligned; float32 [n_rep][N][3], or float64
 *             for SMC_HEIS_DOUBLE; updated in place.
 *  beta:      HOST [n_rep], finite and >= 0 (used as float32 in the float
 *             modes).
 *  tile:      16 or 32 (any precision) or 64 (float modes), with L / tile
 *             even or 1.
 *  hits:      >= 1; (sweep0 + n_sweeps) * hits must not exceed 2^32.
 *  precision: smc_heis_precision.
 *  cap:       0: the proposal is a uniform re-orientation (independent of
 *             the spin); 0 < cap <= 2: small steps, the proposal uniform on
 *             the spherical cap 1 - a.s' <= cap around a = s/|s| (Sec. 4
 *             suggests them for low temperatures): w = cap u0 is one minus
 *             the cosine of the angle, 2 pi u1 the azimuth in the frame
 *             e1 = (-a_y, a_x, 0)/|..| when |a_x| > |a_z|, else
 *             (0, -a_z, a_y)/|..|, and e2 = a x e1.
 *  accepts:   DEVICE int64 [n_rep] or NULL: += the number of accepted moves.
 * SMC_EINVAL for a bad tile, hit count, precision, cap or unaligned spins;
 * SMC_EUNSUPPORTED for other models or 3D.
 */
int smc_heis_dcb_sweep(const smc_desc *desc, void *spins, const double *beta, uint64_t sweep0, int32_t n_sweeps,
                       int32_t tile, int32_t hits, int32_t precision, int32_t palindromic, double cap,
                       int64_t *accepts, void *stream);

/*
 * Which kernel smc_dcb_sweep uses for this batch, tile and beta (HOST
 * [n_rep]), for 16-byte aligned spins and couplings: "k_dcb2d_packed" (four
 * sites per word; tile 16, 32, 64 or 128 and every beta > 0) or "k_dcb2d"
 * (one site per thread).  Results are identical either way.  The same
 * argument checks as smc_dcb_sweep on desc, tile and beta; no device work.
 * kernel_name receives a static string.
 */
int smc_dcb_plan(const smc_desc *desc, const double *beta, int32_t tile, const char **kernel_name);

/*
 * Throughput probe of the random-number generator (Sec. 3.3, Fig. 4
 * measure generators on their own): thread i of n_threads draws the
 * Philox4x32-10 blocks with counters (i + k * n_threads, t, r, tag) for
 * k = 0 .. per_thread-1 under the key of `seed`, and writes the XOR of all
 * their words to out[i] (device, n_threads words, owned by the caller).
 * Not part of the method: it gives the generator's cost per block on its
 * own, against which the sweep kernels' times are read.  SMC_EINVAL if out
 * is NULL, n_threads or per_thread is not positive, or
 * n_threads * per_thread exceeds 2^32 (the block index is one 32-bit word).
 * Asynchronous on `stream`.
 */
int smc_philox_bench(uint64_t seed, uint32_t t, uint32_t r, uint32_t tag, int32_t n_threads, int32_t per_thread,
                     uint32_t *out, void *stream);

/*
 * The random-number study of Sec. 3.3 (Table 1): double-checkerboard sweeps
 * (tile colour 0 then 1, `hits` hits per tile, each colour 0 then colour 1;
 * no palindrome) of a uniform 2D Ising or EA batch whose uniforms come from
 * one of the paper's generators instead of the Philox streams.  Not the
 * method's sampler (its results depend on the generator, which is the point
 * of the study): the sampler is smc_dcb_sweep.
 *  Streams.  Tiles of edge T = tile (B = L / T per direction, B even); the
 *  tiles of one tile colour are numbered q = by (B/2) + bx/2 and the sites
 *  of one colour inside a tile p = v (T/2) + u/2 (site (u, v) of the tile),
 *  the L^2/4 positions (q, p) being the threads of the paper's code.  An LCG
 *  stream j = q T^2/2 + p serves position (q, p) of both tile colours and
 *  both site colours, one number per attempt in sweep order; with
 *  skip-ahead (Eqs. 4-5) stream j delivers x_j, x_{j+M}, x_{j+2M}, ... of
 *  one global sequence (M = L^2/4), otherwise it steps its own seed by the
 *  map.  A lagged Fibonacci generator serves tile q; each round (one colour
 *  of one hit of the tile) takes T^2/2 consecutive numbers, position p the
 *  p-th.  Every attempt consumes a number (also when Delta E <= 0).  The
 *  acceptance is u < floor(2^32 exp(-beta Delta E)) with u the 32-bit number
 *  (LCG64: the top 32 bits).
 *  Seeds (smc_rng_study_init) are Philox4x32-10 draws under desc.seed with
 *  counter word 3 = 16: x_0 of replica r's global sequence from (0, 0, r,
 *  16), stream j's seed from (j, 1, r, 16), word i of tile q's Fibonacci
 *  ring from (q * r_lag + i, 2, r, 16) (word 0; 64-bit values: word 1 above
 *  word 0).
 *  desc:    uniform 2D batch, SMC_ISING or SMC_EA (EA couplings as usual).
 *  tile:    16 or 32 with L / tile even (Fibonacci generators: 16, so that a
 *           round of T^2/2 numbers reads none of its own).
 *  state:   DEVICE, owned by the caller, smc_rng_study_state_bytes bytes
 *           (8-byte aligned); replica-major; written by smc_rng_study_init,
 *           advanced by every sweep (a run split over calls equals one call).
 *  beta:    HOST [n_rep]; hits >= 1; dE_accum: DEVICE int64 [n_rep] or NULL
 *           (+= the energy change).
 * SMC_EINVAL for other tiles, generators, models or a too small state.
 */
int smc_rng_study_state_bytes(const smc_desc *desc, int32_t tile, int32_t generator, int64_t *bytes);
int smc_rng_study_init(const smc_desc *desc, int32_t tile, int32_t generator, void *state, int64_t state_bytes,
                       void *stream);
int smc_rng_study_sweep(const smc_desc *desc, void *spins, const int8_t *couplings, const double *beta,
                        int32_t n_sweeps, int32_t tile, int32_t hits, int32_t generator, void *state,
                        int64_t state_bytes, int64_t *dE_accum, void *stream);

/* Static description of a status code. */
const char *smc_strerror(int status);

/* Detail of the last error raised on the calling host thread ("" if none). */
const char *smc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPINMC_H */

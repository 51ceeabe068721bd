// Internal interfaces between the C-ABI layer (api.hip, runtime.hip, tune.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/spinmc.h"
#include "lattice2d.hpp"
#include "launch_check.hpp"
#include "philox.hpp"
#include "tables.hpp"

namespace smc {

// A launch whose configuration launch_config_error refuses is not issued:
// the description (kernel, grid, workgroup, LDS, reason) is kept for the
// calling thread's error message and hipErrorInvalidConfiguration returned.
hipError_t reject_launch(const char *kernel, uint64_t grid, uint64_t block, uint64_t lds, const char *why);
// The description of the last refused launch on this thread ("" if none),
// cleared by reading it.
std::string take_launch_rejection();

// Every kernel launch of the library goes through this check (inside
// functions that return hipError_t).
#define SMC_LAUNCH(kernel, grid, block, lds, stream, ...)                                                   \
    do {                                                                                                   \
        const dim3 g_ = (grid), b_ = (block);                                                              \
        const uint64_t ng_ = (uint64_t)g_.x * g_.y * g_.z, nb_ = (uint64_t)b_.x * b_.y * b_.z;             \
        const uint64_t lds_ = (uint64_t)(lds);                                                             \
        if (const char *why_ = ::smc::launch_config_error(ng_, nb_, lds_))                                 \
            return ::smc::reject_launch(#kernel, ng_, nb_, lds_, why_);                                    \
        hipLaunchKernelGGL(kernel, g_, b_, lds_, stream, __VA_ARGS__);                                     \
    } while (0)

// Geometry of a batch as the kernels see it.  Uniform batches use (L, N,
// spin_stride, coup_stride, rep_per_sample); uneven ones the inst table.
struct Batch {
    int dim;
    int model;
    int n_rep;
    int L;                  // > 0 uniform, 0 uneven
    int64_t N;              // sites per replica (uniform)
    int rep_per_sample;     // uniform EA
    const smc_inst *inst;   // device [n_rep] (uneven) or nullptr
};

__device__ __forceinline__ smc_inst replica_geom(const Batch &b, int r) {
    if (b.L > 0) {
        smc_inst g;
        g.L = b.L;
        g.sample = r / b.rep_per_sample;
        g.spin_off = (int64_t)r * b.N;
        g.coup_off = (int64_t)g.sample * b.dim * b.N;
        return g;
    }
    return b.inst[r];
}

struct SweepArgs {
    Batch b;
    void *spins;
    const int8_t *coup;        // EA couplings or nullptr
    const ThrRow *thr;         // discrete: rows of thresholds
    const float *beta_f;       // Heisenberg: beta per row
    const int32_t *row_of_rep; // nullptr: row = replica index
    Key key;
    uint32_t t;                // sweep index
    int64_t *dE;               // nullable per-replica accumulator
    int max_L;                 // largest edge in the batch
    int rng_shift;             // the Metropolis draws of replica r use index r >> rng_shift
};

struct SwapArgs {
    const uint32_t *t_dev;     // step index in device memory, or nullptr: use t
    int n_chains, n_temps, beta_per_chain;
    const double *beta;        // device [rows][n_temps]
    int32_t *slot_of_temp;     // [n_chains][n_temps]
    int32_t *row_of_rep;       // [n_rep]: threshold row of each replica
    int64_t *E;                // [n_rep]
    unsigned long long *acc;   // [n_chains][n_temps-1] or nullptr
    Key key;
    uint32_t t;
};

// ---- launchers (each returns the hipError_t of its launch) ----
hipError_t launch_init_spins(const Batch &b, int max_L, int8_t *spins, Key key, hipStream_t s);
hipError_t launch_init_heis(const Batch &b, int max_L, float *spins, Key key, hipStream_t s);
hipError_t launch_init_couplings(int dim, int n_samples, const smc_inst *samples_dev, int max_L, int8_t *coup,
                                 Key key, hipStream_t s);

// Generic in-place half-sweep of colour c over every replica (any L, d).
hipError_t launch_half_sweep_generic(const SweepArgs &a, int c, hipStream_t s);
hipError_t launch_heis_half_sweep_generic(const SweepArgs &a, int c, hipStream_t s);
hipError_t launch_heis_renorm(const Batch &b, float *spins, int max_L, hipStream_t s);

// Heisenberg half-sweeps of uniform 3D batches with a power-of-two edge.
bool heis3d_supported(int dim, int L);
hipError_t launch_heis3d_half(float *spins, const float *beta, int64_t *acc, int n_rep, int L, Key key, uint32_t t,
                              int c, hipStream_t s);
// One-pass (tiled, colour 0 then colour 1 in one launch) sweep from src to dst, L >= 32;
// with renorm the spins written to dst are renormalised.
bool heis3d_tiled_supported(int dim, int L);
hipError_t launch_heis3d_tiled(const float *src, float *dst, const float *beta, int64_t *acc, int n_rep, int L, Key key,
                               uint32_t t, bool renorm, hipStream_t s);

// Parallel tempering of 3D edge-16 chains, all steps in one launch.
bool pt3d_supported(const smc_desc *d, int n_temps);
size_t pt3d_lds_bytes(int model, int n_temps);
hipError_t launch_pt3d(int model, int8_t *spins, const int8_t *coup, int rep_per_sample, int n_chains, int n_temps,
                       int beta_per_chain, const double *beta, const ThrRow *thr, int32_t *slot_of_temp,
                       double *energy, unsigned long long *acc, Key key, uint32_t t0, int n_steps, int m,
                       hipStream_t s);

// Uneven 2D batches: one workgroup per replica with the replica in LDS.
struct Uneven2dArgs {
    int8_t *spins;             // caller's spins (row-major int8 +-1 per replica)
    const smc_inst *inst;      // device [n_rep]
    const uint8_t *csplit;     // colour-split coupling planes at each sample's coup_off, or nullptr (Ising)
    const int32_t *row_of_rep; // threshold row per replica; -1 leaves the replica unchanged
    const ThrRow *thr;
    int64_t *E;                // tracked energy per replica
    const uint32_t *t_dev;     // first sweep index of the launch (device)
    int sweeps;                // sweeps per launch (indices *t_dev .. *t_dev + sweeps - 1), the replica kept in LDS
    Key key;
    uint32_t one2;  // 0x00010001 (opaque to the compiler)
};
bool uneven2d_edge_supported(int L);
size_t uneven2d_lds_bytes(int L);
hipError_t uneven2d_prepare_kernel(bool ea, int L);
Uneven2dArgs make_uneven2d_args(int8_t *spins, const smc_inst *inst, const uint8_t *csplit, const int32_t *row_of_rep,
                                const ThrRow *thr, int64_t *E, const uint32_t *t_dev, Key key);
hipError_t launch_coup_split2d(const int8_t *coup, uint8_t *out, const smc_inst *samples, int n_samples,
                               int64_t chunks_total, const int64_t *chunk_start, hipStream_t s);
hipError_t launch_set_step(uint32_t *t_dev, uint32_t t, hipStream_t s);
hipError_t launch_uneven2d_sweep(const Uneven2dArgs &a, const int32_t *work, int n_work, int L, bool ea, int threads,
                                 hipStream_t s);
hipError_t launch_advance_step(uint32_t *t_dev, hipStream_t s, uint32_t inc = 1);
hipError_t add_uneven2d_sweep_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, size_t n_deps,
                                   const Uneven2dArgs &a, const int32_t *work, int n_work, int L, bool ea,
                                   int threads);
hipError_t add_advance_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, size_t n_deps,
                            uint32_t *t_dev, uint32_t inc = 1);
hipError_t add_pt_swap_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, size_t n_deps,
                            const SwapArgs &a);

// Asynchronous multi-spin coding (2D EA/Ising, L in {16, 32, 64}): replicas
// 32g .. 32g+31 packed into one word per site, all sweeps in one launch.
bool msc2d_supported(int dim, int L);
hipError_t launch_msc_pack(const int8_t *spins, uint32_t *packed, int64_t N, int n_groups, hipStream_t s);
hipError_t launch_msc_pack_coup(const int8_t *coup, uint32_t *packed, int64_t dN, int n_groups, hipStream_t s);
hipError_t launch_msc_unpack(const uint32_t *packed, const uint32_t *gauge, int8_t *spins, int64_t N, int n_groups,
                             hipStream_t s);
// Gauge fixing of packed 2D words (horizontal bonds +1 except the row's
// closing bond); gauge [G][L*L] receives the transformation for unpacking.
hipError_t launch_msc_gauge2d(uint32_t *spins, uint32_t *coup, uint32_t *gauge, int L, int n_groups, hipStream_t s);
hipError_t launch_msc_energy_diff(const double *E0, const double *E1, int64_t *dE, int n, hipStream_t s);
// words_per_draw: 1 (32 replicas share a draw) or 2 (64: words 2h, 2h + 1).
hipError_t launch_msc2d(uint32_t *spins, const uint32_t *coup, const ThrRow *thr, int n_groups, int L, Key key,
                        uint32_t t0, int n_sweeps, int words_per_draw, hipStream_t s);

// Double checkerboard with multi-hit (2D Ising / EA, T x T tiles, T a
// multiple of 16 in [16, 128], L / T even or 1): one launch per tile colour.
// The packed kernel (four sites per word; T in {16, 32, 64, 128}) needs
// thresholds whose high halves fit 16 bits (beta > 0) and 16-byte aligned
// spins and couplings; the per-site kernel takes everything else.
bool dcb2d_supported(int L, int T);
bool dcb2d_packed_supported(int L, int T);
int dcb2d_tiles_per_colour(int L, int T);
hipError_t launch_dcb2d(int8_t *spins, const int8_t *coup, int rep_per_sample, const ThrRow *thr, int64_t *dE_slots,
                        int n_rep, int L, int T, int k, Key key, uint32_t t, int tile_colour, bool rev, bool packed,
                        hipStream_t s);
hipError_t launch_dcb_zero(int64_t *p, int64_t n, hipStream_t s);
// dE[r] = (assign) or += (otherwise) the sum of replica r's slots.
hipError_t launch_dcb_collect(const int64_t *slots, int64_t *dE, int n_rep, int per_rep, bool assign, hipStream_t s);

// Half-sweeps of uniform 3D Ising / EA batches with L a multiple of 16
// (sweep3d.hip): in place, 16-byte aligned spins and couplings, threshold
// high halves <= 0xFFFF; dE (nullable) accumulates per replica.
// EA bonds come as int8 (coup) or bit-packed (pbonds, from
// launch_pack_bonds3d: [sample][L^3 / 16] uint2), the other nullptr.
bool sweep3d_supported(int L);
hipError_t launch_pack_bonds3d(const int8_t *coup, uint2 *out, int L, int n_samples, hipStream_t s);
// Rows per thread along z of the next half-sweep of this batch.
int sweep3d_rows(int L, bool ea, int n_rep);
hipError_t launch_ising3d_half(int8_t *spins, const int8_t *coup, const uint2 *pbonds, int rep_per_sample,
                               const ThrRow *thr, int64_t *dE, int n_rep, int L, Key key, uint32_t t, int c,
                               hipStream_t s);

// 3D double checkerboard (dcb3d.hip): 16^3 tiles, L / 16 even or 1.
bool dcb3d_supported(int L, int T);
int dcb3d_tiles_per_colour(int L, int T);
hipError_t launch_dcb3d(int8_t *spins, const int8_t *coup, int rep_per_sample, const ThrRow *thr, int64_t *dE_slots,
                        int n_rep, int L, int T, int k, Key key, uint32_t t, int tile_colour, bool rev,
                        hipStream_t s);

// Heisenberg double checkerboard (2D; T = 16, 32, or 64 in the float modes;
// L / T even or 1): one launch per tile colour, and the renormalisation of
// every spin of the batch in the mode's arithmetic.  beta is float or double
// per precision.
bool heis_dcb2d_supported(int L, int T, int precision);
hipError_t launch_heis_dcb2d(void *spins, const void *beta, int64_t *acc_slots, int n_rep, int L, int T, int k,
                             int precision, double cap, Key key, uint32_t t, int tile_colour, bool rev,
                             hipStream_t s);
hipError_t launch_heis_dcb_renorm(void *spins, int64_t n_spins, int precision, hipStream_t s);

// Tempering on the 2D colour-split sweep (pt_split2d.hip): per-replica
// threshold rows from row_of_rep, masked energy updates (d is zeroed), and
// the copy back of replicas of valid chains (N a multiple of 16).
hipError_t launch_pt_gather_thr(const ThrRow *rows, const int32_t *row_of_rep, ThrRow *out, int n_rep,
                                hipStream_t s);
hipError_t launch_pt_add_masked(int64_t *d, int64_t *E, const int32_t *row_of_rep, int n_rep, hipStream_t s);
hipError_t launch_copy_valid(const int8_t *src, int8_t *dst, const int32_t *row_of_rep, int64_t N, int n_rep,
                             hipStream_t s);
hipError_t launch_zero64(int64_t *p, int n, hipStream_t s);

// Generator throughput: out[i] = XOR of the four words of the blocks with
// counters (i + k * n_threads, t, r, tag), k < per_thread.
hipError_t launch_philox_bench(Key key, uint32_t t, uint32_t r, uint32_t tag, uint32_t n_threads, int per_thread,
                               uint32_t *out, hipStream_t s);

// Measurement: partials of every replica, then a fixed-order final sum.
hipError_t launch_measure(const Batch &b, const void *spins, const int8_t *coup, int max_L, double *energy,
                          double *magnet, void *scratch, size_t scratch_bytes, hipStream_t s);
size_t measure_scratch_bytes(const Batch &b, int max_L);

// Parallel tempering helpers.
hipError_t launch_pt_prepare(const SwapArgs &a, const double *energy_in, hipStream_t s);
hipError_t launch_pt_swap(const SwapArgs &a, hipStream_t s);
hipError_t launch_pt_finish(const SwapArgs &a, double *energy_out, hipStream_t s);

// ---- tuned launch shapes (tune.hip) ----
// Launch shapes measured by smc_autotune, per device (the current one),
// kind, edge, model (0 Ising, 1 EA) and replica count.  The launchers take
// an environment override first, then a tuned shape, then their default;
// no shape changes results.
enum ShapeKind { kShapeBand2d = 0, kShapePass3d = 1, kShapeHalf3d = 2 };
struct Shape {
    int v[3];  // band2d: rows per band; pass3d: rows per strip, segments per thread, planes per z segment; half3d: rows per thread
};
bool tuned_shape(int kind, int L, int model, int n_rep, Shape *out);
void set_tuned_shape(int kind, int L, int model, int n_rep, const Shape &s);

// ---- one-pass 3D Ising / EA sweep (pass3d.hip): src and dst distinct ----
bool pass3d_supported(int L);
// Whether (rows per strip, segments per thread, planes per z segment) is a
// launch shape of the one-pass sweep for this edge and model.
bool pass3d_shape_valid(int L, bool ea, int ty, int segs, int D);
// The launch shape the next one-pass sweep of this batch takes (false if
// the edge has none).
bool pass3d_launch_shape(int L, bool ea, int n_rep, Shape *out);
hipError_t launch_ising3d_pass(const int8_t *src, int8_t *dst, const uint2 *pbonds, int rep_per_sample,
                               const ThrRow *thr, int64_t *dE, int n_rep, int L, Key key, uint32_t t,
                               hipStream_t s);

// ---- random-number study (rngstudy.hip) ----
bool rng_study_lags(int gen, int *r, int *s);
int64_t rng_study_state_bytes(int gen, int L, int T);  // per replica; 0 for an unknown generator
hipError_t launch_rng_init(int gen, int L, int T, int n_rep, void *state, Key key, hipStream_t s);
hipError_t launch_dcb_rng(int gen, int8_t *spins, const int8_t *coup, int rep_per_sample, const ThrRow *thr,
                          void *state, int64_t *dE, int n_rep, int L, int T, int k, int tile_colour, hipStream_t s);

}  // namespace smc

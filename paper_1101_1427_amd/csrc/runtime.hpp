// The host runtime of the C-ABI layer: error text, per-stream device
// scratch and pinned staging, acceptance tables, argument validation and
// the predicates that choose an execution path.  Used by the entry points
// (api.hip) and the autotuner (tune.hip); defined in runtime.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "internal.hpp"

namespace smc {

// The calling thread's text of the last error (smc_last_error).
std::string &last_error();
// Records the message and returns code.
int fail(int code, const char *fmt, ...);

#define SMC_HIP(call)                                                                                    \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) {                                                                          \
            const std::string why_ = take_launch_rejection();                                            \
            return fail(SMC_EHIP, "%s: %s%s%s", #call, hipGetErrorString(e_), why_.empty() ? "" : ": ", \
                        why_.c_str());                                                                   \
        }                                                                                                \
    } while (0)

// ------------------------------------------------------------------ scratch --
// Device scratch and a pinned staging area, one set per (device, stream):
// calls on one stream are ordered, so reusing the set between them is safe;
// calls on different streams never share a set.
struct Buffer {
    void *p = nullptr;
    size_t bytes = 0;
    // uploaded slots: pinned staging, the event of its last copy, and the
    // bytes last uploaded (an identical upload is skipped)
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t staged = nullptr;
    bool staged_pending = false;
    std::vector<unsigned char> last;
};

enum Slot {
    kTables = 0,
    kInst,
    kSamples,
    kMeasure,
    kEnergy64,
    kRows,
    kBeta,
    kPingPong,
    kCoupSplit,
    kChunks,
    kWork,
    kStep,
    kTuneSpins,
    kTuneInst,
    kTuneWork,
    kTuneRows,
    kTuneE,
    kHeisPing,
    kL2dPart,
    kMscSpins,
    kMscCoup,
    kMscEnergy,
    kMscGauge,
    kDcbSlots,
    kPtThr,
    kPtDelta,
    kPtOut,
    kBonds3d,    // bit-packed 3D EA bonds of the segment sweep
    kPass3d,     // second lattice buffer of the one-pass 3D sweep
    kTuneA,      // scratch lattices of the launch-shape tuner
    kTuneB,
    kNumSlots
};

// An instantiated tempering graph of `steps` steps and the launch arguments
// it was built from (rebuilt when they change).
struct GraphCache {
    std::vector<uint64_t> sig;
    hipGraphExec_t exec = nullptr;
};

struct StreamCtx {
    hipStream_t stream = nullptr;  // the stream whose calls use this set
    Buffer dev[kNumSlots];
    GraphCache graphs[2];  // full chunk of steps, remainder
};

StreamCtx &ctx_for(hipStream_t s);
// Device buffer of at least `bytes` in a slot of the set.
int ensure(StreamCtx &c, Slot slot, size_t bytes, void **out);
// Frees a slot's device buffer once the set's stream has finished with it.
int release(StreamCtx &c, Slot slot);
// Host bytes into a slot through its pinned staging area.
int upload(StreamCtx &c, hipStream_t s, Slot slot, const void *src, size_t bytes, void **dev_out);
// SMC_EINVAL (nothing issued) if s is capturing a graph.
int refuse_capture(hipStream_t s);

// ----------------------------------------------------------------- tables ----
ThrRow threshold_row(double beta, int dim);

// ------------------------------------------------------------------ paths ----
bool use_heis3d(const smc_desc *d);
bool use_heis3d_tiled(const smc_desc *d);
bool pt3d_enabled();
bool use_pt3d(const smc_desc *d, const smc_pt_desc *pt, const void *spins, const std::vector<ThrRow> &rows);
bool use_lattice2d(const smc_desc *d, const void *spins, const std::vector<ThrRow> &rows);
bool sweep3d_shape(const smc_desc *d);
bool pass3d_enabled(const smc_desc *d);
bool use_sweep3d(const smc_desc *d, const void *spins, const int8_t *coup, const std::vector<ThrRow> &rows);
bool use_pt_split2d(const smc_desc *d, const void *spins, const std::vector<ThrRow> &rows);

// --------------------------------------------------------------- validation --
struct Plan {
    Batch b;
    int max_L = 0;
    int64_t n_samples = 0;
    std::vector<smc_inst> samples;  // distinct samples (EA): L, sample, -, coup_off
};

int64_t sites(int dim, int L);
// The coupling samples of a uniform EA batch: sample q at q * d * N.
void fill_uniform_samples(const smc_desc *d, Plan &plan);
int validate(const smc_desc *d, bool need_coup, Plan &plan);
// The instance table of an uneven batch into its scratch slot (plan.b.inst).
int upload_inst(StreamCtx &c, hipStream_t s, const smc_desc *d, Plan &plan);

// --------------------------------------------------------------- tuning ----
// Workgroup size of the LDS-resident 2D kernel for an edge without
// measurement, and with it (tune.hip): measured once per process and
// (device, edge, model) on scratch copies of the replicas reps of rows.
int uneven2d_threads_default(int L);
int uneven2d_threads(StreamCtx &c, hipStream_t s, const Uneven2dArgs &a, int L, bool ea,
                     const std::vector<int32_t> &reps, const std::vector<smc_inst> &rows, int *out);

}  // namespace smc

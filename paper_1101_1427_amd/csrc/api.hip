// C-ABI layer of libspinmc.so: argument validation, acceptance tables,
// per-stream scratch, and dispatch to the sweep / exchange kernels.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "runtime.hpp"

namespace smc {
namespace {

// ------------------------------------------------ uneven 2D tempering ----
// Batches of 2D lattices with edges in {16, 32, ..., 256} (uniform or uneven)
// go to the per-replica LDS kernel; the replicas of one edge form a class
// with its own launch shape.
struct EdgeClass {
    int L = 0, threads = 0;
    int32_t first = 0, count = 0;  // range of the work list
};

bool use_uneven2d(const smc_desc *d, const void *spins, const int8_t *coup, const std::vector<ThrRow> &rows) {
    if (d->dim != 2 || (d->model != SMC_ISING && d->model != SMC_EA)) return false;
    const char *env = getenv("SPINMC_UNEVEN2D");
    if (env && env[0] == '0') return false;
    if (((uintptr_t)spins & 15u) != 0) return false;
    if (d->model == SMC_EA && ((uintptr_t)coup & 15u) != 0) return false;
    for (const ThrRow &r : rows)
        if (r.m[1].x > 0xFFFFu || r.m[2].x > 0xFFFFu) return false;
    if (d->L > 0) return uneven2d_edge_supported(d->L);
    for (int r = 0; r < d->n_rep; ++r) {
        const smc_inst &g = d->inst[r];
        if (!uneven2d_edge_supported(g.L) || g.spin_off % 16) return false;
        if (d->model == SMC_EA && g.coup_off % 16) return false;
    }
    return true;
}

std::vector<smc_inst> inst_rows(const smc_desc *d) {
    std::vector<smc_inst> rows(d->n_rep);
    const int64_t N = (int64_t)d->L * d->L;
    for (int r = 0; r < d->n_rep; ++r) {
        if (d->L > 0) {
            rows[r].L = d->L;
            rows[r].sample = d->model == SMC_EA ? r / d->rep_per_sample : 0;
            rows[r].spin_off = (int64_t)r * N;
            rows[r].coup_off = (int64_t)rows[r].sample * 2 * N;
        } else {
            rows[r] = d->inst[r];
        }
    }
    return rows;
}

// What the LDS-resident 2D kernel needs for a batch: the instance table, the
// replicas grouped by edge (classes, largest first; replica order within a
// class) and the colour-split couplings of every sample.
struct Lds2dSetup {
    std::vector<smc_inst> rows;
    std::vector<EdgeClass> classes;
    std::vector<int32_t> work;
    void *inst_dev = nullptr;
    void *work_dev = nullptr;
    uint8_t *csplit = nullptr;
};

int lds2d_setup(StreamCtx &c, hipStream_t s, const smc_desc *desc, const Plan &plan, const int8_t *couplings,
                Lds2dSetup &st) {
    int rc;
    st.rows = inst_rows(desc);
    if ((rc = upload(c, s, kInst, st.rows.data(), sizeof(smc_inst) * st.rows.size(), &st.inst_dev))) return rc;
    std::map<int, std::vector<int32_t>, std::greater<int>> by_edge;
    for (int r = 0; r < desc->n_rep; ++r) by_edge[st.rows[r].L].push_back(r);
    for (auto &kv : by_edge) {
        EdgeClass e;
        e.L = kv.first;
        e.threads = 0;  // chosen by the caller
        e.first = (int32_t)st.work.size();
        e.count = (int32_t)kv.second.size();
        st.work.insert(st.work.end(), kv.second.begin(), kv.second.end());
        st.classes.push_back(e);
        SMC_HIP(uneven2d_prepare_kernel(desc->model == SMC_EA, e.L));
    }
    if ((rc = upload(c, s, kWork, st.work.data(), sizeof(int32_t) * st.work.size(), &st.work_dev))) return rc;
    if (desc->model == SMC_EA) {
        std::vector<smc_inst> samples;
        if (desc->L > 0) {
            samples.resize((size_t)plan.n_samples);
            for (int64_t q = 0; q < plan.n_samples; ++q)
                samples[(size_t)q] = smc_inst{desc->L, (int32_t)q, 0, q * 2 * (int64_t)desc->L * desc->L};
        } else {
            std::map<int32_t, smc_inst> seen;
            for (const smc_inst &g : st.rows) seen.emplace(g.sample, g);
            for (auto &kv : seen) samples.push_back(kv.second);
        }
        std::vector<int64_t> start(samples.size());
        int64_t total = 0;
        for (size_t k = 0; k < samples.size(); ++k) {
            start[k] = total;
            total += 2 * (int64_t)samples[k].L * samples[k].L / 16;
        }
        void *samp_dev = nullptr, *start_dev = nullptr, *cs = nullptr;
        if ((rc = upload(c, s, kSamples, samples.data(), sizeof(smc_inst) * samples.size(), &samp_dev))) return rc;
        if ((rc = upload(c, s, kChunks, start.data(), sizeof(int64_t) * start.size(), &start_dev))) return rc;
        if ((rc = ensure(c, kCoupSplit, (size_t)desc->coup_len, &cs))) return rc;
        st.csplit = (uint8_t *)cs;
        SMC_HIP(launch_coup_split2d(couplings, st.csplit, (const smc_inst *)samp_dev, (int)samples.size(), total,
                                    (const int64_t *)start_dev, s));
    }
    return SMC_OK;
}

int run_uneven2d(StreamCtx &c, hipStream_t s, const smc_desc *desc, const Plan &plan, const smc_pt_desc *pt,
                 void *spins, const int8_t *couplings, SwapArgs &sw, const ThrRow *thr, double *energy,
                 uint64_t step0, int32_t n_steps, int m) {
    int rc;
    Lds2dSetup st;
    if ((rc = lds2d_setup(c, s, desc, plan, couplings, st))) return rc;
    std::vector<EdgeClass> &classes = st.classes;
    const std::vector<int32_t> &work = st.work;
    const std::vector<smc_inst> &rows = st.rows;
    void *inst_dev = st.inst_dev, *work_dev = st.work_dev;
    uint8_t *csplit = st.csplit;
    // device counters: the step index (exchange rounds) and, with m > 1
    // sweeps per step, the sweep index t*m + j (with m = 1 they coincide)
    void *tp = nullptr;
    if ((rc = ensure(c, kStep, 2 * sizeof(uint32_t), &tp))) return rc;
    uint32_t *t_dev = (uint32_t *)tp;
    uint32_t *sweep_dev = m > 1 ? t_dev + 1 : t_dev;
    SMC_HIP(launch_set_step(t_dev, (uint32_t)step0, s));
    if (m > 1) SMC_HIP(launch_set_step(sweep_dev, (uint32_t)(step0 * (uint64_t)m), s));
    sw.t_dev = t_dev;
    SMC_HIP(launch_pt_prepare(sw, energy, s));
    // every sweep launch runs the m sweeps of a step with the replica in LDS
    Uneven2dArgs a = make_uneven2d_args((int8_t *)spins, (const smc_inst *)inst_dev, csplit, sw.row_of_rep, thr,
                                        sw.E, sweep_dev, make_key(desc->seed));
    const int32_t *wl = (const int32_t *)work_dev;
    const bool ea = desc->model == SMC_EA;
    for (auto &e : classes) {
        const std::vector<int32_t> reps(work.begin() + e.first, work.begin() + e.first + e.count);
        if ((rc = uneven2d_threads(c, s, a, e.L, ea, reps, rows, &e.threads))) return rc;
    }
    a.sweeps = m;

    if (n_steps < 4) {
        // a few steps: plain launches in step order
        for (int32_t k = 0; k < n_steps; ++k) {
            for (const EdgeClass &e : classes)
                SMC_HIP(launch_uneven2d_sweep(a, wl + e.first, e.count, e.L, ea, e.threads, s));
            SMC_HIP(launch_pt_swap(sw, s));
            if (m > 1) SMC_HIP(launch_advance_step(sweep_dev, s, (uint32_t)m));
            SMC_HIP(launch_advance_step(t_dev, s));
        }
    } else {
        // a graph of K steps: per step the edge classes run as parallel
        // branches (m sweeps each), then the exchange round, then (m > 1) the
        // sweep counter, then the step counter
        const int32_t K = n_steps < 32 ? n_steps : 32;
        const int32_t reps = n_steps / K, rest = n_steps % K;
        for (int which = 0; which < 2; ++which) {
            const int32_t steps = which == 0 ? K : rest;
            if (steps == 0) continue;
            std::vector<uint64_t> sig = {(uint64_t)steps, (uint64_t)(uintptr_t)a.spins, (uint64_t)(uintptr_t)a.inst,
                                         (uint64_t)(uintptr_t)a.csplit, (uint64_t)(uintptr_t)a.row_of_rep,
                                         (uint64_t)(uintptr_t)a.thr, (uint64_t)(uintptr_t)a.E,
                                         (uint64_t)(uintptr_t)t_dev, a.key.k0, a.key.k1, (uint64_t)(uintptr_t)wl,
                                         (uint64_t)(uintptr_t)sw.beta, (uint64_t)(uintptr_t)sw.slot_of_temp,
                                         (uint64_t)(uintptr_t)sw.acc, (uint64_t)sw.n_chains, (uint64_t)sw.n_temps,
                                         (uint64_t)sw.beta_per_chain, (uint64_t)m};
            for (const EdgeClass &e : classes) {
                sig.push_back((uint64_t)e.L);
                sig.push_back((uint64_t)e.threads);
                sig.push_back((uint64_t)e.first);
                sig.push_back((uint64_t)e.count);
            }
            GraphCache &gc = c.graphs[which];
            if (gc.exec == nullptr || gc.sig != sig) {
                if (gc.exec) {
                    SMC_HIP(hipStreamSynchronize(s));  // the old executable may still be in flight
                    SMC_HIP(hipGraphExecDestroy(gc.exec));
                    gc.exec = nullptr;
                }
                hipGraph_t g = nullptr;
                SMC_HIP(hipGraphCreate(&g, 0));
                hipError_t e = hipSuccess;
                hipGraphNode_t prev = nullptr;
                std::vector<hipGraphNode_t> sweeps(classes.size());
                for (int32_t k = 0; k < steps && e == hipSuccess; ++k) {
                    for (size_t q = 0; q < classes.size() && e == hipSuccess; ++q) {
                        const EdgeClass &ec = classes[q];
                        e = add_uneven2d_sweep_node(g, &sweeps[q], prev ? &prev : nullptr, prev ? 1 : 0, a,
                                                    wl + ec.first, ec.count, ec.L, ea, ec.threads);
                    }
                    hipGraphNode_t swap = nullptr, after = nullptr;
                    if (e == hipSuccess) e = add_pt_swap_node(g, &swap, sweeps.data(), sweeps.size(), sw);
                    after = swap;
                    if (m > 1 && e == hipSuccess) e = add_advance_node(g, &after, &swap, 1, sweep_dev, (uint32_t)m);
                    if (e == hipSuccess) e = add_advance_node(g, &prev, &after, 1, t_dev);
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&gc.exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    gc.exec = nullptr;
                    return fail(SMC_EHIP, "building the tempering graph: %s", hipGetErrorString(e));
                }
                gc.sig = sig;
            }
            const int32_t launches = which == 0 ? reps : 1;
            for (int32_t k = 0; k < launches; ++k) SMC_HIP(hipGraphLaunch(gc.exec, s));
        }
    }
    SMC_HIP(launch_pt_finish(sw, energy, s));
    return SMC_OK;
}

// Event pairs around the sweep kernels of each call (profiling aid).
struct TimedCall {
    hipEvent_t start, stop;
    int64_t launches;
};
std::mutex g_timing_mutex;
bool g_timing_on = false;
std::vector<TimedCall> g_timed;

void forget_timed() {
    for (TimedCall &c : g_timed) {
        (void)hipEventDestroy(c.start);
        (void)hipEventDestroy(c.stop);
    }
    g_timed.clear();
}

// Records the start event on construction and the stop event on finish().
struct SweepTimer {
    hipStream_t s;
    TimedCall call{nullptr, nullptr, 0};
    bool on = false;
    SweepTimer(hipStream_t stream, int64_t launches) : s(stream) {
        std::lock_guard<std::mutex> lk(g_timing_mutex);
        if (!g_timing_on) return;
        call.launches = launches;
        if (hipEventCreate(&call.start) != hipSuccess) return;
        if (hipEventCreate(&call.stop) != hipSuccess) {
            (void)hipEventDestroy(call.start);
            return;
        }
        on = hipEventRecord(call.start, s) == hipSuccess;
        if (!on) {
            (void)hipEventDestroy(call.start);
            (void)hipEventDestroy(call.stop);
        }
    }
    void finish() {
        if (!on) return;
        on = false;
        std::lock_guard<std::mutex> lk(g_timing_mutex);
        if (hipEventRecord(call.stop, s) == hipSuccess && g_timing_on) {
            g_timed.push_back(call);
        } else {
            (void)hipEventDestroy(call.start);
            (void)hipEventDestroy(call.stop);
        }
    }
    ~SweepTimer() { finish(); }
};

// Sweeps of a uniform 2D Ising / EA batch of edge 16 .. 256 (a multiple of
// 16) on the LDS-resident kernel: each replica stays in one workgroup's LDS
// for up to kLdsSweeps sweeps per launch, so small lattices are not bound
// by two launches per sweep.  Same results as the generic kernels;
// SPINMC_SWEEP_LDS2D=0 sends such batches to them.
constexpr int kLdsSweeps = 256;

// A workgroup sweeps about 6e9 sites per second, so one replica of edge 256
// (65536 sites) takes longer in one workgroup than the generic kernels take
// over the whole chip; above edge 128 the batch must hold at least 2^19 sites.
bool lds2d_sweep_shape(const smc_desc *d) {
    const char *env = getenv("SPINMC_SWEEP_LDS2D");
    if (env && env[0] == '0') return false;
    if (d->dim != 2 || d->L <= 0 || !uneven2d_edge_supported(d->L)) return false;
    return d->L <= 128 || (int64_t)d->n_rep * d->L * d->L >= (int64_t)1 << 19;
}

bool use_sweep_lds2d(const smc_desc *d, const void *spins, const int8_t *coup, const std::vector<ThrRow> &rows) {
    return lds2d_sweep_shape(d) && use_uneven2d(d, spins, coup, rows);
}

int run_sweep_lds2d(StreamCtx &c, hipStream_t s, const smc_desc *desc, const Plan &plan, void *spins,
                    const int8_t *couplings, const ThrRow *thr, int64_t *dE_accum, uint64_t sweep0,
                    int32_t n_sweeps) {
    int rc;
    Lds2dSetup st;
    if ((rc = lds2d_setup(c, s, desc, plan, couplings, st))) return rc;
    // threshold row of replica r: row r; energy changes into dE_accum (or scratch)
    std::vector<int32_t> ident(desc->n_rep);
    for (int r = 0; r < desc->n_rep; ++r) ident[r] = r;
    void *rp = nullptr, *ep = nullptr, *tp = nullptr;
    if ((rc = upload(c, s, kRows, ident.data(), sizeof(int32_t) * ident.size(), &rp))) return rc;
    int64_t *E = dE_accum;
    if (!E) {
        if ((rc = ensure(c, kEnergy64, sizeof(int64_t) * desc->n_rep, &ep))) return rc;
        E = (int64_t *)ep;
    }
    if ((rc = ensure(c, kStep, 2 * sizeof(uint32_t), &tp))) return rc;
    uint32_t *t_dev = (uint32_t *)tp;
    SMC_HIP(launch_set_step(t_dev, (uint32_t)sweep0, s));
    Uneven2dArgs a = make_uneven2d_args((int8_t *)spins, (const smc_inst *)st.inst_dev, st.csplit,
                                        (const int32_t *)rp, thr, E, t_dev, make_key(desc->seed));
    const bool ea = desc->model == SMC_EA;
    for (auto &e : st.classes) {
        const std::vector<int32_t> reps(st.work.begin() + e.first, st.work.begin() + e.first + e.count);
        if ((rc = uneven2d_threads(c, s, a, e.L, ea, reps, st.rows, &e.threads))) return rc;
    }
    const int32_t *wl = (const int32_t *)st.work_dev;
    const int64_t launches = ((int64_t)n_sweeps + kLdsSweeps - 1) / kLdsSweeps * (int64_t)st.classes.size();
    SweepTimer timer(s, launches);
    for (int32_t done = 0; done < n_sweeps;) {
        const int32_t chunk = n_sweeps - done < kLdsSweeps ? n_sweeps - done : kLdsSweeps;
        a.sweeps = chunk;
        for (const EdgeClass &e : st.classes)
            SMC_HIP(launch_uneven2d_sweep(a, wl + e.first, e.count, e.L, ea, e.threads, s));
        done += chunk;
        if (done < n_sweeps) SMC_HIP(launch_advance_step(t_dev, s, (uint32_t)chunk));
    }
    timer.finish();
    return SMC_OK;
}

}  // namespace
}  // namespace smc

using namespace smc;

extern "C" {

const char *smc_strerror(int status) {
    switch (status) {
        case SMC_OK: return "success";
        case SMC_EINVAL: return "invalid argument";
        case SMC_EUNSUPPORTED: return "unsupported combination of arguments";
        case SMC_EHIP: return "HIP runtime error";
        case SMC_ENOMEM: return "out of device memory for scratch";
        default: return "unknown status";
    }
}

const char *smc_last_error(void) { return last_error().c_str(); }

int smc_kernel_timing_enable(int enable) {
    std::lock_guard<std::mutex> lk(g_timing_mutex);
    g_timing_on = enable != 0;
    if (!g_timing_on) forget_timed();
    return SMC_OK;
}

int smc_philox_bench(uint64_t seed, uint32_t t, uint32_t r, uint32_t tag, int32_t n_threads, int32_t per_thread,
                     uint32_t *out, void *stream) {
    last_error().clear();
    if (!out) return fail(SMC_EINVAL, "out is NULL");
    if (n_threads <= 0 || per_thread <= 0) return fail(SMC_EINVAL, "n_threads and per_thread must be positive");
    if ((int64_t)n_threads * per_thread > (int64_t)1 << 32)
        return fail(SMC_EINVAL, "n_threads * per_thread exceeds 2^32");
    SMC_HIP(launch_philox_bench(make_key(seed), t, r, tag, (uint32_t)n_threads, per_thread, out,
                                (hipStream_t)stream));
    return SMC_OK;
}

int smc_kernel_timing_read(double *elapsed_ms, int64_t *launches) {
    last_error().clear();
    if (!elapsed_ms || !launches) return fail(SMC_EINVAL, "output pointers are required");
    std::lock_guard<std::mutex> lk(g_timing_mutex);
    double ms = 0.0;
    int64_t n = 0;
    int rc = SMC_OK;
    for (TimedCall &c : g_timed) {
        float part = 0.0f;
        hipError_t e = hipEventSynchronize(c.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&part, c.start, c.stop);
        if (e != hipSuccess) {
            rc = fail(SMC_EHIP, "%s", hipGetErrorString(e));
            break;
        }
        ms += part;
        n += c.launches;
    }
    forget_timed();
    *elapsed_ms = ms;
    *launches = n;
    return rc;
}

int smc_sweep_plan(const smc_desc *desc, int32_t *launches_per_sweep, const char **kernel_name) {
    last_error().clear();
    Plan plan;
    int rc = validate(desc, false, plan);
    if (rc) return rc;
    if (!launches_per_sweep || !kernel_name) return fail(SMC_EINVAL, "output pointers are required");
    if (desc->model == SMC_HEISENBERG) {
        *launches_per_sweep = 2;
        if (use_heis3d_tiled(desc)) {
            *launches_per_sweep = 1;
            *kernel_name = "k_heis3d_tiled";
        } else {
            *kernel_name = use_heis3d(desc) ? "k_heis3d_half" : "k_heis_half_sweep_generic";
        }
    } else if (desc->model == SMC_ISING && desc->dim == 2 && desc->L > 0 && lattice2d_supported(desc->L)) {
        *launches_per_sweep = 1;
        *kernel_name = "k_ising2d_split";
    } else if (sweep3d_shape(desc)) {
        const bool pass = pass3d_enabled(desc);
        *launches_per_sweep = pass ? 1 : 2;
        *kernel_name = pass ? "k_ising3d_pass" : "k_ising3d_half";
    } else if (lds2d_sweep_shape(desc) && !(getenv("SPINMC_UNEVEN2D") && getenv("SPINMC_UNEVEN2D")[0] == '0')) {
        *launches_per_sweep = 1;  // at most: up to 256 sweeps per launch
        *kernel_name = "k_uneven2d_sweep";
    } else {
        *launches_per_sweep = 2;
        *kernel_name = "k_half_sweep_generic";
    }
    return SMC_OK;
}

int smc_pt_plan(const smc_desc *desc, const smc_pt_desc *pt, int32_t n_steps, int32_t *launches,
                const char **kernel_name) {
    last_error().clear();
    Plan plan;
    int rc = validate(desc, false, plan);
    if (rc) return rc;
    if (!pt || !launches || !kernel_name) return fail(SMC_EINVAL, "pt desc and output pointers are required");
    if (n_steps < 0) return fail(SMC_EINVAL, "n_steps must be >= 0");
    if (pt->n_temps < 2 || !pt->beta) return fail(SMC_EINVAL, "need n_temps >= 2 and beta");
    if (pt->sweeps_per_step < 0) return fail(SMC_EINVAL, "sweeps_per_step must be >= 0");
    const int m = pt->sweeps_per_step > 0 ? pt->sweeps_per_step : 1;
    const int rows_n = pt->beta_per_chain ? pt->n_chains : 1;
    std::vector<ThrRow> all_rows((size_t)rows_n * pt->n_temps);
    for (size_t k = 0; k < all_rows.size(); ++k) all_rows[k] = threshold_row(pt->beta[k], desc->dim);
    bool fits = pt3d_enabled() && pt3d_supported(desc, pt->n_temps);
    for (int64_t k = 0; fits && k < (int64_t)rows_n * pt->n_temps; ++k) {
        const ThrRow r = threshold_row(pt->beta[k], desc->dim);
        fits = r.m[1].x <= 0xFFFFu && r.m[2].x <= 0xFFFFu && r.m[3].x <= 0xFFFFu;
    }
    bool fits2d = !fits && desc->dim == 2 && (desc->model == SMC_ISING || desc->model == SMC_EA);
    if (fits2d) {
        const char *env = getenv("SPINMC_UNEVEN2D");
        if (env && env[0] == '0') fits2d = false;
        for (int r = 0; fits2d && desc->L == 0 && r < desc->n_rep; ++r)
            fits2d = uneven2d_edge_supported(desc->inst[r].L) && desc->inst[r].spin_off % 16 == 0 &&
                     (desc->model != SMC_EA || desc->inst[r].coup_off % 16 == 0);
        if (desc->L > 0) fits2d = uneven2d_edge_supported(desc->L);
        for (int64_t k = 0; fits2d && k < (int64_t)rows_n * pt->n_temps; ++k) {
            const ThrRow r = threshold_row(pt->beta[k], desc->dim);
            fits2d = r.m[1].x <= 0xFFFFu && r.m[2].x <= 0xFFFFu;
        }
    }
    if (fits) {
        *launches = n_steps > 0 ? 1 : 0;
        *kernel_name = "k_pt3d_chain";
    } else if (use_pt_split2d(desc, (const void *)nullptr, all_rows)) {
        // prepare, zero, to split; per step: thresholds, m sweeps, collect, add, exchange; from split, copy, finish
        *launches = n_steps > 0 ? 6 + n_steps * (m + 4) : 0;
        *kernel_name = "k_ising2d_split";
    } else if (fits2d) {
        // set step(s), prepare, (coupling split), graph launches of up to 32 steps, finish
        const int32_t K = n_steps < 32 ? n_steps : 32;
        const int32_t graphs = n_steps < 4 ? 0 : n_steps / K + (n_steps % K ? 1 : 0);
        const int32_t direct = n_steps < 4 ? n_steps * (int32_t)(2 + 7) : 0;
        *launches = n_steps > 0 ? 3 + (desc->model == SMC_EA ? 1 : 0) + graphs + direct : 0;
        *kernel_name = "k_uneven2d_sweep";
    } else {
        *launches = n_steps > 0 ? (2 * m + 1) * n_steps + 2 : 0;
        *kernel_name = "k_half_sweep_generic";
    }
    return SMC_OK;
}

int smc_spin_init(const smc_desc *desc, void *spins, int8_t *couplings, void *stream) {
    last_error().clear();
    Plan plan;
    const bool want_coup = desc && desc->model == SMC_EA && couplings;
    int rc = validate(desc, want_coup, plan);
    if (rc) return rc;
    if (!spins) return fail(SMC_EINVAL, "spins is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    StreamCtx &c = ctx_for(s);
    if ((rc = upload_inst(c, s, desc, plan))) return rc;
    const Key key = make_key(desc->seed);
    if (desc->model == SMC_HEISENBERG) {
        SMC_HIP(launch_init_heis(plan.b, plan.max_L, (float *)spins, key, s));
    } else {
        SMC_HIP(launch_init_spins(plan.b, plan.max_L, (int8_t *)spins, key, s));
    }
    if (want_coup && plan.n_samples > 0) {
        fill_uniform_samples(desc, plan);
        void *p = nullptr;
        if ((rc = upload(c, s, kSamples, plan.samples.data(), sizeof(smc_inst) * plan.samples.size(), &p))) return rc;
        int maxL = 0;
        for (auto &g : plan.samples) maxL = g.L > maxL ? g.L : maxL;
        SMC_HIP(launch_init_couplings(desc->dim, (int)plan.n_samples, (const smc_inst *)p, maxL, couplings, key, s));
    }
    return SMC_OK;
}

// ------------------------------------- asynchronous multi-spin coding ----
// Replicas 32g .. 32g+31 form group g and share its Metropolis draws.
int msc_check(const smc_desc *d, int word_bits) {
    if (d->model != SMC_ISING && d->model != SMC_EA)
        return fail(SMC_EUNSUPPORTED, "multi-spin coding is provided for the Ising and EA models");
    if (word_bits != 32 && word_bits != 64) return fail(SMC_EINVAL, "word_bits must be 32 or 64 (got %d)", word_bits);
    if (d->L <= 0) return fail(SMC_EINVAL, "multi-spin coding needs a uniform batch (L > 0)");
    if (d->n_rep % word_bits != 0)
        return fail(SMC_EINVAL, "n_rep (%d) must be a multiple of %d", d->n_rep, word_bits);
    if (d->model == SMC_EA && d->rep_per_sample != 1)
        return fail(SMC_EINVAL, "multi-spin coding needs one coupling sample per replica (rep_per_sample = 1)");
    return SMC_OK;
}

// The packed kernel serves 2D batches of edge 16, 32 or 64 with 4-byte
// aligned spins and couplings (SPINMC_MSC2D=0 sends them to the generic
// kernels, which give the same results).
bool use_msc2d(const smc_desc *d, const void *spins, const void *coup) {
    const char *env = getenv("SPINMC_MSC2D");
    if (env && env[0] == '0') return false;
    if (((uintptr_t)spins & 3u) || ((uintptr_t)coup & 3u)) return false;
    return msc2d_supported(d->dim, d->L);
}

int smc_metropolis_sweep(const smc_desc *desc, void *spins, const int8_t *couplings, const double *beta,
                         uint64_t sweep0, int32_t n_sweeps, int64_t *dE_accum, void *stream) {
    last_error().clear();
    Plan plan;
    int rc = validate(desc, true, plan);
    if (rc) return rc;
    if (!spins) return fail(SMC_EINVAL, "spins is NULL");
    if (!beta) return fail(SMC_EINVAL, "beta is NULL");
    if (desc->model == SMC_EA && !couplings) return fail(SMC_EINVAL, "couplings are required for EA");
    if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
    if (sweep0 + (uint64_t)n_sweeps > (1ull << 32)) return fail(SMC_EINVAL, "sweep index exceeds 32 bits");
    for (int r = 0; r < desc->n_rep; ++r)
        if (!(beta[r] >= 0.0) || !isfinite(beta[r])) return fail(SMC_EINVAL, "beta[%d] must be finite and >= 0", r);
    if (n_sweeps == 0) return SMC_OK;
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    StreamCtx &c = ctx_for(s);
    if ((rc = upload_inst(c, s, desc, plan))) return rc;

    SweepArgs a;
    memset(&a, 0, sizeof a);
    a.b = plan.b;
    a.spins = spins;
    a.coup = desc->model == SMC_EA ? couplings : nullptr;
    a.key = make_key(desc->seed);
    a.dE = dE_accum;
    a.max_L = plan.max_L;
    a.row_of_rep = nullptr;
    void *p = nullptr;
    if (desc->model == SMC_HEISENBERG) {
        std::vector<float> bf(desc->n_rep);
        for (int r = 0; r < desc->n_rep; ++r) bf[r] = (float)beta[r];
        if ((rc = upload(c, s, kTables, bf.data(), sizeof(float) * bf.size(), &p))) return rc;
        a.beta_f = (const float *)p;
        if (use_heis3d_tiled(desc)) {
            // one-pass sweeps, ping-pong between the caller's buffer and a scratch copy
            const size_t bytes = (size_t)desc->n_rep * 3 * sizeof(float) * (size_t)plan.b.N;
            void *pp = nullptr;
            if ((rc = ensure(c, kHeisPing, bytes, &pp))) return rc;
            float *A = (float *)spins, *B = (float *)pp;
            SweepTimer timer(s, n_sweeps);
            for (int32_t k = 0; k < n_sweeps; ++k) {
                a.t = (uint32_t)(sweep0 + (uint64_t)k);
                float *src = k & 1 ? B : A, *dst = k & 1 ? A : B;
                // the renormalisation is applied as the sweep stores its spins
                const bool renorm =
                    desc->renorm_every > 0 && ((uint64_t)a.t + 1) % (uint64_t)desc->renorm_every == 0;
                SMC_HIP(launch_heis3d_tiled(src, dst, a.beta_f, dE_accum, desc->n_rep, desc->L, a.key, a.t, renorm,
                                            s));
            }
            timer.finish();
            if (n_sweeps & 1) SMC_HIP(hipMemcpyAsync(A, B, bytes, hipMemcpyDeviceToDevice, s));
            return SMC_OK;
        }
        SweepTimer timer(s, 2 * (int64_t)n_sweeps);  // the renormalisations run inside the same pair
        const bool fast = use_heis3d(desc);
        for (int32_t k = 0; k < n_sweeps; ++k) {
            a.t = (uint32_t)(sweep0 + (uint64_t)k);
            for (int col = 0; col < 2; ++col) {
                if (fast)
                    SMC_HIP(launch_heis3d_half((float *)spins, a.beta_f, dE_accum, desc->n_rep, desc->L, a.key, a.t,
                                               col, s));
                else
                    SMC_HIP(launch_heis_half_sweep_generic(a, col, s));
            }
            if (desc->renorm_every > 0 && ((uint64_t)a.t + 1) % (uint64_t)desc->renorm_every == 0)
                SMC_HIP(launch_heis_renorm(plan.b, (float *)spins, plan.max_L, s));
        }
        return SMC_OK;
    }
    std::vector<ThrRow> rows(desc->n_rep);
    for (int r = 0; r < desc->n_rep; ++r) rows[r] = threshold_row(beta[r], desc->dim);
    if ((rc = upload(c, s, kTables, rows.data(), sizeof(ThrRow) * rows.size(), &p))) return rc;
    a.thr = (const ThrRow *)p;
    if (use_sweep_lds2d(desc, spins, couplings, rows))
        return run_sweep_lds2d(c, s, desc, plan, spins, couplings, a.thr, dE_accum, sweep0, n_sweeps);
    if (use_lattice2d(desc, spins, rows)) {
        // one-pass sweeps on the colour-split layout, ping-pong between two buffers
        const size_t bytes = (size_t)desc->n_rep * lattice2d_split_bytes(desc->L);
        void *pp = nullptr;
        if ((rc = ensure(c, kPingPong, 2 * bytes, &pp))) return rc;
        uint8_t *A = (uint8_t *)pp, *B = A + bytes;
        // energy changes: per-wave partial sums over the call, collected once at the end
        int64_t *part = nullptr;
        if (dE_accum) {
            void *q = nullptr;
            const size_t slots = lattice2d_de_slots(desc->L, desc->n_rep);
            if (slots == 0) return fail(SMC_EINVAL, "no band shape for L=%d", desc->L);
            if ((rc = ensure(c, kL2dPart, slots * sizeof(int64_t), &q))) return rc;
            part = (int64_t *)q;
        }
        const char *fuse_env = getenv("SPINMC_L2D_FUSE");
        if (fuse_env && fuse_env[0] == '0') {
            // separate layout conversions around the sweeps (for comparison)
            SMC_HIP(launch_to_split((const int8_t *)spins, A, desc->L, desc->n_rep, s));
            SweepTimer timer(s, n_sweeps);
            for (int32_t k = 0; k < n_sweeps; ++k) {
                const uint32_t t = (uint32_t)(sweep0 + (uint64_t)k);
                SMC_HIP(launch_ising2d_split(k & 1 ? B : A, false, k & 1 ? A : B, false, desc->L, desc->n_rep,
                                             a.thr, part, k == 0, a.key, t, s));
            }
            timer.finish();
            if (part) SMC_HIP(launch_lattice2d_de_collect(part, dE_accum, desc->L, desc->n_rep, s));
            SMC_HIP(launch_from_split(n_sweeps & 1 ? B : A, (int8_t *)spins, desc->L, desc->n_rep, s));
            return SMC_OK;
        }
        // The first sweep reads the caller's lattice, the last one writes it
        // back; the sweeps between ping-pong on the split layout (sweep k
        // leaves its result in A for even k, in B for odd k).  A single sweep
        // ends in A and is converted back.
        SweepTimer timer(s, n_sweeps);
        for (int32_t k = 0; k < n_sweeps; ++k) {
            const uint32_t t = (uint32_t)(sweep0 + (uint64_t)k);
            const bool first = k == 0, last = k == n_sweeps - 1 && n_sweeps > 1;
            const void *src = first ? spins : (k & 1 ? (const void *)A : (const void *)B);
            void *dst = last ? spins : (k & 1 ? (void *)B : (void *)A);
            SMC_HIP(launch_ising2d_split(src, first, dst, last, desc->L, desc->n_rep, a.thr, part, first, a.key, t,
                                         s));
        }
        timer.finish();
        if (part) SMC_HIP(launch_lattice2d_de_collect(part, dE_accum, desc->L, desc->n_rep, s));
        if (n_sweeps == 1) SMC_HIP(launch_from_split(A, (int8_t *)spins, desc->L, desc->n_rep, s));
        return SMC_OK;
    }
    if (use_sweep3d(desc, spins, a.coup, rows)) {
        // EA calls of several sweeps read the bonds bit-packed (one pass to
        // pack them: 3 B per site per sample in, 0.5 B out; the int8 bonds
        // cost 3 B per site and launch); SPINMC_SWEEP3D_PACK=0 keeps the int8 bonds
        const int8_t *coup8 = a.coup;
        const uint2 *packed = nullptr;
        const char *env = getenv("SPINMC_SWEEP3D_PACK");
        const bool pass = pass3d_enabled(desc);
        if (a.coup && (pass || (n_sweeps >= 4 && !(env && env[0] == '0')))) {
            void *q = nullptr;
            if ((rc = ensure(c, kBonds3d, (size_t)plan.n_samples * (size_t)(plan.b.N / 16) * sizeof(uint2), &q)))
                return rc;
            packed = (const uint2 *)q;
            coup8 = nullptr;
            SMC_HIP(launch_pack_bonds3d(a.coup, (uint2 *)q, desc->L, (int)plan.n_samples, s));
        }
        if (pass) {
            // one launch per sweep, ping-pong between the caller's lattice and
            // a second buffer; an odd count ends with one copy back
            const size_t bytes = (size_t)desc->n_rep * (size_t)plan.b.N;
            void *q = nullptr;
            if ((rc = ensure(c, kPass3d, bytes, &q))) return rc;
            int8_t *A = (int8_t *)spins, *B = (int8_t *)q;
            SweepTimer timer(s, n_sweeps);
            for (int32_t k = 0; k < n_sweeps; ++k) {
                const uint32_t t = (uint32_t)(sweep0 + (uint64_t)k);
                SMC_HIP(launch_ising3d_pass(k & 1 ? B : A, k & 1 ? A : B, packed, plan.b.rep_per_sample, a.thr,
                                            dE_accum, desc->n_rep, desc->L, a.key, t, s));
            }
            timer.finish();
            if (n_sweeps & 1) SMC_HIP(hipMemcpyAsync(A, B, bytes, hipMemcpyDeviceToDevice, s));
            return SMC_OK;
        }
        SweepTimer timer(s, 2 * (int64_t)n_sweeps);
        for (int32_t k = 0; k < n_sweeps; ++k) {
            const uint32_t t = (uint32_t)(sweep0 + (uint64_t)k);
            for (int col = 0; col < 2; ++col)
                SMC_HIP(launch_ising3d_half((int8_t *)spins, coup8, packed, plan.b.rep_per_sample, a.thr, dE_accum,
                                            desc->n_rep, desc->L, a.key, t, col, s));
        }
        return SMC_OK;
    }
    SweepTimer timer(s, 2 * (int64_t)n_sweeps);
    for (int32_t k = 0; k < n_sweeps; ++k) {
        a.t = (uint32_t)(sweep0 + (uint64_t)k);
        SMC_HIP(launch_half_sweep_generic(a, 0, s));
        SMC_HIP(launch_half_sweep_generic(a, 1, s));
    }
    return SMC_OK;
}

int smc_msc_sweep(const smc_desc *desc, void *spins, const int8_t *couplings, const double *beta, uint64_t sweep0,
                  int32_t n_sweeps, int32_t word_bits, int64_t *dE_accum, void *stream) {
    last_error().clear();
    Plan plan;
    int rc = validate(desc, true, plan);
    if (rc) return rc;
    if ((rc = msc_check(desc, word_bits))) return rc;
    if (!spins) return fail(SMC_EINVAL, "spins is NULL");
    if (!beta) return fail(SMC_EINVAL, "beta is NULL");
    if (desc->model == SMC_EA && !couplings) return fail(SMC_EINVAL, "couplings are required for EA");
    if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
    if (sweep0 + (uint64_t)n_sweeps > (1ull << 32)) return fail(SMC_EINVAL, "sweep index exceeds 32 bits");
    for (int r = 0; r < desc->n_rep; ++r) {
        if (!(beta[r] >= 0.0) || !isfinite(beta[r])) return fail(SMC_EINVAL, "beta[%d] must be finite and >= 0", r);
        if (beta[r] != beta[r - r % word_bits])
            return fail(SMC_EINVAL, "beta[%d] differs from the rest of its group of %d", r, word_bits);
    }
    if (n_sweeps == 0) return SMC_OK;
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    StreamCtx &c = ctx_for(s);
    if ((rc = upload_inst(c, s, desc, plan))) return rc;
    const int G = desc->n_rep / 32;
    const bool ea = desc->model == SMC_EA;
    if (use_msc2d(desc, spins, ea ? couplings : nullptr)) {
        const int64_t N = (int64_t)desc->L * desc->L;
        std::vector<ThrRow> rows(G);
        for (int g = 0; g < G; ++g)
            rows[g] = (g > 0 && beta[32 * g] == beta[32 * (g - 1)]) ? rows[g - 1] : threshold_row(beta[32 * g], desc->dim);
        void *tp = nullptr, *sp = nullptr, *cp = nullptr, *ep = nullptr, *mp = nullptr;
        if ((rc = upload(c, s, kTables, rows.data(), sizeof(ThrRow) * rows.size(), &tp))) return rc;
        if ((rc = ensure(c, kMscSpins, sizeof(uint32_t) * (size_t)(G * N), &sp))) return rc;
        if ((rc = ensure(c, kMscCoup, sizeof(uint32_t) * (size_t)(G * 2 * N), &cp))) return rc;
        void *gp = nullptr;
        if ((rc = ensure(c, kMscGauge, sizeof(uint32_t) * (size_t)(G * N), &gp))) return rc;
        const size_t mbytes = measure_scratch_bytes(plan.b, plan.max_L);
        if (dE_accum) {
            if ((rc = ensure(c, kMscEnergy, 2 * sizeof(double) * (size_t)desc->n_rep, &ep))) return rc;
            if ((rc = ensure(c, kMeasure, mbytes, &mp))) return rc;
            SMC_HIP(launch_measure(plan.b, spins, ea ? couplings : nullptr, plan.max_L, (double *)ep, nullptr, mp,
                                   mbytes, s));
        }
        SMC_HIP(launch_msc_pack((const int8_t *)spins, (uint32_t *)sp, N, G, s));
        SMC_HIP(launch_msc_pack_coup(ea ? couplings : nullptr, (uint32_t *)cp, 2 * N, G, s));
        SMC_HIP(launch_msc_gauge2d((uint32_t *)sp, (uint32_t *)cp, (uint32_t *)gp, desc->L, G, s));
        SweepTimer timer(s, 1);  // all sweeps in one launch
        SMC_HIP(launch_msc2d((uint32_t *)sp, (const uint32_t *)cp, (const ThrRow *)tp, G, desc->L,
                             make_key(desc->seed), (uint32_t)sweep0, n_sweeps, word_bits / 32, s));
        timer.finish();
        SMC_HIP(launch_msc_unpack((const uint32_t *)sp, (const uint32_t *)gp, (int8_t *)spins, N, G, s));
        if (dE_accum) {
            double *E0 = (double *)ep, *E1 = E0 + desc->n_rep;
            SMC_HIP(launch_measure(plan.b, spins, ea ? couplings : nullptr, plan.max_L, E1, nullptr, mp, mbytes, s));
            SMC_HIP(launch_msc_energy_diff(E0, E1, dE_accum, desc->n_rep, s));
        }
        return SMC_OK;
    }
    // generic per-site kernels with the group index in the draws' counters
    std::vector<ThrRow> rows(desc->n_rep);
    for (int r = 0; r < desc->n_rep; ++r) rows[r] = threshold_row(beta[r], desc->dim);
    void *p = nullptr;
    if ((rc = upload(c, s, kTables, rows.data(), sizeof(ThrRow) * rows.size(), &p))) return rc;
    SweepArgs a;
    memset(&a, 0, sizeof a);
    a.b = plan.b;
    a.spins = spins;
    a.coup = ea ? couplings : nullptr;
    a.thr = (const ThrRow *)p;
    a.key = make_key(desc->seed);
    a.dE = dE_accum;
    a.max_L = plan.max_L;
    a.row_of_rep = nullptr;
    a.rng_shift = word_bits == 64 ? 6 : 5;  // the draw group r / word_bits
    SweepTimer timer(s, 2 * (int64_t)n_sweeps);
    for (int32_t k = 0; k < n_sweeps; ++k) {
        a.t = (uint32_t)(sweep0 + (uint64_t)k);
        SMC_HIP(launch_half_sweep_generic(a, 0, s));
        SMC_HIP(launch_half_sweep_generic(a, 1, s));
    }
    return SMC_OK;
}

// The packed double-checkerboard kernel: thresholds with 16-bit high halves,
// 16-byte aligned buffers, a power-of-two tile; SPINMC_DCB_PACKED=0 forces
// the per-site kernel (same results).
static bool use_dcb_packed(const smc_desc *d, const std::vector<ThrRow> &rows, const void *spins,
                           const int8_t *coup, int tile) {
    const char *env = getenv("SPINMC_DCB_PACKED");
    if (env && env[0] == '0') return false;
    if (d->dim != 2 || !dcb2d_packed_supported(d->L, tile)) return false;
    if (((uintptr_t)spins & 15u) || (d->model == SMC_EA && ((uintptr_t)coup & 15u))) return false;
    for (const ThrRow &r : rows)
        if (r.m[1].x > 0xFFFFu || r.m[2].x > 0xFFFFu) return false;
    return true;
}

// Checks shared by smc_dcb_sweep and smc_dcb_plan.
static int dcb_check(const smc_desc *desc, const double *beta, int tile) {
    Plan plan;
    int rc = validate(desc, true, plan);
    if (rc) return rc;
    if (desc->model != SMC_ISING && desc->model != SMC_EA)
        return fail(SMC_EUNSUPPORTED, "the double checkerboard is provided for the Ising and EA models");
    if (desc->L <= 0) return fail(SMC_EINVAL, "the double checkerboard needs a uniform batch (L > 0)");
    if (desc->dim == 2 && !dcb2d_supported(desc->L, tile))
        return fail(SMC_EINVAL, "tile %d: need a multiple of 16 in [16, 128] dividing L = %d into an even number "
                                "of tiles per row (or one)", tile, desc->L);
    if (desc->dim == 3 && !dcb3d_supported(desc->L, tile))
        return fail(SMC_EINVAL, "tile %d: 3D tiles are 16 x 16 x 16, dividing L = %d into an even number of tiles "
                                "per direction (or one)", tile, desc->L);
    if (!beta) return fail(SMC_EINVAL, "beta is NULL");
    for (int r = 0; r < desc->n_rep; ++r)
        if (!(beta[r] >= 0.0) || !isfinite(beta[r])) return fail(SMC_EINVAL, "beta[%d] must be finite and >= 0", r);
    return SMC_OK;
}

static std::vector<ThrRow> dcb_rows(const smc_desc *desc, const double *beta) {
    std::vector<ThrRow> rows(desc->n_rep);
    for (int r = 0; r < desc->n_rep; ++r)
        rows[r] = (r > 0 && beta[r] == beta[r - 1]) ? rows[r - 1] : threshold_row(beta[r], desc->dim);
    return rows;
}

int smc_dcb_plan(const smc_desc *desc, const double *beta, int32_t tile, const char **kernel_name) {
    last_error().clear();
    if (!kernel_name) return fail(SMC_EINVAL, "kernel_name is NULL");
    int rc = dcb_check(desc, beta, tile);
    if (rc) return rc;
    *kernel_name = desc->dim == 3 ? "k_dcb3d"
                   : use_dcb_packed(desc, dcb_rows(desc, beta), nullptr, nullptr, tile) ? "k_dcb2d_packed"
                                                                                        : "k_dcb2d";
    return SMC_OK;
}

int smc_dcb_sweep(const smc_desc *desc, void *spins, const int8_t *couplings, const double *beta, uint64_t sweep0,
                  int32_t n_sweeps, int32_t tile, int32_t hits, int32_t palindromic, int64_t *dE_accum,
                  int64_t *dE_trace, void *stream) {
    last_error().clear();
    int rc = dcb_check(desc, beta, tile);
    if (rc) return rc;
    if (hits < 1) return fail(SMC_EINVAL, "hits must be >= 1");
    if (!spins) return fail(SMC_EINVAL, "spins is NULL");
    if (desc->model == SMC_EA && !couplings) return fail(SMC_EINVAL, "couplings are required for EA");
    if (desc->dim == 3 && (((uintptr_t)spins & 15u) || (desc->model == SMC_EA && ((uintptr_t)couplings & 15u))))
        return fail(SMC_EINVAL, "3D double checkerboard: spins (and EA couplings) must be 16-byte aligned");
    if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
    if ((sweep0 + (uint64_t)n_sweeps) * (uint64_t)hits > (1ull << 32))
        return fail(SMC_EINVAL, "(sweep0 + n_sweeps) * hits exceeds 2^32 (the hit index is one 32-bit word)");
    if (n_sweeps == 0) return SMC_OK;
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    StreamCtx &c = ctx_for(s);
    const std::vector<ThrRow> rows = dcb_rows(desc, beta);
    void *tp = nullptr, *sp = nullptr;
    if ((rc = upload(c, s, kTables, rows.data(), sizeof(ThrRow) * rows.size(), &tp))) return rc;
    const int per_rep =
        2 * (desc->dim == 3 ? dcb3d_tiles_per_colour(desc->L, tile) : dcb2d_tiles_per_colour(desc->L, tile));
    if (dE_accum || dE_trace) {
        if ((rc = ensure(c, kDcbSlots, sizeof(int64_t) * (size_t)desc->n_rep * per_rep, &sp))) return rc;
        SMC_HIP(launch_dcb_zero((int64_t *)sp, (int64_t)desc->n_rep * per_rep, s));
    }
    const bool ea = desc->model == SMC_EA;
    const bool packed = use_dcb_packed(desc, rows, spins, ea ? couplings : nullptr, tile);
    SweepTimer timer(s, 2 * (int64_t)n_sweeps);
    for (int32_t m = 0; m < n_sweeps; ++m) {
        const uint64_t t = sweep0 + (uint64_t)m;
        const bool rev = palindromic && (t & 1u);
        for (int ci = 0; ci < 2; ++ci) {
            if (desc->dim == 3)
                SMC_HIP(launch_dcb3d((int8_t *)spins, ea ? couplings : nullptr, ea ? desc->rep_per_sample : 1,
                                     (const ThrRow *)tp, (int64_t *)sp, desc->n_rep, desc->L, tile, hits,
                                     make_key(desc->seed), (uint32_t)t, rev ? 1 - ci : ci, rev, s));
            else
                SMC_HIP(launch_dcb2d((int8_t *)spins, ea ? couplings : nullptr, ea ? desc->rep_per_sample : 1,
                                     (const ThrRow *)tp, (int64_t *)sp, desc->n_rep, desc->L, tile, hits,
                                     make_key(desc->seed), (uint32_t)t, rev ? 1 - ci : ci, rev, packed, s));
        }
        if (dE_trace)
            SMC_HIP(launch_dcb_collect((const int64_t *)sp, dE_trace + (int64_t)m * desc->n_rep, desc->n_rep, per_rep,
                                       true, s));
    }
    timer.finish();
    if (dE_accum) SMC_HIP(launch_dcb_collect((const int64_t *)sp, dE_accum, desc->n_rep, per_rep, false, s));
    return SMC_OK;
}

int smc_heis_dcb_sweep(const smc_desc *desc, void *spins, const double *beta, uint64_t sweep0, int32_t n_sweeps,
                       int32_t tile, int32_t hits, int32_t precision, int32_t palindromic, double cap,
                       int64_t *accepts, void *stream) {
    last_error().clear();
    Plan plan;
    int rc = validate(desc, false, plan);
    if (rc) return rc;
    if (desc->model != SMC_HEISENBERG)
        return fail(SMC_EUNSUPPORTED, "smc_heis_dcb_sweep is for the Heisenberg model (smc_dcb_sweep: Ising, EA)");
    if (desc->dim != 2) return fail(SMC_EUNSUPPORTED, "the Heisenberg double checkerboard is provided for 2D");
    if (desc->L <= 0) return fail(SMC_EINVAL, "the double checkerboard needs a uniform batch (L > 0)");
    if (precision < SMC_HEIS_FLOAT || precision > SMC_HEIS_DOUBLE)
        return fail(SMC_EINVAL, "unknown precision %d", precision);
    if (!heis_dcb2d_supported(desc->L, tile, precision))
        return fail(SMC_EINVAL, "tile %d: need 16, 32 or (float modes) 64, dividing L = %d into an even number "
                                "of tiles per row (or one)", tile, desc->L);
    if (hits < 1) return fail(SMC_EINVAL, "hits must be >= 1");
    if (!(cap >= 0.0 && cap <= 2.0)) return fail(SMC_EINVAL, "cap must be in [0, 2]");
    if (!spins) return fail(SMC_EINVAL, "spins is NULL");
    if ((uintptr_t)spins & 15u) return fail(SMC_EINVAL, "spins must be 16-byte aligned");
    if (!beta) return fail(SMC_EINVAL, "beta is NULL");
    if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
    if ((sweep0 + (uint64_t)n_sweeps) * (uint64_t)hits > (1ull << 32))
        return fail(SMC_EINVAL, "(sweep0 + n_sweeps) * hits exceeds 2^32 (the hit index is one 32-bit word)");
    for (int r = 0; r < desc->n_rep; ++r)
        if (!(beta[r] >= 0.0) || !isfinite(beta[r])) return fail(SMC_EINVAL, "beta[%d] must be finite and >= 0", r);
    if (n_sweeps == 0) return SMC_OK;
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    StreamCtx &c = ctx_for(s);
    void *bp = nullptr, *sp = nullptr;
    if (precision == SMC_HEIS_DOUBLE) {
        if ((rc = upload(c, s, kTables, beta, sizeof(double) * desc->n_rep, &bp))) return rc;
    } else {
        std::vector<float> bf(desc->n_rep);
        for (int r = 0; r < desc->n_rep; ++r) bf[r] = (float)beta[r];
        if ((rc = upload(c, s, kTables, bf.data(), sizeof(float) * bf.size(), &bp))) return rc;
    }
    const int per_rep = 2 * dcb2d_tiles_per_colour(desc->L, tile);
    if (accepts) {
        if ((rc = ensure(c, kDcbSlots, sizeof(int64_t) * (size_t)desc->n_rep * per_rep, &sp))) return rc;
        SMC_HIP(launch_dcb_zero((int64_t *)sp, (int64_t)desc->n_rep * per_rep, s));
    }
    const int64_t n_spins = (int64_t)desc->n_rep * desc->L * desc->L;
    SweepTimer timer(s, 2 * (int64_t)n_sweeps);
    for (int32_t m = 0; m < n_sweeps; ++m) {
        const uint64_t t = sweep0 + (uint64_t)m;
        const bool rev = palindromic && (t & 1u);
        for (int ci = 0; ci < 2; ++ci)
            SMC_HIP(launch_heis_dcb2d(spins, bp, (int64_t *)sp, desc->n_rep, desc->L, tile, hits, precision, cap,
                                      make_key(desc->seed), (uint32_t)t, rev ? 1 - ci : ci, rev, s));
        if (desc->renorm_every > 0 && (t + 1) % (uint64_t)desc->renorm_every == 0)
            SMC_HIP(launch_heis_dcb_renorm(spins, n_spins, precision, s));
    }
    timer.finish();
    if (accepts) SMC_HIP(launch_dcb_collect((const int64_t *)sp, accepts, desc->n_rep, per_rep, false, s));
    return SMC_OK;
}

// Checks shared by the random-number study calls; per-replica state bytes.
static int rng_study_check(const smc_desc *desc, int32_t tile, int32_t generator, int64_t *per_rep) {
    if (!desc) return fail(SMC_EINVAL, "desc is NULL");
    if (desc->dim != 2 || desc->L <= 0 || (desc->model != SMC_ISING && desc->model != SMC_EA))
        return fail(SMC_EINVAL, "the random-number study takes uniform 2D Ising or EA batches");
    if (generator < SMC_RNG_LCG32 || generator > SMC_RNG_FIB1279)
        return fail(SMC_EINVAL, "unknown generator %d", generator);
    if (tile != 16 && tile != 32) return fail(SMC_EINVAL, "tile must be 16 or 32 (got %d)", tile);
    int r = 0, s = 0;
    if (rng_study_lags(generator, &r, &s) && tile != 16)
        return fail(SMC_EINVAL, "the lagged Fibonacci generators take tile 16 (a round of T^2/2 numbers must "
                                "not exceed min(s, r - s))");
    if (desc->L % tile || (desc->L / tile) % 2)
        return fail(SMC_EINVAL, "L / tile must be an even integer (L=%d, tile=%d)", desc->L, tile);
    *per_rep = rng_study_state_bytes(generator, desc->L, tile);
    return SMC_OK;
}

int smc_rng_study_state_bytes(const smc_desc *desc, int32_t tile, int32_t generator, int64_t *bytes) {
    last_error().clear();
    int64_t per = 0;
    int rc = rng_study_check(desc, tile, generator, &per);
    if (rc) return rc;
    if (!bytes) return fail(SMC_EINVAL, "bytes is NULL");
    if (desc->n_rep < 1) return fail(SMC_EINVAL, "n_rep must be >= 1");
    *bytes = per * desc->n_rep;
    return SMC_OK;
}

int smc_rng_study_init(const smc_desc *desc, int32_t tile, int32_t generator, void *state, int64_t state_bytes,
                       void *stream) {
    last_error().clear();
    int64_t per = 0;
    int rc = rng_study_check(desc, tile, generator, &per);
    if (rc) return rc;
    if (desc->n_rep < 1) return fail(SMC_EINVAL, "n_rep must be >= 1");
    if (!state || ((uintptr_t)state & 7u)) return fail(SMC_EINVAL, "state must be a non-NULL 8-byte aligned pointer");
    if (state_bytes < per * desc->n_rep)
        return fail(SMC_EINVAL, "state holds %lld bytes, needs %lld", (long long)state_bytes,
                    (long long)(per * desc->n_rep));
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    SMC_HIP(launch_rng_init(generator, desc->L, tile, desc->n_rep, state, make_key(desc->seed), s));
    return SMC_OK;
}

int smc_rng_study_sweep(const smc_desc *desc, void *spins, const int8_t *couplings, const double *beta,
                        int32_t n_sweeps, int32_t tile, int32_t hits, int32_t generator, void *state,
                        int64_t state_bytes, int64_t *dE_accum, void *stream) {
    last_error().clear();
    int64_t per = 0;
    int rc = rng_study_check(desc, tile, generator, &per);
    if (rc) return rc;
    Plan plan;
    if ((rc = validate(desc, desc->model == SMC_EA, plan))) return rc;
    if (!spins) return fail(SMC_EINVAL, "spins is NULL");
    if (desc->model == SMC_EA && !couplings) return fail(SMC_EINVAL, "couplings are required for EA");
    if (!beta) return fail(SMC_EINVAL, "beta is NULL");
    for (int r = 0; r < desc->n_rep; ++r)
        if (!(beta[r] >= 0.0) || !isfinite(beta[r])) return fail(SMC_EINVAL, "beta[%d] must be finite and >= 0", r);
    if (hits < 1) return fail(SMC_EINVAL, "hits must be >= 1");
    if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
    if (!state || ((uintptr_t)state & 7u)) return fail(SMC_EINVAL, "state must be a non-NULL 8-byte aligned pointer");
    if (state_bytes < per * desc->n_rep)
        return fail(SMC_EINVAL, "state holds %lld bytes, needs %lld", (long long)state_bytes,
                    (long long)(per * desc->n_rep));
    if (n_sweeps == 0) return SMC_OK;
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    StreamCtx &c = ctx_for(s);
    std::vector<ThrRow> rows((size_t)desc->n_rep);
    for (int r = 0; r < desc->n_rep; ++r) rows[r] = threshold_row(beta[r], 2);
    void *p = nullptr;
    if ((rc = upload(c, s, kTables, rows.data(), sizeof(ThrRow) * rows.size(), &p))) return rc;
    const int rps = desc->model == SMC_EA ? desc->rep_per_sample : 1;
    for (int32_t t = 0; t < n_sweeps; ++t)
        for (int tc = 0; tc < 2; ++tc)
            SMC_HIP(launch_dcb_rng(generator, (int8_t *)spins, desc->model == SMC_EA ? couplings : nullptr, rps,
                                   (const ThrRow *)p, state, dE_accum, desc->n_rep, desc->L, tile, hits, tc, s));
    return SMC_OK;
}

int smc_msc_plan(const smc_desc *desc, int32_t n_sweeps, int32_t word_bits, int32_t *launches,
                 const char **kernel_name) {
    last_error().clear();
    if (!launches || !kernel_name) return fail(SMC_EINVAL, "output pointers are required");
    Plan plan;
    int rc = validate(desc, false, plan);
    if (rc) return rc;
    if ((rc = msc_check(desc, word_bits))) return rc;
    if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
    if (use_msc2d(desc, nullptr, nullptr)) {
        *kernel_name = "k_msc2d";
        *launches = n_sweeps > 0 ? 1 : 0;
    } else {
        *kernel_name = "k_half_sweep_generic";
        *launches = 2 * n_sweeps;
    }
    return SMC_OK;
}

int run_pt_split2d(StreamCtx &c, hipStream_t s, const smc_desc *desc, void *spins, SwapArgs &sw,
                   const ThrRow *thr_rows, double *energy, uint64_t step0, int32_t n_steps, int m) {
    int rc;
    const int L = desc->L, n_rep = desc->n_rep;
    const int64_t N = (int64_t)L * L;
    const size_t bytes = (size_t)n_rep * lattice2d_split_bytes(L);
    const size_t slots = lattice2d_de_slots(L, n_rep);
    if (slots == 0) return fail(SMC_EINVAL, "no band shape for L=%d", L);
    void *pp = nullptr, *q = nullptr, *tr = nullptr, *dd = nullptr, *op = nullptr;
    if ((rc = ensure(c, kPingPong, 2 * bytes, &pp))) return rc;
    if ((rc = ensure(c, kL2dPart, slots * sizeof(int64_t), &q))) return rc;
    if ((rc = ensure(c, kPtThr, sizeof(ThrRow) * (size_t)n_rep, &tr))) return rc;
    if ((rc = ensure(c, kPtDelta, sizeof(int64_t) * (size_t)n_rep, &dd))) return rc;
    if ((rc = ensure(c, kPtOut, (size_t)N * (size_t)n_rep, &op))) return rc;
    uint8_t *A = (uint8_t *)pp, *B = A + bytes;
    int64_t *part = (int64_t *)q, *d = (int64_t *)dd;
    ThrRow *thr_rep = (ThrRow *)tr;
    const Key key = make_key(desc->seed);
    SMC_HIP(launch_pt_prepare(sw, energy, s));
    SMC_HIP(launch_zero64(d, n_rep, s));
    SMC_HIP(launch_to_split((const int8_t *)spins, A, L, n_rep, s));
    int64_t done = 0;  // sweeps so far (ping-pong parity)
    SweepTimer timer(s, (int64_t)n_steps * m);
    for (int32_t st = 0; st < n_steps; ++st) {
        const uint32_t t = (uint32_t)(step0 + (uint64_t)st);
        sw.t = t;
        SMC_HIP(launch_pt_gather_thr(thr_rows, sw.row_of_rep, thr_rep, n_rep, s));
        for (int j = 0; j < m; ++j, ++done)
            SMC_HIP(launch_ising2d_split(done & 1 ? B : A, false, done & 1 ? A : B, false, L, n_rep, thr_rep, part,
                                         j == 0, key,
                                         t * (uint32_t)m + (uint32_t)j, s));
        SMC_HIP(launch_lattice2d_de_collect(part, d, L, n_rep, s));
        SMC_HIP(launch_pt_add_masked(d, sw.E, sw.row_of_rep, n_rep, s));
        SMC_HIP(launch_pt_swap(sw, s));
    }
    timer.finish();
    // back to lattice order; replicas of chains that are not permutations keep their spins
    SMC_HIP(launch_from_split(done & 1 ? B : A, (int8_t *)op, L, n_rep, s));
    SMC_HIP(launch_copy_valid((const int8_t *)op, (int8_t *)spins, sw.row_of_rep, N, n_rep, s));
    SMC_HIP(launch_pt_finish(sw, energy, s));
    return SMC_OK;
}

int smc_pt_sweep_swap(const smc_desc *desc, const smc_pt_desc *pt, void *spins, const int8_t *couplings,
                      int32_t *slot_of_temp, double *energy, uint64_t step0, int32_t n_steps,
                      uint64_t *swap_accepts, void *stream) {
    last_error().clear();
    Plan plan;
    int rc = validate(desc, true, plan);
    if (rc) return rc;
    if (!pt) return fail(SMC_EINVAL, "pt desc is NULL");
    if (desc->model == SMC_HEISENBERG)
        return fail(SMC_EUNSUPPORTED, "parallel tempering is provided for Ising and EA models");
    if (pt->n_chains < 1 || pt->n_temps < 2) return fail(SMC_EINVAL, "need n_chains >= 1 and n_temps >= 2");
    if ((int64_t)pt->n_chains * pt->n_temps != desc->n_rep)
        return fail(SMC_EINVAL, "n_rep (%d) must equal n_chains * n_temps", desc->n_rep);
    if (!pt->beta) return fail(SMC_EINVAL, "beta is NULL");
    if (!spins || !slot_of_temp || !energy) return fail(SMC_EINVAL, "spins, slot_of_temp and energy are required");
    if (desc->model == SMC_EA && !couplings) return fail(SMC_EINVAL, "couplings are required for EA");
    if (n_steps < 0) return fail(SMC_EINVAL, "n_steps must be >= 0");
    if (pt->sweeps_per_step < 0) return fail(SMC_EINVAL, "sweeps_per_step must be >= 0");
    const int m = pt->sweeps_per_step > 0 ? pt->sweeps_per_step : 1;
    if ((step0 + (uint64_t)n_steps) * (uint64_t)m > (1ull << 32))
        return fail(SMC_EINVAL, "(step0 + n_steps) * sweeps_per_step exceeds 2^32 (the sweep index is 32 bits)");
    const int n = pt->n_temps;
    const int rows_n = pt->beta_per_chain ? pt->n_chains : 1;
    for (int64_t k = 0; k < (int64_t)rows_n * n; ++k)
        if (!(pt->beta[k] >= 0.0) || !isfinite(pt->beta[k])) return fail(SMC_EINVAL, "beta[%lld] invalid", (long long)k);
    if (desc->model == SMC_EA) {
        if (desc->L > 0) {
            if (desc->rep_per_sample % n) return fail(SMC_EINVAL, "rep_per_sample must be a multiple of n_temps");
        } else {
            for (int q = 0; q < pt->n_chains; ++q)
                for (int k = 1; k < n; ++k)
                    if (desc->inst[q * n + k].sample != desc->inst[q * n].sample)
                        return fail(SMC_EINVAL, "chain %d mixes coupling samples", q);
        }
    }
    if (desc->L == 0) {
        for (int q = 0; q < pt->n_chains; ++q)
            for (int k = 1; k < n; ++k)
                if (desc->inst[q * n + k].L != desc->inst[q * n].L)
                    return fail(SMC_EINVAL, "chain %d mixes lattice sizes", q);
    }
    if (n_steps == 0) return SMC_OK;
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    StreamCtx &c = ctx_for(s);
    if ((rc = upload_inst(c, s, desc, plan))) return rc;

    // tables: beta per (row, k) and threshold rows (row * n + k)
    std::vector<ThrRow> rows((size_t)rows_n * n);
    for (size_t k = 0; k < rows.size(); ++k) rows[k] = threshold_row(pt->beta[k], desc->dim);
    void *thr = nullptr, *bdev = nullptr, *E64 = nullptr, *rowrep = nullptr;
    if ((rc = upload(c, s, kTables, rows.data(), sizeof(ThrRow) * rows.size(), &thr))) return rc;
    if ((rc = upload(c, s, kBeta, pt->beta, sizeof(double) * rows.size(), &bdev))) return rc;
    if (use_pt3d(desc, pt, spins, rows)) {
        SMC_HIP(launch_pt3d(desc->model, (int8_t *)spins, desc->model == SMC_EA ? couplings : nullptr,
                            desc->rep_per_sample, pt->n_chains, n, pt->beta_per_chain ? 1 : 0, (const double *)bdev,
                            (const ThrRow *)thr, slot_of_temp, energy, (unsigned long long *)swap_accepts,
                            make_key(desc->seed), (uint32_t)step0, n_steps, m, s));
        return SMC_OK;
    }
    if ((rc = ensure(c, kEnergy64, sizeof(int64_t) * desc->n_rep, &E64))) return rc;
    if ((rc = ensure(c, kRows, sizeof(int32_t) * desc->n_rep, &rowrep))) return rc;

    SwapArgs sw;
    sw.t_dev = nullptr;
    sw.n_chains = pt->n_chains;
    sw.n_temps = n;
    sw.beta_per_chain = pt->beta_per_chain ? 1 : 0;
    sw.beta = (const double *)bdev;
    sw.slot_of_temp = slot_of_temp;
    sw.row_of_rep = (int32_t *)rowrep;
    sw.E = (int64_t *)E64;
    sw.acc = (unsigned long long *)swap_accepts;
    sw.key = make_key(desc->seed);
    sw.t = 0;

    SweepArgs a;
    memset(&a, 0, sizeof a);
    a.b = plan.b;
    a.spins = spins;
    a.coup = desc->model == SMC_EA ? couplings : nullptr;
    a.key = make_key(desc->seed);
    a.dE = (int64_t *)E64;
    a.max_L = plan.max_L;
    a.thr = (const ThrRow *)thr;
    a.row_of_rep = (const int32_t *)rowrep;

    if (use_pt_split2d(desc, spins, rows))
        return run_pt_split2d(c, s, desc, spins, sw, (const ThrRow *)thr, energy, step0, n_steps, m);
    if (use_uneven2d(desc, spins, couplings, rows))
        return run_uneven2d(c, s, desc, plan, pt, spins, couplings, sw, (const ThrRow *)thr, energy, step0, n_steps,
                            m);
    SMC_HIP(launch_pt_prepare(sw, energy, s));
    for (int32_t k = 0; k < n_steps; ++k) {
        const uint32_t t = (uint32_t)(step0 + (uint64_t)k);
        sw.t = t;
        for (int j = 0; j < m; ++j) {
            a.t = t * (uint32_t)m + (uint32_t)j;
            SMC_HIP(launch_half_sweep_generic(a, 0, s));
            SMC_HIP(launch_half_sweep_generic(a, 1, s));
        }
        SMC_HIP(launch_pt_swap(sw, s));
    }
    SMC_HIP(launch_pt_finish(sw, energy, s));
    return SMC_OK;
}

int smc_measure_energy_magnetisation(const smc_desc *desc, const void *spins, const int8_t *couplings,
                                     double *energy, double *magnetisation, void *stream) {
    last_error().clear();
    Plan plan;
    int rc = validate(desc, true, plan);
    if (rc) return rc;
    if (!spins || !energy) return fail(SMC_EINVAL, "spins and energy are required");
    if (desc->model == SMC_EA && !couplings) return fail(SMC_EINVAL, "couplings are required for EA");
    hipStream_t s = (hipStream_t)stream;
    if (int rc_cap = refuse_capture(s)) return rc_cap;
    StreamCtx &c = ctx_for(s);
    if ((rc = upload_inst(c, s, desc, plan))) return rc;
    const size_t bytes = measure_scratch_bytes(plan.b, plan.max_L);
    void *p = nullptr;
    if ((rc = ensure(c, kMeasure, bytes, &p))) return rc;
    SMC_HIP(launch_measure(plan.b, spins, desc->model == SMC_EA ? couplings : nullptr, plan.max_L, energy,
                           magnetisation, p, bytes, s));
    return SMC_OK;
}

}  // extern "C"

// ------------------------------------------------------ allocation-free call --
// smc_measure_energy_magnetisation_noalloc keeps its partial sums in this
// fixed array instead of the per-stream scratch.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the device
// symbol): the device address of each GPU's copy is looked up once per device
// with hipGetSymbolAddress and that address is what the kernels receive.
namespace smc {
constexpr size_t kNoAllocScratchBytes = 16u << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
void *g_noalloc_ptr[kMaxDevices] = {};

int noalloc_scratch(void **out) {
    int dev = 0;
    SMC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SMC_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_noalloc_mutex);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        SMC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(SMC_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_noalloc_ptr[dev] = ptr;
    }
    *out = g_noalloc_ptr[dev];
    return SMC_OK;
}
}  // namespace
}  // namespace smc

extern "C" {

int smc_measure_energy_magnetisation_noalloc(const smc_desc *desc, const void *spins, const int8_t *couplings,
                                             double *energy, double *magnetisation, void *stream) {
    using namespace smc;
    last_error().clear();
    Plan plan;
    int rc = validate(desc, true, plan);
    if (rc) return rc;
    if (desc->L <= 0) return fail(SMC_EUNSUPPORTED, "the allocation-free measurement takes uniform batches only");
    if (!spins || !energy) return fail(SMC_EINVAL, "spins and energy are required");
    if (desc->model == SMC_EA && !couplings) return fail(SMC_EINVAL, "couplings are required for EA");
    const size_t bytes = measure_scratch_bytes(plan.b, plan.max_L);
    if (bytes > kNoAllocScratchBytes)
        return fail(SMC_EINVAL, "batch needs %zu bytes of partial sums; the allocation-free call holds at most %zu",
                    bytes, kNoAllocScratchBytes);
    void *p = nullptr;
    if ((rc = noalloc_scratch(&p))) return rc;
    SMC_HIP(launch_measure(plan.b, spins, desc->model == SMC_EA ? couplings : nullptr, plan.max_L, energy,
                           magnetisation, p, bytes, (hipStream_t)stream));
    return SMC_OK;
}

}  // extern "C"

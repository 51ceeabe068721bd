// The host runtime of the C-ABI layer (declared in runtime.hpp).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "runtime.hpp"

namespace smc {

thread_local std::string g_launch_rejection;

hipError_t reject_launch(const char *kernel, uint64_t grid, uint64_t block, uint64_t lds, const char *why) {
    char buf[256];
    snprintf(buf, sizeof buf, "launch of %s refused (%s): %llu workgroups of %llu, %llu bytes of LDS", kernel, why,
             (unsigned long long)grid, (unsigned long long)block, (unsigned long long)lds);
    g_launch_rejection = buf;
    return hipErrorInvalidConfiguration;
}

std::string take_launch_rejection() {
    std::string r;
    r.swap(g_launch_rejection);
    return r;
}

namespace {
thread_local std::string g_last_error;
}  // namespace

std::string &last_error() { return g_last_error; }

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// ------------------------------------------------------------------ scratch --

namespace {
std::mutex g_ctx_mutex;
std::map<std::pair<int, hipStream_t>, StreamCtx> g_ctx;
}  // namespace

StreamCtx &ctx_for(hipStream_t s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_ctx_mutex);
    StreamCtx &c = g_ctx[std::make_pair(dev, s)];
    c.stream = s;
    return c;
}

// Device buffer of at least `bytes`.  Only calls on this set's stream use
// the buffer, so growing waits for that stream (not the whole device)
// before the old allocation is freed.
int ensure(StreamCtx &c, Slot slot, size_t bytes, void **out) {
    Buffer &b = c.dev[slot];
    if (b.bytes < bytes) {
        if (b.p) {
            SMC_HIP(hipStreamSynchronize(c.stream));
            SMC_HIP(hipFree(b.p));
            b.p = nullptr;
            b.bytes = 0;
        }
        b.last.clear();
        size_t want = bytes < 256 ? 256 : bytes;
        if (hipMalloc(&b.p, want) != hipSuccess) {
            (void)hipGetLastError();
            b.p = nullptr;
            return fail(SMC_ENOMEM, "could not allocate %zu bytes of scratch", want);
        }
        b.bytes = want;
    }
    *out = b.p;
    return SMC_OK;
}

int release(StreamCtx &c, Slot slot) {
    Buffer &b = c.dev[slot];
    if (b.p) {
        SMC_HIP(hipStreamSynchronize(c.stream));
        SMC_HIP(hipFree(b.p));
    }
    b.p = nullptr;
    b.bytes = 0;
    b.last.clear();
    return SMC_OK;
}

// Copy host bytes into a device scratch slot through that slot's pinned
// staging area.  The staging area is reused only after its previous copy has
// completed; an upload identical to the slot's previous one is skipped (the
// device copy is only ever written by uploads, in stream order).
int upload(StreamCtx &c, hipStream_t s, Slot slot, const void *src, size_t bytes, void **dev_out) {
    int rc = ensure(c, slot, bytes, dev_out);
    if (rc) return rc;
    Buffer &b = c.dev[slot];
    if (b.last.size() == bytes && memcmp(b.last.data(), src, bytes) == 0) return SMC_OK;
    if (b.staged_pending) {
        SMC_HIP(hipEventSynchronize(b.staged));
        b.staged_pending = false;
    }
    if (b.pinned_bytes < bytes) {
        if (b.pinned) SMC_HIP(hipHostFree(b.pinned));
        b.pinned = nullptr;
        b.pinned_bytes = 0;
        size_t want = bytes < 4096 ? 4096 : bytes;
        if (hipHostMalloc(&b.pinned, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            b.pinned = nullptr;
            return fail(SMC_ENOMEM, "could not allocate %zu bytes of pinned staging", want);
        }
        b.pinned_bytes = want;
    }
    if (!b.staged) SMC_HIP(hipEventCreateWithFlags(&b.staged, hipEventDisableTiming));
    memcpy(b.pinned, src, bytes);
    b.last.assign((const unsigned char *)src, (const unsigned char *)src + bytes);
    SMC_HIP(hipMemcpyAsync(*dev_out, b.pinned, bytes, hipMemcpyHostToDevice, s));
    SMC_HIP(hipEventRecord(b.staged, s));
    b.staged_pending = true;
    return SMC_OK;
}

// Calls stage host data (tables, instance lists) through pinned buffers,
// grow their scratch on demand and build graphs of their own; none of that
// can be recorded into a caller's stream capture, so a call on a capturing
// stream is refused before anything is issued.
int refuse_capture(hipStream_t s) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    SMC_HIP(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone)
        return fail(SMC_EINVAL, "the stream is capturing a graph: this call cannot be captured");
    return SMC_OK;
}

// ----------------------------------------------------------------- tables ----
// thr[m] = floor(2^32 exp(-4 m beta)) for Delta E = 4m > 0, computed in
// float64 with the C library's exp and split as (thr >> 16, thr & 0xffff).
ThrRow threshold_row(double beta, int dim) {
    ThrRow row;
    row.m[0] = make_uint2(65536u, 0u);
    for (int m = 1; m <= 3; ++m) {
        uint64_t thr = 0;
        if (m <= dim) {
            const double p = exp(-beta * (4.0 * m));
            thr = (uint64_t)floor(4294967296.0 * p);
        }
        row.m[m] = make_uint2((uint32_t)(thr >> 16), (uint32_t)(thr & 0xFFFFu));
    }
    return row;
}

// The chain-resident tempering kernel serves 3D edge-16 batches of at most
// 32 temperatures with 16-byte aligned spins and thresholds below 2^32.
// Uniform 3D Heisenberg batches with a power-of-two edge take the indexed
// kernel (SPINMC_HEIS3D=0 sends them to the generic one).
bool use_heis3d(const smc_desc *d) {
    const char *env = getenv("SPINMC_HEIS3D");
    if (env && env[0] == '0') return false;
    return d->model == SMC_HEISENBERG && d->L > 0 && heis3d_supported(d->dim, d->L);
}

// ... and with an edge of at least 32 the one-pass tiled kernel
// (SPINMC_HEIS_TILED=0 keeps the two half-sweep launches).
bool use_heis3d_tiled(const smc_desc *d) {
    const char *env = getenv("SPINMC_HEIS_TILED");
    if (env && env[0] == '0') return false;
    return use_heis3d(d) && heis3d_tiled_supported(d->dim, d->L);
}

bool pt3d_enabled() {
    const char *env = getenv("SPINMC_PT3D");
    return !(env && env[0] == '0');
}

bool use_pt3d(const smc_desc *d, const smc_pt_desc *pt, const void *spins, const std::vector<ThrRow> &rows) {
    if (!pt3d_enabled() || !pt3d_supported(d, pt->n_temps)) return false;
    if (((uintptr_t)spins & 15u) != 0) return false;
    for (const ThrRow &r : rows)
        if (r.m[1].x > 0xFFFFu || r.m[2].x > 0xFFFFu || r.m[3].x > 0xFFFFu) return false;
    return true;
}

// The one-pass split-layout kernel serves uniform 2D Ising batches whose
// edge it supports, with 16-byte aligned spins and thresholds below 2^32
// (beta > 0 up to rounding; the generic kernels cover the rest).
bool use_lattice2d(const smc_desc *d, const void *spins, const std::vector<ThrRow> &rows) {
    if (d->model != SMC_ISING || d->dim != 2 || d->L <= 0 || !lattice2d_supported(d->L)) return false;
    if (((uintptr_t)spins & 15u) != 0) return false;
    for (const ThrRow &r : rows)
        if (r.m[1].x > 0xFFFFu || r.m[2].x > 0xFFFFu) return false;
    return true;
}

// Uniform 3D Ising / EA batches with an edge that is a multiple of 16 take
// the segment-per-thread half-sweeps when spins (and couplings) are 16-byte
// aligned and every threshold has a 16-bit high half; SPINMC_SWEEP3D=0 keeps
// them on the generic kernels (same results).
bool sweep3d_shape(const smc_desc *d) {
    const char *env = getenv("SPINMC_SWEEP3D");
    if (env && env[0] == '0') return false;
    return d->dim == 3 && d->L > 0 && (d->model == SMC_ISING || d->model == SMC_EA) && sweep3d_supported(d->L);
}

// ... and, with an edge of 512 .. 1024, the one-pass sweep (below 512 its
// strips are too few to fill the chip and the two half-sweep launches are
// faster; SPINMC_SWEEP3D_PASS=1 takes it for every edge of 32 .. 1024 it
// supports, SPINMC_SWEEP3D_PASS=0 never).
bool pass3d_enabled(const smc_desc *d) {
    const char *env = getenv("SPINMC_SWEEP3D_PASS");
    if (env && env[0] == '0') return false;
    if (!(env && env[0] == '1') && d->L < 512) return false;
    return pass3d_supported(d->L);
}

bool use_sweep3d(const smc_desc *d, const void *spins, const int8_t *coup, const std::vector<ThrRow> &rows) {
    if (!sweep3d_shape(d)) return false;
    if (((uintptr_t)spins & 15u) != 0 || (d->model == SMC_EA && ((uintptr_t)coup & 15u) != 0)) return false;
    for (const ThrRow &r : rows)
        if (r.m[1].x > 0xFFFFu || r.m[2].x > 0xFFFFu || r.m[3].x > 0xFFFFu) return false;
    return true;
}

// Tempering of a uniform 2D Ising batch on the one-pass colour-split sweep:
// L a power of two in [1024, 16384], aligned spins, thresholds of every
// temperature with 16-bit high halves; SPINMC_PT_SPLIT2D=0 sends such
// batches to the generic kernels (same results).
bool use_pt_split2d(const smc_desc *d, const void *spins, const std::vector<ThrRow> &rows) {
    const char *env = getenv("SPINMC_PT_SPLIT2D");
    if (env && env[0] == '0') return false;
    return use_lattice2d(d, spins, rows);
}

// --------------------------------------------------------------- validation --

int64_t sites(int dim, int L) { return dim == 3 ? (int64_t)L * L * L : (int64_t)L * L; }

// The coupling samples of a uniform EA batch: sample q at q * d * N.
void fill_uniform_samples(const smc_desc *d, Plan &plan) {
    if (d->L <= 0 || d->model != SMC_EA || !plan.samples.empty()) return;
    plan.samples.resize((size_t)plan.n_samples);
    for (int64_t q = 0; q < plan.n_samples; ++q) {
        smc_inst &g = plan.samples[(size_t)q];
        g.L = d->L;
        g.sample = (int32_t)q;
        g.spin_off = 0;
        g.coup_off = q * d->dim * plan.b.N;
    }
}

int validate(const smc_desc *d, bool need_coup, Plan &plan) {
    if (!d) return fail(SMC_EINVAL, "desc is NULL");
    if (d->model < SMC_ISING || d->model > SMC_HEISENBERG) return fail(SMC_EINVAL, "unknown model %d", d->model);
    if (d->dim != 2 && d->dim != 3) return fail(SMC_EINVAL, "dim must be 2 or 3 (got %d)", d->dim);
    if (d->n_rep < 1) return fail(SMC_EINVAL, "n_rep must be >= 1 (got %d)", d->n_rep);
    if (d->spins_len <= 0) return fail(SMC_EINVAL, "spins_len must be > 0");
    if (d->model == SMC_HEISENBERG && d->renorm_every < 0) return fail(SMC_EINVAL, "renorm_every must be >= 0");
    const bool ea = d->model == SMC_EA;
    const int per_site = d->model == SMC_HEISENBERG ? 3 : 1;
    Batch &b = plan.b;
    b.dim = d->dim;
    b.model = d->model;
    b.n_rep = d->n_rep;
    b.L = d->L;
    b.rep_per_sample = 1;
    b.inst = nullptr;
    b.N = 0;
    plan.samples.clear();
    if (d->L > 0) {
        if (d->inst) return fail(SMC_EINVAL, "inst must be NULL for a uniform batch (L > 0)");
        if (d->L % 2 || d->L < 4) return fail(SMC_EINVAL, "L must be even and >= 4 (got %d)", d->L);
        if (d->L > (d->dim == 3 ? 1024 : 65536)) return fail(SMC_EINVAL, "L too large (got %d)", d->L);
        b.N = sites(d->dim, d->L);
        if (b.N / 2 > 0xFFFFFFFFll) return fail(SMC_EINVAL, "lattice too large for 32-bit site counters");
        plan.max_L = d->L;
        if ((int64_t)d->n_rep * b.N * per_site > d->spins_len)
            return fail(SMC_EINVAL, "spin buffer too small: need %lld elements, have %lld",
                        (long long)((int64_t)d->n_rep * b.N * per_site), (long long)d->spins_len);
        if (ea) {
            if (d->rep_per_sample < 1) return fail(SMC_EINVAL, "rep_per_sample must be >= 1 for EA");
            b.rep_per_sample = d->rep_per_sample;
            plan.n_samples = (d->n_rep + d->rep_per_sample - 1) / d->rep_per_sample;
            // the sample table is built only where a path needs it (fill_uniform_samples)
            if (need_coup) {
                if (d->coup_len <= 0) return fail(SMC_EINVAL, "coup_len must be > 0 for EA");
                if (plan.n_samples * d->dim * b.N > d->coup_len)
                    return fail(SMC_EINVAL, "couplings of sample %lld lie outside the coupling buffer",
                                (long long)(d->coup_len / (d->dim * b.N)));
            }
        }
    } else {
        if (!d->inst) return fail(SMC_EINVAL, "inst is required when L == 0");
        std::map<int32_t, smc_inst> seen;
        for (int r = 0; r < d->n_rep; ++r) {
            const smc_inst &g = d->inst[r];
            if (g.L % 2 || g.L < 4 || g.L > (d->dim == 3 ? 1024 : 65536))
                return fail(SMC_EINVAL, "inst[%d].L must be even and in [4, limit] (got %d)", r, g.L);
            const int64_t N = sites(d->dim, g.L);
            if (g.spin_off < 0 || g.spin_off > d->spins_len / per_site - N)
                return fail(SMC_EINVAL, "inst[%d] spins lie outside the spin buffer", r);
            if (ea) {
                if (g.sample < 0) return fail(SMC_EINVAL, "inst[%d].sample must be >= 0", r);
                auto it = seen.find(g.sample);
                if (it == seen.end()) {
                    seen[g.sample] = g;
                } else if (it->second.L != g.L || it->second.coup_off != g.coup_off) {
                    return fail(SMC_EINVAL, "inst[%d]: sample %d used with two geometries", r, g.sample);
                }
            }
            if (g.L > plan.max_L) plan.max_L = g.L;
        }
        for (auto &kv : seen) plan.samples.push_back(kv.second);
        plan.n_samples = (int64_t)plan.samples.size();
    }
    if (ea && need_coup && d->L == 0) {
        if (d->coup_len <= 0) return fail(SMC_EINVAL, "coup_len must be > 0 for EA");
        for (const smc_inst &g : plan.samples) {
            const int64_t need = (int64_t)d->dim * sites(d->dim, g.L);
            if (g.coup_off < 0 || g.coup_off > d->coup_len - need)
                return fail(SMC_EINVAL, "couplings of sample %d lie outside the coupling buffer", g.sample);
        }
    }
    return SMC_OK;
}

int upload_inst(StreamCtx &c, hipStream_t s, const smc_desc *d, Plan &plan) {
    if (d->L > 0) return SMC_OK;
    void *p = nullptr;
    int rc = upload(c, s, kInst, d->inst, sizeof(smc_inst) * (size_t)d->n_rep, &p);
    plan.b.inst = (const smc_inst *)p;
    return rc;
}

}  // namespace smc

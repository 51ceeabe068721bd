// Launch-shape tuning: the workgroup size of the LDS-resident 2D kernel
// per edge, the band height of the one-pass 2D Ising sweep, the strip shape
// of the one-pass 3D sweep and the rows per thread of the 3D half-sweeps,
// each measured on scratch lattices of the batch's shape (smc_autotune) and
// kept per process and device (and in an optional cache file).  A shape
// changes the schedule only, never the results.  The tile of the double
// checkerboard is an argument of its own entry point, not a launch shape:
// it changes the chain, so it is never tuned.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "runtime.hpp"

namespace smc {
namespace {

std::mutex g_tune_mutex;
std::map<std::tuple<int, int, int>, int> g_tuned;  // (device, edge, EA) -> workgroup size of the 2D LDS kernel
std::map<std::tuple<int, int, int, int, int>, Shape> g_shapes;  // (device, kind, edge, model, replicas) -> shape

const char *const kKindName[] = {"band2d", "pass3d", "half3d"};

int current_device() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    return dev;
}

// The device's identity in the autotune cache file: architecture and CUs.
std::string device_tag(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "";
    std::string arch(p.gcnArchName);
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    return arch + ":" + std::to_string(p.multiProcessorCount);
}


// Mean milliseconds of one call of `sweep` over reps calls after one
// untimed call, on stream s.
int time_calls(hipStream_t s, int reps, const std::function<hipError_t(int)> &sweep, float *ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SMC_HIP(hipEventCreate(&e0));
    SMC_HIP(hipEventCreate(&e1));
    hipError_t err = sweep(0);
    if (err == hipSuccess) err = hipEventRecord(e0, s);
    for (int k = 1; k <= reps && err == hipSuccess; ++k) err = sweep(k);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float total = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&total, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) {
        const std::string why = take_launch_rejection();
        return fail(SMC_EHIP, "autotuning: %s%s%s", hipGetErrorString(err), why.empty() ? "" : ": ", why.c_str());
    }
    *ms = total / (float)reps;
    return SMC_OK;
}

// The fastest of the candidate shapes of one kind for (edge, model,
// replicas).  Each is set as the tuned shape and timed over enough calls to
// last about 5 ms; a first round over all candidates is not counted (it
// brings the clocks up), the next two are and the lower time of each
// candidate is kept.  The default shape dflt (the one the launcher would
// take untuned) stays unless another is more than 2 % faster, so that
// noise does not move the choice.
int pick_shape(int kind, int L, int model, int n_rep, const std::vector<Shape> &cands, const Shape &dflt,
               hipStream_t s, const std::function<hipError_t(int)> &sweep) {
    if (cands.empty()) return SMC_OK;
    std::vector<float> best(cands.size(), 1e30f);
    int reps = 3;
    for (int round = 0; round < 3; ++round)
        for (size_t i = 0; i < cands.size(); ++i) {
            set_tuned_shape(kind, L, model, n_rep, cands[i]);
            float ms = 0.0f;
            const int rc = time_calls(s, reps, sweep, &ms);
            if (rc) return rc;
            if (round == 0 && i == 0) reps = std::max(3, std::min(64, (int)(5.0f / std::max(ms, 1e-3f))));
            if (round > 0) best[i] = std::min(best[i], ms);
        }
    size_t pick = 0, d = cands.size();
    for (size_t i = 0; i < cands.size(); ++i) {
        if (best[i] < best[pick]) pick = i;
        if (cands[i].v[0] == dflt.v[0] && cands[i].v[1] == dflt.v[1] && cands[i].v[2] == dflt.v[2]) d = i;
    }
    if (d < cands.size() && best[pick] > 0.98f * best[d]) pick = d;
    set_tuned_shape(kind, L, model, n_rep, cands[pick]);
    return SMC_OK;
}

// Band height of the one-pass 2D Ising sweep: heights 4 .. 128 that divide
// L, each timed on scratch copies of the batch in the colour-split layout
// (random spins: the sweep stores only the bytes that flip).
int tune_band2d(StreamCtx &c, hipStream_t s, const Batch &b, Key key) {
    if (getenv("SPINMC_L2D_H")) return SMC_OK;  // the environment fixes the height
    const int L = b.L, n_rep = b.n_rep;
    const size_t bytes = (size_t)n_rep * lattice2d_split_bytes(L);
    void *R = nullptr, *A = nullptr, *B = nullptr, *tp = nullptr;
    int rc;
    if ((rc = ensure(c, kTuneSpins, (size_t)n_rep * (size_t)L * L, &R)) || (rc = ensure(c, kTuneA, bytes, &A)) ||
        (rc = ensure(c, kTuneB, bytes, &B)))
        return rc;
    const std::vector<ThrRow> rows((size_t)n_rep, threshold_row(0.44, 2));
    if ((rc = upload(c, s, kTables, rows.data(), sizeof(ThrRow) * rows.size(), &tp))) return rc;
    SMC_HIP(launch_init_spins(b, L, (int8_t *)R, key, s));
    SMC_HIP(launch_to_split((const int8_t *)R, (uint8_t *)A, L, n_rep, s));
    const Shape dflt{{lattice2d_band_height(L, n_rep), 0, 0}};  // not tuned yet: the heuristic's height
    std::vector<Shape> cands;
    for (int H = 4; H <= 128; H <<= 1)
        if (L % H == 0) cands.push_back(Shape{{H, 0, 0}});
    return pick_shape(kShapeBand2d, L, 0, n_rep, cands, dflt, s, [&](int k) {
        return launch_ising2d_split(k & 1 ? B : A, false, k & 1 ? A : B, false, L, n_rep, (const ThrRow *)tp, nullptr,
                                    false, key, (uint32_t)k, s);
    });
}

// Scratch for a 3D batch: random spins (n_rep lattices) and, for EA,
// bit-packed bonds all ferromagnetic (the sweep's time does not depend on
// their values).
int scratch3d(StreamCtx &c, hipStream_t s, const Batch &b, bool ea, int64_t n_samples, Key key, void **spins,
              void **bonds, void **thr) {
    const int L = b.L, n_rep = b.n_rep;
    const int64_t N = (int64_t)L * L * L;
    int rc;
    if ((rc = ensure(c, kTuneA, (size_t)(n_rep * N), spins))) return rc;
    SMC_HIP(launch_init_spins(b, L, (int8_t *)*spins, key, s));
    *bonds = nullptr;
    if (ea) {
        if ((rc = ensure(c, kBonds3d, (size_t)n_samples * (size_t)(N / 16) * sizeof(uint2), bonds))) return rc;
        SMC_HIP(hipMemsetAsync(*bonds, 0, (size_t)n_samples * (size_t)(N / 16) * sizeof(uint2), s));
    }
    const std::vector<ThrRow> rows((size_t)n_rep, threshold_row(0.2216, 3));
    return upload(c, s, kTables, rows.data(), sizeof(ThrRow) * rows.size(), thr);
}

// Strip shape of the one-pass 3D sweep: every valid (rows per strip,
// segments per thread, planes per z segment), timed between two scratch
// lattices.
int tune_pass3d(StreamCtx &c, hipStream_t s, const Batch &b, bool ea, int64_t n_samples, Key key) {
    if (getenv("SPINMC_PASS3D_TY") || getenv("SPINMC_PASS3D_SEGS") || getenv("SPINMC_PASS3D_D")) return SMC_OK;
    const int L = b.L, n_rep = b.n_rep, rps = b.rep_per_sample;
    void *A = nullptr, *B = nullptr, *pb = nullptr, *tp = nullptr;
    int rc;
    if ((rc = scratch3d(c, s, b, ea, n_samples, key, &A, &pb, &tp))) return rc;
    const size_t bytes = (size_t)n_rep * (size_t)L * L * L;
    if ((rc = ensure(c, kTuneB, bytes, &B))) return rc;
    Shape dflt{{0, 0, 0}};
    (void)pass3d_launch_shape(L, ea, n_rep, &dflt);  // not tuned yet: the default shape
    std::vector<Shape> cands;
    for (int ty : {8, 16})
        for (int segs : {1, 2})
            for (int D : {16, 32, 64, 128, 256, 512})
                if (pass3d_shape_valid(L, ea, ty, segs, D)) cands.push_back(Shape{{ty, segs, D}});
    return pick_shape(kShapePass3d, L, ea ? 1 : 0, n_rep, cands, dflt, s, [&](int k) {
        return launch_ising3d_pass((const int8_t *)(k & 1 ? B : A), (int8_t *)(k & 1 ? A : B), (const uint2 *)pb, rps,
                                   (const ThrRow *)tp, nullptr, n_rep, L, key, (uint32_t)k, s);
    });
}

// Rows per thread of the 3D half-sweeps: 1 .. 16 where they regroup the
// workgroups evenly, timed on a scratch lattice (both colours per call).
int tune_half3d(StreamCtx &c, hipStream_t s, const Batch &b, bool ea, int64_t n_samples, Key key) {
    if (getenv("SPINMC_SWEEP3D_Z")) return SMC_OK;
    const int L = b.L, n_rep = b.n_rep, rps = b.rep_per_sample;
    void *A = nullptr, *pb = nullptr, *tp = nullptr;
    int rc;
    if ((rc = scratch3d(c, s, b, ea, n_samples, key, &A, &pb, &tp))) return rc;
    const int64_t B = L / 16;
    const Shape dflt{{sweep3d_rows(L, ea, n_rep), 0, 0}};
    std::vector<Shape> cands;
    for (int Z = 1; Z <= 16; Z <<= 1)
        if ((B * B * B) % Z == 0) cands.push_back(Shape{{Z, 0, 0}});
    return pick_shape(kShapeHalf3d, L, ea ? 1 : 0, n_rep, cands, dflt, s, [&](int k) {
        hipError_t e = hipSuccess;
        for (int col = 0; col < 2 && e == hipSuccess; ++col)
            e = launch_ising3d_half((int8_t *)A, nullptr, (const uint2 *)pb, rps, (const ThrRow *)tp, nullptr, n_rep,
                                    L, key, (uint32_t)k, col, s);
        return e;
    });
}

}  // namespace

bool tuned_shape(int kind, int L, int model, int n_rep, Shape *out) {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    if (g_shapes.empty()) return false;
    auto it = g_shapes.find(std::make_tuple(current_device(), kind, L, model, n_rep));
    if (it == g_shapes.end()) return false;
    *out = it->second;
    return true;
}

void set_tuned_shape(int kind, int L, int model, int n_rep, const Shape &sh) {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    g_shapes[std::make_tuple(current_device(), kind, L, model, n_rep)] = sh;
}

// Threads per workgroup for an edge, without measurement: about four draw
// groups per thread and colour, between one and eight waves.
int uneven2d_threads_default(int L) {
    const int groups = L * L / 16;
    int t = 64;
    while (t < 512 && 4 * t < groups) t <<= 1;
    return t;
}

// Autotuned workgroup size per (device, edge, model), measured once per
// process: the sweep kernel runs on scratch copies of up to 4096 replicas of
// the edge (enough workgroups to fill the chip) with every candidate size and
// the fastest is kept.  The choice changes
// the schedule only, never the results.  SPINMC_U2D_THREADS=n forces n;
// SPINMC_AUTOTUNE=0 takes the default without measuring.

int uneven2d_threads(StreamCtx &c, hipStream_t s, const Uneven2dArgs &a, int L, bool ea,
                     const std::vector<int32_t> &reps, const std::vector<smc_inst> &rows, int *out) {
    if (const char *f = getenv("SPINMC_U2D_THREADS")) {
        const int v = atoi(f);
        if (v == 64 || v == 128 || v == 256 || v == 512) {
            *out = v;
            return SMC_OK;
        }
    }
    const char *env = getenv("SPINMC_AUTOTUNE");
    if (env && env[0] == '0') {
        *out = uneven2d_threads_default(L);
        return SMC_OK;
    }
    int dev = 0;
    SMC_HIP(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, L, ea ? 1 : 0);
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            *out = it->second;
            return SMC_OK;
        }
    }
    // scratch copies of the first replicas of the edge (couplings are read in place)
    int rc;
    const int M = (int)std::min<size_t>(reps.size(), 4096);
    const int64_t N = (int64_t)L * L;
    void *sp = nullptr, *ip = nullptr, *wp = nullptr, *rp = nullptr, *ep = nullptr;
    if ((rc = ensure(c, kTuneSpins, (size_t)(M * N), &sp))) return rc;
    std::vector<smc_inst> tinst(M);
    std::vector<int32_t> twork(M), trows(M, 0);
    for (int m = 0; m < M; ++m) {
        tinst[m] = rows[reps[m]];
        tinst[m].spin_off = (int64_t)m * N;
        twork[m] = m;
    }
    // one copy per run of replicas that sit back to back in the caller's
    // array (the temperatures of a chain usually do)
    for (int m = 0; m < M;) {
        int e = m + 1;
        while (e < M && rows[reps[e]].spin_off == rows[reps[e - 1]].spin_off + N) ++e;
        SMC_HIP(hipMemcpyAsync((int8_t *)sp + (int64_t)m * N, a.spins + rows[reps[m]].spin_off,
                               (size_t)((int64_t)(e - m) * N), hipMemcpyDeviceToDevice, s));
        m = e;
    }
    if ((rc = upload(c, s, kTuneInst, tinst.data(), sizeof(smc_inst) * M, &ip))) return rc;
    if ((rc = upload(c, s, kTuneWork, twork.data(), sizeof(int32_t) * M, &wp))) return rc;
    if ((rc = upload(c, s, kTuneRows, trows.data(), sizeof(int32_t) * M, &rp))) return rc;
    if ((rc = ensure(c, kTuneE, sizeof(int64_t) * M, &ep))) return rc;
    Uneven2dArgs t = a;
    t.spins = (int8_t *)sp;
    t.inst = (const smc_inst *)ip;
    t.row_of_rep = (const int32_t *)rp;
    t.E = (int64_t *)ep;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SMC_HIP(hipEventCreate(&e0));
    SMC_HIP(hipEventCreate(&e1));
    int best = uneven2d_threads_default(L);
    float best_ms = 1e30f;
    hipError_t err = hipSuccess;
    for (int th = 64; th <= 512 && err == hipSuccess; th <<= 1) {
        err = launch_uneven2d_sweep(t, (const int32_t *)wp, M, L, ea, th, s);  // warm-up
        if (err == hipSuccess) err = hipEventRecord(e0, s);
        for (int k = 0; k < 3 && err == hipSuccess; ++k) err = launch_uneven2d_sweep(t, (const int32_t *)wp, M, L, ea, th, s);
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = th;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(SMC_EHIP, "autotuning the 2D sweep: %s", hipGetErrorString(err));
    {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        g_tuned[key] = best;
    }
    *out = best;
    return SMC_OK;
}

}  // namespace smc

extern "C" {

int smc_autotune(const smc_desc *desc, const char *cache_path, void *stream) {
    using namespace smc;
    last_error().clear();
    Plan plan;
    int rc = validate(desc, false, plan);
    if (rc) return rc;
    const bool ea = desc->model == SMC_EA;
    const int model = ea ? 1 : 0;
    const bool spin_model = desc->model == SMC_ISING || ea;
    // what this batch has to tune
    std::map<int, int> count;  // 2D edges of the LDS-resident kernel -> replicas
    if (desc->dim == 2 && spin_model)
        for (int r = 0; r < desc->n_rep; ++r) {
            const int L = desc->L > 0 ? desc->L : desc->inst[r].L;
            if (uneven2d_edge_supported(L)) ++count[L];
        }
    const bool band2d = desc->dim == 2 && desc->model == SMC_ISING && desc->L > 0 && lattice2d_supported(desc->L);
    const bool seg3d = desc->dim == 3 && spin_model && desc->L > 0 && sweep3d_shape(desc);
    const bool pass3d = seg3d && pass3d_enabled(desc);
    if (count.empty() && !band2d && !seg3d) return SMC_OK;
    const int dev = current_device();
    const std::string tag = device_tag(dev);
    std::vector<std::string> keep;  // lines of other devices
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char line[256];
            while (fgets(line, sizeof line, f)) {
                char t[160], kind[16];
                int L = 0, m = 0, n = 0, v0 = 0, v1 = 0, v2 = 0;
                if (line[0] == '#' ||
                    sscanf(line, "%159s %15s %d %d %d %d %d %d", t, kind, &L, &m, &n, &v0, &v1, &v2) != 8)
                    continue;
                if (tag != t) {
                    keep.emplace_back(line);
                    continue;
                }
                if (!strcmp(kind, "u2d")) {
                    if (uneven2d_edge_supported(L) && (m == 0 || m == 1) &&
                        (v0 == 64 || v0 == 128 || v0 == 256 || v0 == 512)) {
                        std::lock_guard<std::mutex> lk(g_tune_mutex);
                        g_tuned[std::make_tuple(dev, L, m)] = v0;
                    }
                    continue;
                }
                for (int k = 0; k < 3; ++k) {
                    if (strcmp(kind, kKindName[k]) || n < 1 || (m != 0 && m != 1)) continue;
                    const bool ok = k == kShapeBand2d   ? (lattice2d_supported(L) && v0 >= 4 && v0 % 4 == 0 && L % v0 == 0)
                                    : k == kShapePass3d ? pass3d_shape_valid(L, m == 1, v0, v1, v2)
                                                        : (sweep3d_supported(L) && (v0 == 1 || v0 == 2 || v0 == 4 ||
                                                                                    v0 == 8 || v0 == 16));
                    if (ok) set_tuned_shape(k, L, m, n, Shape{{v0, v1, v2}});
                }
            }
            fclose(f);
        }
    }
    // measure what is not known yet, on scratch lattices
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    SMC_HIP(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone) return fail(SMC_EINVAL, "smc_autotune cannot run under stream capture");
    StreamCtx &c = ctx_for(s);
    const Key key = make_key(desc->seed);
    Shape known;
    if (!count.empty()) {
        const ThrRow row = threshold_row(0.44, 2);
        void *tp = nullptr, *st = nullptr;
        if ((rc = upload(c, s, kTables, &row, sizeof row, &tp))) return rc;
        if ((rc = ensure(c, kStep, 2 * sizeof(uint32_t), &st))) return rc;
        SMC_HIP(launch_set_step((uint32_t *)st, 0u, s));
        for (auto &kv : count) {
            const int L = kv.first, M = std::min(kv.second, 4096);
            const int64_t N = (int64_t)L * L;
            void *sp = nullptr, *cp = nullptr;
            if ((rc = ensure(c, kPingPong, (size_t)(M * N), &sp))) return rc;
            SMC_HIP(hipMemsetAsync(sp, 0x01, (size_t)(M * N), s));
            if (ea) {
                if ((rc = ensure(c, kCoupSplit, (size_t)(2 * N), &cp))) return rc;
                SMC_HIP(hipMemsetAsync(cp, 0, (size_t)(2 * N), s));
            }
            std::vector<smc_inst> rows(M);
            std::vector<int32_t> reps(M);
            for (int m = 0; m < M; ++m) {
                rows[m] = smc_inst{L, 0, (int64_t)m * N, 0};
                reps[m] = m;
            }
            SMC_HIP(uneven2d_prepare_kernel(ea, L));
            const Uneven2dArgs a = make_uneven2d_args((int8_t *)sp, nullptr, (const uint8_t *)cp, nullptr,
                                                      (const ThrRow *)tp, nullptr, (const uint32_t *)st, key);
            int th = 0;
            if ((rc = uneven2d_threads(c, s, a, L, ea, reps, rows, &th))) return rc;
        }
    }
    if (band2d && !tuned_shape(kShapeBand2d, desc->L, 0, desc->n_rep, &known))
        if ((rc = tune_band2d(c, s, plan.b, key))) return rc;
    if (pass3d && !tuned_shape(kShapePass3d, desc->L, model, desc->n_rep, &known))
        if ((rc = tune_pass3d(c, s, plan.b, ea, plan.n_samples, key))) return rc;
    if (seg3d && !pass3d && !tuned_shape(kShapeHalf3d, desc->L, model, desc->n_rep, &known))
        if ((rc = tune_half3d(c, s, plan.b, ea, plan.n_samples, key))) return rc;
    // the tuner's scratch lattices are not kept (the sweeps allocate their own)
    if ((rc = release(c, kTuneA)) || (rc = release(c, kTuneB))) return rc;
    if ((band2d || seg3d) && (rc = release(c, kTuneSpins))) return rc;
    if (cache_path) {
        FILE *f = fopen(cache_path, "w");
        if (!f) return fail(SMC_EINVAL, "cannot write the autotune cache %s", cache_path);
        fprintf(f, "# spinmc autotune cache: device kind edge model(0 Ising, 1 EA) replicas v0 v1 v2\n"
                   "# u2d: workgroup size of the LDS-resident 2D sweep (replicas 0: any); band2d: rows per band of\n"
                   "# the one-pass 2D sweep; pass3d: rows per strip, segments per thread, planes per z segment of\n"
                   "# the one-pass 3D sweep; half3d: rows per thread of the 3D half-sweeps\n");
        for (const std::string &l : keep) fputs(l.c_str(), f);
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        for (const auto &kv : g_tuned)
            if (std::get<0>(kv.first) == dev)
                fprintf(f, "%s u2d %d %d 0 %d 0 0\n", tag.c_str(), std::get<1>(kv.first), std::get<2>(kv.first),
                        kv.second);
        for (const auto &kv : g_shapes)
            if (std::get<0>(kv.first) == dev)
                fprintf(f, "%s %s %d %d %d %d %d %d\n", tag.c_str(), kKindName[std::get<1>(kv.first)],
                        std::get<2>(kv.first), std::get<3>(kv.first), std::get<4>(kv.first), kv.second.v[0],
                        kv.second.v[1], kv.second.v[2]);
        fclose(f);
    }
    return SMC_OK;
}

}  // extern "C"

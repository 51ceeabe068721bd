// Parallel tempering of large uniform 2D Ising batches (Sec. 6) on the
// one-pass colour-split sweep (lattice2d.hip): the helpers that let the
// sweep kernel, which takes one threshold row per replica, follow the
// temperatures as they move between replicas.
//
// Per step: the threshold row of every replica is gathered from its current
// temperature (row_of_rep, kept by the exchange kernel), the m sweeps run,
// their energy changes are collected and added to the tracked energies, and
// the exchange round follows.  A chain whose slot_of_temp row is not a
// permutation (row_of_rep = -1) must be left unchanged: its replicas are
// swept with an arbitrary row (the sweep has no per-replica switch), but
// their energy changes are dropped and their spins are not copied back.
#include "internal.hpp"

namespace smc {
namespace {

__global__ __launch_bounds__(256) void k_pt_gather_thr(const ThrRow *rows, const int32_t *row_of_rep, ThrRow *out,
                                                       int n_rep) {
    const int r = (int)(blockIdx.x * 256 + threadIdx.x);
    if (r >= n_rep) return;
    const int row = row_of_rep[r];
    out[r] = rows[row >= 0 ? row : 0];
}

// E[r] += d[r] for replicas of valid chains; d[r] = 0 for the next step.
__global__ __launch_bounds__(256) void k_pt_add_masked(int64_t *d, int64_t *E, const int32_t *row_of_rep, int n_rep) {
    const int r = (int)(blockIdx.x * 256 + threadIdx.x);
    if (r >= n_rep) return;
    if (row_of_rep[r] >= 0) E[r] += d[r];
    d[r] = 0;
}

// dst replica r = src replica r (N bytes each, N a multiple of 16) for
// replicas of valid chains.
__global__ __launch_bounds__(256) void k_copy_valid(const int8_t *src, int8_t *dst, const int32_t *row_of_rep,
                                                    int64_t N, int n_rep) {
    const int64_t per = N / 16;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= per * n_rep) return;
    const int r = (int)(i / per);
    if (row_of_rep[r] < 0) return;
    ((uint4 *)dst)[i] = ((const uint4 *)src)[i];
}

__global__ __launch_bounds__(256) void k_zero64(int64_t *p, int n) {
    const int i = (int)(blockIdx.x * 256 + threadIdx.x);
    if (i < n) p[i] = 0;
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_pt_gather_thr(const ThrRow *rows, const int32_t *row_of_rep, ThrRow *out, int n_rep,
                                hipStream_t s) {
    SMC_LAUNCH(k_pt_gather_thr, dim3(blocks_of(n_rep)), dim3(256), 0, s, rows, row_of_rep, out, n_rep);
    return hipGetLastError();
}

hipError_t launch_pt_add_masked(int64_t *d, int64_t *E, const int32_t *row_of_rep, int n_rep, hipStream_t s) {
    SMC_LAUNCH(k_pt_add_masked, dim3(blocks_of(n_rep)), dim3(256), 0, s, d, E, row_of_rep, n_rep);
    return hipGetLastError();
}

hipError_t launch_copy_valid(const int8_t *src, int8_t *dst, const int32_t *row_of_rep, int64_t N, int n_rep,
                             hipStream_t s) {
    if (N % 16) return hipErrorInvalidValue;
    SMC_LAUNCH(k_copy_valid, dim3(blocks_of(N / 16 * n_rep)), dim3(256), 0, s, src, dst, row_of_rep, N,
                       n_rep);
    return hipGetLastError();
}

hipError_t launch_zero64(int64_t *p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    SMC_LAUNCH(k_zero64, dim3(blocks_of(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace smc

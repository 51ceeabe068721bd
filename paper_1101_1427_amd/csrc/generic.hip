// Generic kernels: initial state, per-site half-sweeps for any edge L and
// dimension, Heisenberg renormalisation, measurements and the
// parallel-tempering exchange.  The optimised kernels (lattice2d.hip,
// pt3d.hip) produce the same results; these serve every shape.
#include <string.h>

#include "heis_math.hpp"
#include "internal.hpp"

namespace smc {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int64_t n_sites(int dim, int L) {
    return dim == 3 ? (int64_t)L * L * L : (int64_t)L * L;
}

// Block-wide sum of an int64 (kBlock threads, wave64).
__device__ __forceinline__ long long block_sum_ll(long long v, long long *smem) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) smem[wave] = v;
    __syncthreads();
    long long tot = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += smem[w];
    return tot;  // valid in thread 0
}

__device__ __forceinline__ double block_sum_d(double v, double *smem) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) smem[wave] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += smem[w];
    return tot;
}

// Lattice position of the colour-c site of the pair (2h, 2h+1).
struct Site {
    int x, y, z;
    int64_t i;
};

__device__ __forceinline__ Site site_of_pair(int dim, int L, int64_t h, int c) {
    const int64_t i0 = 2 * h;
    Site st;
    st.x = (int)(i0 % L);
    const int64_t q = i0 / L;
    st.y = (int)(q % L);
    st.z = dim == 3 ? (int)(q / L) : 0;
    const int dx = ((st.y + st.z) & 1) ^ c;  // x of i0 is even
    st.x += dx;
    st.i = i0 + dx;
    return st;
}

// ------------------------------------------------------------------ init ----
__global__ __launch_bounds__(kBlock) void k_init_spins(Batch b, int8_t *spins, Key key, int bpr) {
    const int r = blockIdx.x / bpr;
    const smc_inst g = replica_geom(b, r);
    const int64_t N = n_sites(b.dim, g.L);
    const int64_t q = (int64_t)(blockIdx.x % bpr) * blockDim.x + threadIdx.x;  // group of 4 sites
    if (4 * q >= N) return;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)q, 0u, (uint32_t)r, 2 * kTagInit), key);
    int8_t *s = spins + g.spin_off + 4 * q;
    s[0] = (w.x >> 31) ? -1 : 1;
    s[1] = (w.y >> 31) ? -1 : 1;
    s[2] = (w.z >> 31) ? -1 : 1;
    s[3] = (w.w >> 31) ? -1 : 1;
}

__device__ __forceinline__ float3 sphere_point(float u0, float u1) {
    const float z = 2.0f * u0 - 1.0f;
    const float rho = sqrtf(1.0f - z * z);
    float sn, cs;
    sincospif(2.0f * u1, &sn, &cs);
    return make_float3(rho * cs, rho * sn, z);
}

__global__ __launch_bounds__(kBlock) void k_init_heis(Batch b, float *spins, Key key, int bpr) {
    const int r = blockIdx.x / bpr;
    const smc_inst g = replica_geom(b, r);
    const int64_t N = n_sites(b.dim, g.L);
    const int64_t i = (int64_t)(blockIdx.x % bpr) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)i, 0u, (uint32_t)r, 2 * kTagInit), key);
    const float3 p = sphere_point(unit23f(w.x), unit23f(w.y));
    float *s = spins + 3 * (g.spin_off + i);
    s[0] = p.x;
    s[1] = p.y;
    s[2] = p.z;
}

// samples[q] gives (L, sample id, -, coup_off) of every distinct sample.
__global__ __launch_bounds__(kBlock) void k_init_couplings(int dim, const smc_inst *samples, int8_t *coup, Key key, int bpr) {
    const smc_inst g = samples[blockIdx.x / bpr];
    const int64_t N = n_sites(dim, g.L);
    const int64_t q = (int64_t)(blockIdx.x % bpr) * blockDim.x + threadIdx.x;  // group of 4 bonds
    if (4 * q >= dim * N) return;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)q, 0u, (uint32_t)g.sample, 2 * kTagCoup), key);
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t bnd = 4 * q + j;
        if (bnd < dim * N) {
            const int64_t i = bnd / dim;
            const int mu = (int)(bnd - i * dim);
            coup[g.coup_off + mu * N + i] = (ws[j] >> 31) ? -1 : 1;
        }
    }
}

// ---------------------------------------------------- discrete half-sweep ----
__global__ __launch_bounds__(kBlock) void k_half_sweep_generic(SweepArgs a, int c, int bpr) {
    __shared__ long long red[kBlock / 64];
    const int r = blockIdx.x / bpr;
    const smc_inst g = replica_geom(a.b, r);
    const int L = g.L, dim = a.b.dim;
    const int64_t N = n_sites(dim, L);
    const int64_t h = (int64_t)(blockIdx.x % bpr) * blockDim.x + threadIdx.x;
    // a replica without a threshold row (its tempering chain is not a valid
    // permutation) is left unchanged
    const int row = a.row_of_rep ? a.row_of_rep[r] : r;
    int dE = 0;
    if (h < N / 2 && row >= 0) {
        int8_t *s = (int8_t *)a.spins + g.spin_off;
        const int8_t *J = a.coup ? a.coup + g.coup_off : nullptr;
        const Site st = site_of_pair(dim, L, h, c);
        const int64_t LL = L;
        const int64_t i = st.i;
        const int64_t ixp = i + (st.x == L - 1 ? 1 - LL : 1);
        const int64_t ixm = i - (st.x == 0 ? 1 - LL : 1);
        const int64_t iyp = i + (st.y == L - 1 ? (1 - LL) * LL : LL);
        const int64_t iym = i - (st.y == 0 ? (1 - LL) * LL : LL);
        int hf;
        if (J) {
            hf = J[i] * s[ixp] + J[ixm] * s[ixm] + J[N + i] * s[iyp] + J[N + iym] * s[iym];
        } else {
            hf = s[ixp] + s[ixm] + s[iyp] + s[iym];
        }
        if (dim == 3) {
            const int64_t P = LL * LL;
            const int64_t izp = i + (st.z == L - 1 ? (1 - LL) * P : P);
            const int64_t izm = i - (st.z == 0 ? (1 - LL) * P : P);
            hf += J ? J[2 * N + i] * s[izp] + J[2 * N + izm] * s[izm] : s[izp] + s[izm];
        }
        const int si = s[i];
        const int d = 2 * si * hf;
        bool acc = d <= 0;
        if (!acc) {
            const uint2 th = a.thr[row].m[d >> 2];
            const uint32_t rr = (uint32_t)r >> a.rng_shift;
            const uint4 w = philox4x32_10(make_uint4((uint32_t)(h >> 3), a.t, rr, 2 * kTagHead + c), a.key);
            acc = metropolis_accept(head16_of(w, (uint32_t)(h & 7)), th, (uint32_t)h, a.t, rr, c, a.key);
        }
        if (acc) {
            s[i] = (int8_t)(-si);
            dE = d;
        }
    }
    if (a.dE) {
        const long long tot = block_sum_ll(dE, red);
        if (threadIdx.x == 0 && tot != 0)
            atomicAdd((unsigned long long *)&a.dE[r], (unsigned long long)tot);
    }
}

// -------------------------------------------------- Heisenberg half-sweep ----
__device__ __forceinline__ float3 ld3(const float *s, int64_t i) {
    return make_float3(s[3 * i], s[3 * i + 1], s[3 * i + 2]);
}

__global__ __launch_bounds__(kBlock) void k_heis_half_sweep_generic(SweepArgs a, int c, int bpr) {
    __shared__ long long red[kBlock / 64];
    const int r = blockIdx.x / bpr;
    const smc_inst g = replica_geom(a.b, r);
    const int L = g.L, dim = a.b.dim;
    const int64_t N = n_sites(dim, L);
    const int64_t h = (int64_t)(blockIdx.x % bpr) * blockDim.x + threadIdx.x;
    int n_acc = 0;
    if (h < N / 2) {
        float *s = (float *)a.spins + 3 * g.spin_off;
        const Site st = site_of_pair(dim, L, h, c);
        const int64_t LL = L;
        const int64_t i = st.i;
        float3 hf = make_float3(0.f, 0.f, 0.f);
        auto add = [&](int64_t j) {
            const float3 v = ld3(s, j);
            hf.x += v.x;
            hf.y += v.y;
            hf.z += v.z;
        };
        add(i + (st.x == L - 1 ? 1 - LL : 1));
        add(i - (st.x == 0 ? 1 - LL : 1));
        add(i + (st.y == L - 1 ? (1 - LL) * LL : LL));
        add(i - (st.y == 0 ? (1 - LL) * LL : LL));
        if (dim == 3) {
            const int64_t P = LL * LL;
            add(i + (st.z == L - 1 ? (1 - LL) * P : P));
            add(i - (st.z == 0 ? (1 - LL) * P : P));
        }
        const uint4 w = philox4x32_10(make_uint4((uint32_t)h, a.t, (uint32_t)r, 2 * kTagHeis + c), a.key);
        const float3 sp = heis_proposal(unit23f(w.x), unit23f(w.y));
        const float3 so = ld3(s, i);
        const float dE = -((sp.x - so.x) * hf.x + (sp.y - so.y) * hf.y + (sp.z - so.z) * hf.z);
        const int row = a.row_of_rep ? a.row_of_rep[r] : r;
        const float beta = a.beta_f[row];
        if (dE <= 0.0f || unit23f(w.z) < heis_boltzmann(beta, dE)) {
            s[3 * i] = sp.x;
            s[3 * i + 1] = sp.y;
            s[3 * i + 2] = sp.z;
            n_acc = 1;
        }
    }
    if (a.dE) {
        const long long tot = block_sum_ll(n_acc, red);
        if (threadIdx.x == 0 && tot != 0)
            atomicAdd((unsigned long long *)&a.dE[r], (unsigned long long)tot);
    }
}

__global__ __launch_bounds__(kBlock) void k_heis_renorm(Batch b, float *spins, int bpr) {
    const int r = blockIdx.x / bpr;
    const smc_inst g = replica_geom(b, r);
    const int64_t N = n_sites(b.dim, g.L);
    const int64_t i = (int64_t)(blockIdx.x % bpr) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    float *s = spins + 3 * (g.spin_off + i);
    const float3 u = heis_unit(s[0], s[1], s[2]);
    s[0] = u.x;
    s[1] = u.y;
    s[2] = u.z;
}

// ------------------------------------------------------------ measurement ----
struct Partial {
    double e, mx, my, mz;
};

__global__ __launch_bounds__(kBlock) void k_measure_partials(Batch b, const void *spins, const int8_t *coup,
                                                             Partial *part, int nblk) {
    __shared__ double red[kBlock / 64];
    const int r = blockIdx.x / nblk;
    const int bx = blockIdx.x % nblk;
    const smc_inst g = replica_geom(b, r);
    const int L = g.L, dim = b.dim;
    const int64_t N = n_sites(dim, L);
    const int64_t LL = L;
    double e = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    if (b.model == SMC_HEISENBERG) {
        const float *s = (const float *)spins + 3 * g.spin_off;
        for (int64_t i = (int64_t)bx * blockDim.x + threadIdx.x; i < N; i += (int64_t)nblk * blockDim.x) {
            const int x = (int)(i % L);
            const int64_t q = i / L;
            const int y = (int)(q % L);
            const int z = dim == 3 ? (int)(q / L) : 0;
            const float3 si = ld3(s, i);
            const float3 a = ld3(s, i + (x == L - 1 ? 1 - LL : 1));
            const float3 bb = ld3(s, i + (y == L - 1 ? (1 - LL) * LL : LL));
            double loc = (double)si.x * a.x + (double)si.y * a.y + (double)si.z * a.z;
            loc += (double)si.x * bb.x + (double)si.y * bb.y + (double)si.z * bb.z;
            if (dim == 3) {
                const int64_t P = LL * LL;
                const float3 cc = ld3(s, i + (z == L - 1 ? (1 - LL) * P : P));
                loc += (double)si.x * cc.x + (double)si.y * cc.y + (double)si.z * cc.z;
            }
            e -= loc;
            mx += si.x;
            my += si.y;
            mz += si.z;
        }
    } else {
        const int8_t *s = (const int8_t *)spins + g.spin_off;
        const int8_t *J = coup ? coup + g.coup_off : nullptr;
        long long ei = 0, mi = 0;
        for (int64_t i = (int64_t)bx * blockDim.x + threadIdx.x; i < N; i += (int64_t)nblk * blockDim.x) {
            const int x = (int)(i % L);
            const int64_t q = i / L;
            const int y = (int)(q % L);
            const int z = dim == 3 ? (int)(q / L) : 0;
            const int si = s[i];
            const int a = s[i + (x == L - 1 ? 1 - LL : 1)];
            const int bb = s[i + (y == L - 1 ? (1 - LL) * LL : LL)];
            int loc = J ? J[i] * a + J[N + i] * bb : a + bb;
            if (dim == 3) {
                const int64_t P = LL * LL;
                const int cc = s[i + (z == L - 1 ? (1 - LL) * P : P)];
                loc += J ? J[2 * N + i] * cc : cc;
            }
            ei -= si * loc;
            mi += si;
        }
        e = (double)ei;  // exact: |partial| < 2^53
        mx = (double)mi;
    }
    const double te = block_sum_d(e, red);
    const double tx = block_sum_d(mx, red);
    const double ty = block_sum_d(my, red);
    const double tz = block_sum_d(mz, red);
    if (threadIdx.x == 0) part[(int64_t)r * nblk + bx] = Partial{te, tx, ty, tz};
}

__global__ void k_measure_final(int n_rep, int nblk, int vec, const Partial *part, double *energy, double *magnet) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rep) return;
    double e = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    for (int k = 0; k < nblk; ++k) {
        const Partial p = part[(int64_t)r * nblk + k];
        e += p.e;
        mx += p.mx;
        my += p.my;
        mz += p.mz;
    }
    energy[r] = e;
    if (magnet) {
        if (vec) {
            magnet[3 * r] = mx;
            magnet[3 * r + 1] = my;
            magnet[3 * r + 2] = mz;
        } else {
            magnet[r] = mx;
        }
    }
}

int measure_blocks(const Batch &b, int max_L) {
    const int64_t N = b.dim == 3 ? (int64_t)max_L * max_L * max_L : (int64_t)max_L * max_L;
    int64_t nb = (N + 4095) / 4096;
    if (nb < 1) nb = 1;
    if (nb > 2048) nb = 2048;
    return (int)nb;
}

// -------------------------------------------------------- parallel tempering --
// Energies in, and the threshold row of every replica from the chain's
// permutation; a chain whose slot_of_temp row is not a permutation gets row
// -1 for all its replicas, and the sweeps and exchanges leave it unchanged.
__global__ void k_pt_prepare(SwapArgs a, const double *energy_in) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n_chains) return;
    const int n = a.n_temps;
    const int base = a.beta_per_chain ? q * n : 0;
    for (int k = 0; k < n; ++k) {
        a.E[q * n + k] = (int64_t)energy_in[q * n + k];
        a.row_of_rep[q * n + k] = -1;
    }
    bool ok = true;
    for (int k = 0; k < n; ++k) {
        const int slot = a.slot_of_temp[q * n + k];
        if ((unsigned)slot >= (unsigned)n || a.row_of_rep[q * n + slot] >= 0) {
            ok = false;
            break;
        }
        a.row_of_rep[q * n + slot] = base + k;
    }
    if (!ok)
        for (int k = 0; k < n; ++k) a.row_of_rep[q * n + k] = -1;
}

__global__ void k_pt_swap(SwapArgs a) {
#pragma clang fp contract(off)
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n_chains) return;
    a.t = a.t_dev ? *a.t_dev : a.t;
    const int n = a.n_temps;
    const int base = a.beta_per_chain ? q * n : 0;
    int32_t *sot = a.slot_of_temp + (int64_t)q * n;
    if (a.row_of_rep[q * n] < 0) return;  // not a permutation: chain left unchanged
    for (int k = (int)(a.t & 1u); k + 1 < n; k += 2) {
        const int A = sot[k], B = sot[k + 1];
        const double x = (a.beta[base + k + 1] - a.beta[base + k]) * (double)(a.E[q * n + B] - a.E[q * n + A]);
        bool accept = x >= 0.0;
        if (!accept) {
            const uint4 w = philox4x32_10(make_uint4((uint32_t)k, a.t, (uint32_t)q, 2 * kTagSwap), a.key);
            accept = unit53(w.x, w.y) < exp(x);
        }
        if (accept) {
            sot[k] = B;
            sot[k + 1] = A;
            a.row_of_rep[q * n + B] = base + k;
            a.row_of_rep[q * n + A] = base + k + 1;
            if (a.acc) a.acc[(int64_t)q * (n - 1) + k] += 1ull;
        }
    }
}

__global__ void k_pt_finish(SwapArgs a, double *energy_out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.n_chains * a.n_temps) return;
    energy_out[r] = (double)a.E[r];
}

int64_t sites_of(int dim, int L) { return dim == 3 ? (int64_t)L * L * L : (int64_t)L * L; }

// Blocks per replica for kBlock threads covering `work` items, and the
// flattened grid of n_rep replicas.
int blocks_for(int64_t work) { return (int)((work + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_init_spins(const Batch &b, int max_L, int8_t *spins, Key key, hipStream_t s) {
    const int bpr = blocks_for((sites_of(b.dim, max_L) + 3) / 4);
    SMC_LAUNCH(k_init_spins, dim3(bpr * b.n_rep), dim3(kBlock), 0, s, b, spins, key, bpr);
    return hipGetLastError();
}

hipError_t launch_init_heis(const Batch &b, int max_L, float *spins, Key key, hipStream_t s) {
    const int bpr = blocks_for(sites_of(b.dim, max_L));
    SMC_LAUNCH(k_init_heis, dim3(bpr * b.n_rep), dim3(kBlock), 0, s, b, spins, key, bpr);
    return hipGetLastError();
}

hipError_t launch_init_couplings(int dim, int n_samples, const smc_inst *samples_dev, int max_L, int8_t *coup,
                                 Key key, hipStream_t s) {
    const int bpr = blocks_for((dim * sites_of(dim, max_L) + 3) / 4);
    SMC_LAUNCH(k_init_couplings, dim3(bpr * n_samples), dim3(kBlock), 0, s, dim, samples_dev, coup, key,
                       bpr);
    return hipGetLastError();
}

hipError_t launch_half_sweep_generic(const SweepArgs &a, int c, hipStream_t s) {
    const int bpr = blocks_for(sites_of(a.b.dim, a.max_L) / 2);
    SMC_LAUNCH(k_half_sweep_generic, dim3(bpr * a.b.n_rep), dim3(kBlock), 0, s, a, c, bpr);
    return hipGetLastError();
}

hipError_t launch_heis_half_sweep_generic(const SweepArgs &a, int c, hipStream_t s) {
    const int bpr = blocks_for(sites_of(a.b.dim, a.max_L) / 2);
    SMC_LAUNCH(k_heis_half_sweep_generic, dim3(bpr * a.b.n_rep), dim3(kBlock), 0, s, a, c, bpr);
    return hipGetLastError();
}

hipError_t launch_heis_renorm(const Batch &b, float *spins, int max_L, hipStream_t s) {
    const int bpr = blocks_for(sites_of(b.dim, max_L));
    SMC_LAUNCH(k_heis_renorm, dim3(bpr * b.n_rep), dim3(kBlock), 0, s, b, spins, bpr);
    return hipGetLastError();
}

size_t measure_scratch_bytes(const Batch &b, int max_L) {
    return (size_t)measure_blocks(b, max_L) * (size_t)b.n_rep * sizeof(Partial);
}

hipError_t launch_measure(const Batch &b, const void *spins, const int8_t *coup, int max_L, double *energy,
                          double *magnet, void *scratch, size_t scratch_bytes, hipStream_t s) {
    const int nblk = measure_blocks(b, max_L);
    if (scratch_bytes < measure_scratch_bytes(b, max_L)) return hipErrorInvalidValue;
    Partial *part = (Partial *)scratch;
    SMC_LAUNCH(k_measure_partials, dim3(nblk * b.n_rep), dim3(kBlock), 0, s, b, spins, coup, part, nblk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    SMC_LAUNCH(k_measure_final, dim3((b.n_rep + 255) / 256), dim3(256), 0, s, b.n_rep, nblk,
                       b.model == SMC_HEISENBERG ? 1 : 0, part, energy, magnet);
    return hipGetLastError();
}

hipError_t launch_pt_prepare(const SwapArgs &a, const double *energy_in, hipStream_t s) {
    SMC_LAUNCH(k_pt_prepare, dim3((a.n_chains + 255) / 256), dim3(256), 0, s, a, energy_in);
    return hipGetLastError();
}

hipError_t launch_pt_swap(const SwapArgs &a, hipStream_t s) {
    SMC_LAUNCH(k_pt_swap, dim3((a.n_chains + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t add_pt_swap_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, size_t n_deps,
                            const SwapArgs &a) {
    SwapArgs args = a;
    void *params[] = {&args};
    hipKernelNodeParams p;
    memset(&p, 0, sizeof p);
    p.func = (void *)k_pt_swap;
    p.gridDim = dim3((unsigned)((a.n_chains + 255) / 256));
    p.blockDim = dim3(256);
    p.kernelParams = params;
    if (const char *why = launch_config_error(p.gridDim.x, 256, 0))
        return reject_launch("k_pt_swap (graph node)", p.gridDim.x, 256, 0, why);
    return hipGraphAddKernelNode(node, g, deps, n_deps, &p);
}

hipError_t launch_pt_finish(const SwapArgs &a, double *energy_out, hipStream_t s) {
    const int n = a.n_chains * a.n_temps;
    SMC_LAUNCH(k_pt_finish, dim3((n + 255) / 256), dim3(256), 0, s, a, energy_out);
    return hipGetLastError();
}

}  // namespace smc

// Heisenberg half-sweeps of uniform 3D batches whose edge is a power of two
// (Sec. 4, Eq. 10): the same update as the generic kernel (same proposal
// and acceptance functions, same float32 arithmetic in the same order, same
// random numbers), with 32-bit shift/mask indexing instead of 64-bit
// divisions and one 12-byte load per neighbour.  A thread handles the
// colour-c sites of site pairs (2p, 2p+1), whose in-colour index is p.
#include "heis_math.hpp"
#include "internal.hpp"

namespace smc {
namespace {

constexpr int kThreads = 256;

struct Heis3dArgs {
    float *spins;       // [n_rep][N][3]
    const float *beta;  // per replica (float32)
    int64_t *acc;       // per replica: += accepted moves, or nullptr
    Key key;
    uint32_t t;
    int lgL;            // log2 of the edge
    int64_t N;          // sites per replica
    int bpr;            // blocks per replica
};

struct F3 {
    float x, y, z;
};

__device__ __forceinline__ F3 ld(const float *s, uint32_t i) { return *(const F3 *)(s + 3 * (size_t)i); }

// The loads of one site: its six neighbours and itself.
struct SiteLoads {
    F3 nb[6];
    F3 so;
};

__device__ __forceinline__ SiteLoads load_site(const float *s, uint32_t p, int lgL, int c, uint32_t &i) {
    const uint32_t L = 1u << lgL, m = L - 1u;
    const uint32_t row = p >> (lgL - 1), pi = p & ((L >> 1) - 1u);
    const uint32_t y = row & m, z = row >> lgL;
    const uint32_t x = 2u * pi + (((y ^ z) & 1u) ^ (uint32_t)c);
    const uint32_t base = row << lgL;  // site (0, y, z)
    const uint32_t P = L << lgL;       // sites per z plane
    i = base + x;
    SiteLoads l;
    // neighbours in the order of the generic kernel: +x, -x, +y, -y, +z, -z
    l.nb[0] = ld(s, base + ((x + 1u) & m));
    l.nb[1] = ld(s, base + ((x - 1u) & m));
    l.nb[2] = ld(s, i - y * L + ((y + 1u) & m) * L);
    l.nb[3] = ld(s, i - y * L + ((y - 1u) & m) * L);
    l.nb[4] = ld(s, i - z * P + ((z + 1u) & m) * P);
    l.nb[5] = ld(s, i - z * P + ((z - 1u) & m) * P);
    l.so = ld(s, i);
    return l;
}

// Each thread updates kSitesPerThread sites (pairs p, p + kThreads, ...) and
// issues all their loads before the first update, so that a wave keeps
// several loads per lane in flight.
constexpr int kSitesPerThread = 4;

__global__ __launch_bounds__(kThreads) void k_heis3d_half(Heis3dArgs a, int c) {
    __shared__ int red[kThreads / 64];
    const int r = blockIdx.x / a.bpr;
    const uint32_t p0 = (uint32_t)(blockIdx.x % a.bpr) * (kThreads * kSitesPerThread) + threadIdx.x;
    float *s = a.spins + (size_t)r * 3 * (size_t)a.N;
    const int64_t pairs = a.N / 2;
    SiteLoads l[kSitesPerThread];
    uint32_t idx[kSitesPerThread];
#pragma unroll
    for (int q = 0; q < kSitesPerThread; ++q) {
        const uint32_t p = p0 + (uint32_t)(q * kThreads);
        if ((int64_t)p < pairs) l[q] = load_site(s, p, a.lgL, c, idx[q]);
    }
    const float beta = a.beta[r];
    int n_acc = 0;
#pragma unroll
    for (int q = 0; q < kSitesPerThread; ++q) {
        const uint32_t p = p0 + (uint32_t)(q * kThreads);
        if ((int64_t)p >= pairs) continue;
        float3 hf = make_float3(0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            hf.x += l[q].nb[k].x;
            hf.y += l[q].nb[k].y;
            hf.z += l[q].nb[k].z;
        }
        const F3 so = l[q].so;
        const uint4 w = philox4x32_10(make_uint4(p, a.t, (uint32_t)r, 2 * kTagHeis + (uint32_t)c), a.key);
        const float3 sp = heis_proposal(unit23f(w.x), unit23f(w.y));
        const float dE = -((sp.x - so.x) * hf.x + (sp.y - so.y) * hf.y + (sp.z - so.z) * hf.z);
        if (dE <= 0.0f || unit23f(w.z) < heis_boltzmann(beta, dE)) {
            F3 v;
            v.x = sp.x;
            v.y = sp.y;
            v.z = sp.z;
            *(F3 *)(s + 3 * (size_t)idx[q]) = v;
            ++n_acc;
        }
    }
    if (a.acc) {
        int v = n_acc;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            const int tot = red[0] + red[1] + red[2] + red[3];
            if (tot) atomicAdd((unsigned long long *)&a.acc[r], (unsigned long long)tot);
        }
    }
}

}  // namespace

bool heis3d_supported(int dim, int L) { return dim == 3 && L >= 4 && L <= 1024 && (L & (L - 1)) == 0; }

hipError_t launch_heis3d_half(float *spins, const float *beta, int64_t *acc, int n_rep, int L, Key key, uint32_t t,
                              int c, hipStream_t s) {
    Heis3dArgs a;
    a.spins = spins;
    a.beta = beta;
    a.acc = acc;
    a.key = key;
    a.t = t;
    a.lgL = 0;
    while ((1 << a.lgL) < L) ++a.lgL;
    a.N = (int64_t)L * L * L;
    a.bpr = (int)((a.N / 2 + kThreads * kSitesPerThread - 1) / (kThreads * kSitesPerThread));
    hipLaunchKernelGGL(k_heis3d_half, dim3((unsigned)(a.bpr * n_rep)), dim3(kThreads), 0, s, a, c);
    return hipGetLastError();
}

}  // namespace smc

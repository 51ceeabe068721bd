// Double checkerboard sweeps with multi-hit updates (Sec. 3.2, Sec. 3.4) of
// 2D Ising and +-J EA lattices.  The lattice is cut into T x T tiles whose
// tile colour is (bx + by) & 1.  A sweep is two launches, one per tile
// colour; a workgroup loads its tile and a one-site halo into LDS, gives the
// tile k hits (colour-0 sites, then colour-1 sites, each a Metropolis
// attempt with the halo held fixed) and writes the tile back in place:
// tiles of one colour share no bond, so each launch reads only spins it
// does not write (a lattice of one tile refreshes its wrapped halo after
// every half-hit instead).  With the palindromic order, odd sweeps run both
// orders backwards.
//
// Random numbers: hit j of sweep t uses the plain sweep's draws of "sweep"
// t*k + j: the 16-bit head of in-colour site h is half h & 7 of the block
// (h/8, t*k + j, r, 6 + c); a head equal to the high half of the threshold
// takes the 16-bit tail of (h, t*k + j, r, 8 + c).  A thread handles the
// eight in-colour sites of one such block (16 consecutive columns of a tile
// row), so T is a multiple of 16.
#include "internal.hpp"

namespace smc {
namespace {

constexpr int kDcbMaxThreads = 1024;

struct DcbArgs {
    int8_t *spins;         // caller's spins, replica r at r * N (updated in place)
    const int8_t *coup;    // EA couplings [sample][2][N], replica r using sample r / rep_per_sample, or nullptr
    int rep_per_sample;
    const ThrRow *thr;     // per replica
    int64_t *dE_slots;     // [n_rep][2 * tiles_per_colour] partial sums, or nullptr
    Key key;
    uint32_t t;            // sweep index
    int k;                 // hits per tile
    int L, T, B;           // edge, tile edge, tiles per direction
    int tile_colour;
    int rev;               // 1: colour-1 sites first
    int tiles_per_colour;
};

__global__ __launch_bounds__(kDcbMaxThreads) void k_dcb2d(DcbArgs a) {
    extern __shared__ __align__(16) int8_t smem[];  // spins, bonds to +x, bonds to +y: (T+2)^2 each
    __shared__ long long red[kDcbMaxThreads / 64];
    const int L = a.L, T = a.T, W = T + 2;
    const int r = (int)blockIdx.x / a.tiles_per_colour;
    const int ti = (int)blockIdx.x % a.tiles_per_colour;
    // ti-th tile of the tile colour in row-major tile order
    int bx, by;
    if (a.B == 1) {
        bx = by = 0;
    } else {
        const int half = a.B / 2;  // tiles of one colour per tile row
        by = ti / half;
        bx = 2 * (ti % half) + ((by + a.tile_colour) & 1);
    }
    const int x0 = bx * T, y0 = by * T;
    const int64_t N = (int64_t)L * L;
    int8_t *S = a.spins + (int64_t)r * N;
    const int8_t *Jx = a.coup ? a.coup + (int64_t)(r / a.rep_per_sample) * 2 * N : nullptr;
    const int8_t *Jy = Jx ? Jx + N : nullptr;
    int8_t *ts = smem, *tx = smem + W * W, *ty = smem + 2 * W * W;
    // tile and halo: cell (u, v) of the staged square is site (x0 + u - 1, y0 + v - 1) mod L
    for (int q = threadIdx.x; q < W * W; q += blockDim.x) {
        const int v = q / W, u = q % W;
        const int x = (x0 + u - 1 + L) % L, y = (y0 + v - 1 + L) % L;
        const int64_t i = (int64_t)y * L + x;
        ts[q] = S[i];
        tx[q] = Jx ? Jx[i] : (int8_t)1;
        ty[q] = Jy ? Jy[i] : (int8_t)1;
    }
    const ThrRow th = a.thr[r];
    __syncthreads();

    const int segs = T / 16;
    const int v = (int)threadIdx.x / segs, seg = (int)threadIdx.x % segs;
    const int y = y0 + v;
    long long dE = 0;
    for (int j = 0; j < a.k; ++j) {
        const uint32_t tj = a.t * (uint32_t)a.k + (uint32_t)j;
        for (int ci = 0; ci < 2; ++ci) {
            const int c = a.rev ? 1 - ci : ci;
            // in-colour sites h0 .. h0+7: columns x0 + 16 seg + 2m + ((c + y) & 1)
            const uint32_t h0 = (uint32_t)(y * (L / 2) + x0 / 2 + 8 * seg);
            const uint4 w = philox4x32_10(make_uint4(h0 >> 3, tj, (uint32_t)r, 2 * kTagHead + (uint32_t)c), a.key);
            const int off = (c + y) & 1;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int u = 16 * seg + 2 * m + off;  // tile column
                const int q = (v + 1) * W + (u + 1);
                const int s = ts[q];
                const int hsum = tx[q] * ts[q + 1] + tx[q - 1] * ts[q - 1] + ty[q] * ts[q + W] + ty[q - W] * ts[q - W];
                const int d = 2 * s * hsum;
                bool flip = d <= 0;
                if (!flip) {
                    const uint32_t word = m < 2 ? w.x : m < 4 ? w.y : m < 6 ? w.z : w.w;
                    const uint32_t head = (m & 1) ? (word >> 16) : (word & 0xFFFFu);
                    flip = metropolis_accept(head, th.m[d >> 2], h0 + (uint32_t)m, tj, (uint32_t)r, (uint32_t)c, a.key);
                }
                if (flip) {
                    ts[q] = (int8_t)(-s);
                    dE += d;
                }
            }
            __syncthreads();
            if (a.B == 1) {
                // a single tile: its halo wraps onto its own sites, so the
                // halo copies take the values just updated
                for (int e = threadIdx.x; e < 4 * W; e += blockDim.x) {
                    const int side = e / W, p = e % W;
                    const int hv = side == 0 ? 0 : side == 1 ? W - 1 : p;
                    const int hu = side == 2 ? 0 : side == 3 ? W - 1 : p;
                    const int sv = (hv + T - 1) % T + 1, su = (hu + T - 1) % T + 1;
                    ts[hv * W + hu] = ts[sv * W + su];
                }
                __syncthreads();
            }
        }
    }
    // the tile back, in place
    for (int q = threadIdx.x; q < T * T; q += blockDim.x) {
        const int vv = q / T, u = q % T;
        S[(int64_t)(y0 + vv) * L + (x0 + u)] = ts[(vv + 1) * W + (u + 1)];
    }
    if (a.dE_slots) {
        long long tot = dE;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long sum = 0;
            for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) sum += red[w];
            // this workgroup's own slot (tile index and tile colour): no atomics
            int64_t *slot = a.dE_slots + (int64_t)r * 2 * a.tiles_per_colour + a.tile_colour * a.tiles_per_colour + ti;
            *slot += sum;
        }
    }
}

__global__ __launch_bounds__(256) void k_dcb_zero(int64_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// dE[r] += the sum of replica r's slots.
__global__ __launch_bounds__(256) void k_dcb_collect(const int64_t *slots, int64_t *dE, int per_rep) {
    __shared__ long long red[4];
    const int r = (int)blockIdx.x;
    long long v = 0;
    for (int i = (int)threadIdx.x; i < per_rep; i += 256) v += slots[(int64_t)r * per_rep + i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) dE[r] += red[0] + red[1] + red[2] + red[3];
}

}  // namespace

bool dcb2d_supported(int L, int T) {
    if (T < 16 || T > 128 || T % 16 || L % T) return false;
    const int B = L / T;
    return B == 1 || B % 2 == 0;
}

int dcb2d_tiles_per_colour(int L, int T) {
    const int B = L / T;
    return B == 1 ? 1 : B * B / 2;
}

hipError_t launch_dcb_zero(int64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dcb_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_dcb_collect(const int64_t *slots, int64_t *dE, int n_rep, int per_rep, hipStream_t s) {
    hipLaunchKernelGGL(k_dcb_collect, dim3((unsigned)n_rep), dim3(256), 0, s, slots, dE, per_rep);
    return hipGetLastError();
}

hipError_t launch_dcb2d(int8_t *spins, const int8_t *coup, int rep_per_sample, const ThrRow *thr, int64_t *dE_slots,
                        int n_rep, int L, int T, int k, Key key, uint32_t t, int tile_colour, bool rev, hipStream_t s) {
    if (!dcb2d_supported(L, T) || k < 1 || rep_per_sample < 1) return hipErrorInvalidValue;
    DcbArgs a;
    a.spins = spins;
    a.coup = coup;
    a.rep_per_sample = rep_per_sample;
    a.thr = thr;
    a.dE_slots = dE_slots;
    a.key = key;
    a.t = t;
    a.k = k;
    a.L = L;
    a.T = T;
    a.B = L / T;
    a.tile_colour = tile_colour;
    a.rev = rev ? 1 : 0;
    a.tiles_per_colour = dcb2d_tiles_per_colour(L, T);
    if (a.B == 1 && tile_colour == 1) return hipSuccess;  // one tile, of tile colour 0
    const unsigned threads = (unsigned)(T * T / 16);
    const size_t lds = (size_t)3 * (T + 2) * (T + 2);
    const unsigned blocks = (unsigned)(n_rep * a.tiles_per_colour);
    hipLaunchKernelGGL(k_dcb2d, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

}  // namespace smc

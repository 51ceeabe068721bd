// Double checkerboard sweeps with multi-hit updates of 3D Ising and +-J EA
// lattices (the tiled update of Sec. 3.2 and Sec. 3.4 carried over to three
// dimensions).  The lattice is cut into 16 x 16 x 16 tiles of tile colour
// (bx + by + bz) & 1; a sweep is two launches, one per tile colour.  A
// workgroup stages its tile with a one-site halo (and the bonds, for EA) in
// LDS, gives the tile k hits (colour-0 sites, x + y + z even, then colour-1
// sites, the halo held fixed) and writes the tile back in place.  A lattice
// of one tile refreshes its wrapped halo after every half-hit instead.
//
// Random numbers: hit j of sweep t draws as plain sweep t*k + j.  A thread
// owns one 16-site row segment of the tile (x0 .. x0 + 15 at fixed y, z):
// its eight colour-c sites are the in-colour indices h0 .. h0 + 7 of one
// Philox block (h0 / 8, t*k + j, r, 6 + c).
#include "internal.hpp"

namespace smc {
namespace {

constexpr int kT3 = 16;                 // tile edge
constexpr int kW3 = kT3 + 2;            // staged cube edge
constexpr int kCube = kW3 * kW3 * kW3;  // staged sites
constexpr int kThreads3 = kT3 * kT3;    // one row segment per thread

struct Dcb3dArgs {
    int8_t *spins;         // replica r at r * N (updated in place)
    const int8_t *coup;    // EA couplings [sample][3][N], or nullptr
    int rep_per_sample;
    const ThrRow *thr;     // per replica
    int64_t *dE_slots;     // [n_rep][2 * tiles_per_colour], or nullptr
    Key key;
    uint32_t t;
    int k, L, B;
    int tile_colour, rev, tiles_per_colour;
};

__device__ __forceinline__ int cube(int u, int v, int w) { return (w * kW3 + v) * kW3 + u; }

__global__ __launch_bounds__(kThreads3) void k_dcb3d(Dcb3dArgs a) {
    // spins, bonds to +x, +y, +z of every staged site
    __shared__ int8_t ts[kCube], tx[kCube], ty[kCube], tz[kCube];
    __shared__ long long red[kThreads3 / 64];
    const int L = a.L;
    const int r = (int)blockIdx.x / a.tiles_per_colour;
    const int ti = (int)blockIdx.x % a.tiles_per_colour;
    int bx = 0, by = 0, bz = 0;
    if (a.B > 1) {
        const int half = a.B / 2, row = ti / half;  // row = bz * B + by
        bz = row / a.B;
        by = row % a.B;
        bx = 2 * (ti % half) + ((by + bz + a.tile_colour) & 1);
    }
    const int x0 = bx * kT3, y0 = by * kT3, z0 = bz * kT3;
    const int64_t N = (int64_t)L * L * L;
    int8_t *S = a.spins + (int64_t)r * N;
    const int8_t *J = a.coup ? a.coup + (int64_t)(r / a.rep_per_sample) * 3 * N : nullptr;
    // staged cell (u, v, w) = site (x0 + u - 1, y0 + v - 1, z0 + w - 1) mod L
    for (int q = threadIdx.x; q < kCube; q += kThreads3) {
        const int u = q % kW3, v = (q / kW3) % kW3, w = q / (kW3 * kW3);
        const int x = (x0 + u - 1 + L) % L, y = (y0 + v - 1 + L) % L, z = (z0 + w - 1 + L) % L;
        const int64_t i = ((int64_t)z * L + y) * L + x;
        ts[q] = S[i];
        tx[q] = J ? J[i] : (int8_t)1;
        ty[q] = J ? J[N + i] : (int8_t)1;
        tz[q] = J ? J[2 * N + i] : (int8_t)1;
    }
    const ThrRow th = a.thr[r];
    __syncthreads();

    const int v = (int)threadIdx.x % kT3, w = (int)threadIdx.x / kT3;  // the thread's row (y0 + v, z0 + w)
    const int y = y0 + v, z = z0 + w;
    const uint32_t h0 = (uint32_t)((((int64_t)z * L + y) * L + x0) >> 1);
    long long dE = 0;
    for (int j = 0; j < a.k; ++j) {
        const uint32_t tj = a.t * (uint32_t)a.k + (uint32_t)j;
        for (int ci = 0; ci < 2; ++ci) {
            const int c = a.rev ? 1 - ci : ci;
            const uint4 wd = philox4x32_10(make_uint4(h0 >> 3, tj, (uint32_t)r, 2 * kTagHead + (uint32_t)c), a.key);
            const int off = (c + y + z) & 1;  // x0 is even
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int q = cube(2 * m + off + 1, v + 1, w + 1);
                const int s = ts[q];
                const int hsum = tx[q] * ts[q + 1] + tx[q - 1] * ts[q - 1] + ty[q] * ts[q + kW3] +
                                 ty[q - kW3] * ts[q - kW3] + tz[q] * ts[q + kW3 * kW3] +
                                 tz[q - kW3 * kW3] * ts[q - kW3 * kW3];
                const int d = 2 * s * hsum;
                bool flip = d <= 0;
                if (!flip) {
                    const uint32_t word = m < 2 ? wd.x : m < 4 ? wd.y : m < 6 ? wd.z : wd.w;
                    const uint32_t head = (m & 1) ? (word >> 16) : (word & 0xFFFFu);
                    const uint2 tr = d == 4 ? th.m[1] : d == 8 ? th.m[2] : th.m[3];
                    flip = metropolis_accept(head, tr, h0 + (uint32_t)m, tj, (uint32_t)r, (uint32_t)c, a.key);
                }
                if (flip) {
                    ts[q] = (int8_t)(-s);
                    dE += d;
                }
            }
            __syncthreads();
            if (a.B == 1) {
                // a single tile: the halo copies take the values just updated
                for (int q = threadIdx.x; q < kCube; q += kThreads3) {
                    const int u = q % kW3, vv = (q / kW3) % kW3, ww = q / (kW3 * kW3);
                    if (u >= 1 && u <= kT3 && vv >= 1 && vv <= kT3 && ww >= 1 && ww <= kT3) continue;
                    const int su = (u + kT3 - 1) % kT3 + 1, sv = (vv + kT3 - 1) % kT3 + 1,
                              sw = (ww + kT3 - 1) % kT3 + 1;
                    ts[q] = ts[cube(su, sv, sw)];
                }
                __syncthreads();
            }
        }
    }
    // the tile back, in place
    for (int q = threadIdx.x; q < kT3 * kT3 * kT3; q += kThreads3) {
        const int u = q % kT3, vv = (q / kT3) % kT3, ww = q / (kT3 * kT3);
        S[((int64_t)(z0 + ww) * L + (y0 + vv)) * L + (x0 + u)] = ts[cube(u + 1, vv + 1, ww + 1)];
    }
    if (a.dE_slots) {
        long long tot = dE;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long sum = 0;
            for (int i = 0; i < kThreads3 / 64; ++i) sum += red[i];
            a.dE_slots[(int64_t)r * 2 * a.tiles_per_colour + a.tile_colour * a.tiles_per_colour + ti] += sum;
        }
    }
}

}  // namespace

bool dcb3d_supported(int L, int T) {
    if (T != kT3 || L % T) return false;
    const int B = L / T;
    return B == 1 || B % 2 == 0;
}

int dcb3d_tiles_per_colour(int L, int T) {
    const int B = L / T;
    return B == 1 ? 1 : B * B * B / 2;
}

hipError_t launch_dcb3d(int8_t *spins, const int8_t *coup, int rep_per_sample, const ThrRow *thr, int64_t *dE_slots,
                        int n_rep, int L, int T, int k, Key key, uint32_t t, int tile_colour, bool rev,
                        hipStream_t s) {
    if (!dcb3d_supported(L, T) || k < 1 || rep_per_sample < 1) return hipErrorInvalidValue;
    const int B = L / T;
    if (B == 1 && tile_colour == 1) return hipSuccess;  // one tile, of tile colour 0
    Dcb3dArgs a;
    a.spins = spins;
    a.coup = coup;
    a.rep_per_sample = rep_per_sample;
    a.thr = thr;
    a.dE_slots = dE_slots;
    a.key = key;
    a.t = t;
    a.k = k;
    a.L = L;
    a.B = B;
    a.tile_colour = tile_colour;
    a.rev = rev ? 1 : 0;
    a.tiles_per_colour = dcb3d_tiles_per_colour(L, T);
    const unsigned blocks = (unsigned)(n_rep * a.tiles_per_colour);
    hipLaunchKernelGGL(k_dcb3d, dim3(blocks), dim3(kThreads3), 0, s, a);
    return hipGetLastError();
}

}  // namespace smc

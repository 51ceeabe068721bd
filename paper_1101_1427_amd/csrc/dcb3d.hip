// Double checkerboard sweeps with multi-hit updates of 3D Ising and +-J EA
// lattices (the tiled update of Sec. 3.2 and Sec. 3.4 carried over to three
// dimensions).  The lattice is cut into 16 x 16 x 16 tiles of tile colour
// (bx + by + bz) & 1; a sweep is two launches, one per tile colour.  A
// workgroup stages its tile, the halo rows around it and the x neighbours
// beyond its row ends (and the bonds, for EA) in LDS, gives the tile k hits
// (colour-0 sites, x + y + z even, then colour-1 sites, the halo held
// fixed) and writes the tile back in place.  A lattice of one tile refreshes
// its wrapped halo after every half-hit instead.
//
// Random numbers: hit j of sweep t draws as plain sweep t*k + j.  A thread
// owns one 16-site row segment of the tile (x0 .. x0 + 15 at fixed y, z) and
// updates its eight colour-c sites four to a word (segment3d.hpp), from the
// Philox block (h0 / 8, t*k + j, r, 2*HEAD + c) of their in-colour indices
// h0 .. h0 + 7.
#include "internal.hpp"
#include "segment3d.hpp"

namespace smc {
namespace {

using namespace seg3d;

constexpr int kT3 = 16;                 // tile edge
constexpr int kW3 = kT3 + 2;            // rows per direction with the halo
constexpr int kThreads3 = kT3 * kT3;    // one row segment per thread

struct Dcb3dArgs {
    int8_t *spins;         // replica r at r * N (updated in place)
    const int8_t *coup;    // EA couplings [sample][3][N], or nullptr
    int rep_per_sample;
    const ThrRow *thr;     // per replica (a high half of 0x10000, beta = 0, is exact too)
    int64_t *dE_slots;     // [n_rep][2 * tiles_per_colour], or nullptr
    Key key;
    uint32_t t;
    int k, L, B;
    int tile_colour, rev, tiles_per_colour;
};

__device__ __forceinline__ uint32_t bit_of(int8_t v) { return ((uint32_t)(uint8_t)v >> 1) & 1u; }

template <bool EA>
__global__ __launch_bounds__(kThreads3) void k_dcb3d(Dcb3dArgs a) {
    // rows R[w][v] (w, v = 0 .. 17 with the halo; the tile's 16 x sites),
    // x neighbours beyond the row ends of the tile's rows, and for EA the
    // bonds: +x of the tile's rows and the bond entering each row from x0 - 1,
    // +y of rows v = 0 .. 16 (v = 0: the bonds into the tile from y0 - 1), +z
    // of rows w = 0 .. 16
    __shared__ uint4 R[kW3 * kW3];
    __shared__ uint8_t XL[kThreads3], XR[kThreads3];
    __shared__ uint4 JX[EA ? kThreads3 : 1], JY[EA ? kT3 * (kT3 + 1) : 1], JZ[EA ? (kT3 + 1) * kT3 : 1];
    __shared__ uint8_t JXL[EA ? kThreads3 : 1];
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
    const int64_t LL = L, N = LL * LL * LL;
    int8_t *S = a.spins + (int64_t)r * N;
    const int8_t *J = EA ? a.coup + (int64_t)(r / a.rep_per_sample) * 3 * N : nullptr;
    const int xl = (x0 + L - 1) % L, xr = (x0 + kT3) % L;
    auto row_index = [&](int y, int z) -> int64_t { return ((int64_t)z * L + y) * LL; };
    // staged row (w, v) = lattice row (y0 + v - 1, z0 + w - 1) mod L
    for (int q = threadIdx.x; q < kW3 * kW3; q += kThreads3) {
        const int v = q % kW3, w = q / kW3;
        const int y = (y0 + v - 1 + L) % L, z = (z0 + w - 1 + L) % L;
        R[q] = *(const uint4 *)(S + row_index(y, z) + x0);
    }
    {
        const int v = (int)threadIdx.x % kT3, w = (int)threadIdx.x / kT3;
        const int64_t ri = row_index(y0 + v, z0 + w);
        XL[threadIdx.x] = (uint8_t)S[ri + xl];
        XR[threadIdx.x] = (uint8_t)S[ri + xr];
        if constexpr (EA) {
            JX[threadIdx.x] = *(const uint4 *)(J + ri + x0);
            JXL[threadIdx.x] = (uint8_t)J[ri + xl];
        }
    }
    if constexpr (EA) {
        for (int q = threadIdx.x; q < kT3 * (kT3 + 1); q += kThreads3) {
            // JY[w][v], v = 0 .. 16: bonds +y of row (y0 + v - 1, z0 + w)
            const int v = q % (kT3 + 1), w = q / (kT3 + 1);
            JY[q] = *(const uint4 *)(J + N + row_index((y0 + v - 1 + L) % L, z0 + w) + x0);
            // JZ[w][v], w = 0 .. 16: bonds +z of row (y0 + v, z0 + w - 1)
            const int v2 = q % kT3, w2 = q / kT3;
            JZ[q] = *(const uint4 *)(J + 2 * N + row_index(y0 + v2, (z0 + w2 - 1 + L) % L) + x0);
        }
    }
    const ThrRow th = a.thr[r];
    __syncthreads();

    const int v = (int)threadIdx.x % kT3, w = (int)threadIdx.x / kT3;  // the thread's row (y0 + v, z0 + w)
    const int y = y0 + v, z = z0 + w;
    const int q = (w + 1) * kW3 + (v + 1);
    const uint32_t h0 = (uint32_t)((row_index(y, z) + x0) >> 1);
    long long dE = 0;
    for (int j = 0; j < a.k; ++j) {
        const uint32_t tj = a.t * (uint32_t)a.k + (uint32_t)j;
        for (int ci = 0; ci < 2; ++ci) {
            const int c = a.rev ? 1 - ci : ci;
            const int A = ((y + z) & 1) ^ c;  // x0 is even
            const uint4 own = R[q];
            uint4 jx = make_uint4(0u, 0u, 0u, 0u), jy = jx, jym = jx, jz = jx, jzm = jx;
            uint32_t jeb = 0u;
            if constexpr (EA) {
                jx = JX[threadIdx.x];
                jeb = bit_of((int8_t)JXL[threadIdx.x]);
                jy = JY[w * (kT3 + 1) + v + 1];
                jym = JY[w * (kT3 + 1) + v];
                jz = JZ[(w + 1) * kT3 + v];
                jzm = JZ[w * kT3 + v];
            }
            Bonds3 bd{};
            if constexpr (EA) bd = bonds_from_bytes(jx, jeb, jy, jym, jz, jzm, A);
            const RowOut o = segment_update<EA>(own, R[q - 1], R[q + 1], R[q - kW3], R[q + kW3],
                                                A ? XR[threadIdx.x] : XL[threadIdx.x], A, bd, th,
                                                h0, (uint32_t)c, tj, (uint32_t)r, a.key, 0x00010001u);
            if (o.F0 | o.F1) R[q] = apply_flips(own, o, A);
            dE += flip_energy(o);
            __syncthreads();
            if (a.B == 1) {
                // a single tile: the halo copies take the values just updated
                for (int p = threadIdx.x; p < kW3 * kW3; p += kThreads3) {
                    const int pv = p % kW3, pw = p / kW3;
                    const bool hv = pv == 0 || pv == kW3 - 1, hw = pw == 0 || pw == kW3 - 1;
                    if (hv == hw) continue;  // interior rows, and the corner rows no update reads
                    const int sv = (pv + kT3 - 1) % kT3 + 1, sw = (pw + kT3 - 1) % kT3 + 1;
                    R[p] = R[sw * kW3 + sv];
                }
                const uint4 me = R[q];
                XL[threadIdx.x] = (uint8_t)(me.w >> 24);  // x = 15 wraps to x - 1 of x = 0
                XR[threadIdx.x] = (uint8_t)me.x;          // x = 0 wraps to x + 1 of x = 15
                __syncthreads();
            }
        }
    }
    // the tile back, in place
    *(uint4 *)(S + row_index(y, z) + x0) = R[q];
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
    if (coup)
        SMC_LAUNCH(k_dcb3d<true>, dim3(blocks), dim3(kThreads3), 0, s, a);
    else
        SMC_LAUNCH(k_dcb3d<false>, dim3(blocks), dim3(kThreads3), 0, s, a);
    return hipGetLastError();
}

}  // namespace smc

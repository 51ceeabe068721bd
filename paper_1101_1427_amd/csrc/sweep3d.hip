// Checkerboard half-sweeps of uniform 3D Ising and +-J EA batches (Eq. 2 on
// the simple cubic lattice, the 3D update of Sec. 3) with an edge L that is
// a multiple of 16, in place on the caller's row-major int8 spins.
//
// One thread owns one 16-site row segment (x0 .. x0 + 15 of row (y, z)).  It
// loads the segment, the segments of rows y +- 1 and z +- 1 and the one
// site beyond the segment's end that its x neighbours need, splits even-x
// and odd-x sites with byte permutes (the colour-c sites of row (y, z) are
// the even-x ones iff (y + z) & 1 == c), counts the unsatisfied bonds of its
// eight colour-c sites four to a word, and decides them against one Philox
// block: they are the in-colour indices h0 .. h0 + 7 with h0 = i0 / 2 for
// the segment's first site i0, so the block (h0 / 8, t, r, 2*HEAD + c)
// holds their 16-bit heads in order.  The results are those of the per-site
// kernels bit for bit.
//
// Sites of the other colour are stored back unchanged, so a thread that
// reads a segment while its owner writes it sees the same values either way.
#include <stdlib.h>

#include "internal.hpp"
#include "segment3d.hpp"

namespace smc {
namespace {

using namespace seg3d;

constexpr int kThreads = 256;

struct Sweep3dArgs {
    int8_t *spins;          // replica r at r * L^3
    const int8_t *coup;     // EA: [sample][3][L^3] (bond i -> i + mu at mu * L^3 + i), or nullptr
    int rep_per_sample;
    const ThrRow *thr;      // per replica (high halves <= 0xFFFF, checked on the host)
    const uint2 *pbonds;    // EA bit-packed: [sample][L^3 / 16] (pack_bonds3d), or nullptr
    int64_t *dE;            // per replica, or nullptr
    Key key;
    uint32_t t;
    int L, c;
    int blocks_per_rep;
    uint32_t one2;  // 0x00010001 (opaque to the compiler, keeps the packed 16-bit ops)
};

// Z rows per thread: the segments (x0, y, z0 .. z0 + Z - 1), each row's
// z + 1 neighbour becoming the next row, the row itself the next z - 1.
// M: 0 Ising, 1 EA with the int8 bonds, 2 EA with bit-packed bonds.
template <int M, int Z, bool NT>
__global__ __launch_bounds__(kThreads) void k_ising3d_half(Sweep3dArgs a) {
    constexpr bool EA = M != 0;
    __shared__ long long red[kThreads / 64];
    const int L = a.L;
    const int r = (int)blockIdx.x / a.blocks_per_rep;
    const int64_t g = (int64_t)((int)blockIdx.x % a.blocks_per_rep) * kThreads + threadIdx.x;
    const int segs = L >> 4;
    const int64_t LL = L, P = LL * LL, N = P * LL;
    const bool valid = g < N / (16 * Z);
    long long dE = 0;
    if (valid) {
        const int64_t rowq = g / segs;  // zq * L + y
        const int x0 = (int)(g - rowq * segs) << 4;
        const int y = (int)(rowq % L), z0 = (int)(rowq / L) * Z;
        int8_t *S = a.spins + (int64_t)r * N;
        const int8_t *J = M == 1 ? a.coup + (int64_t)(r / a.rep_per_sample) * 3 * N : nullptr;
        const uint2 *PB = M == 2 ? a.pbonds + (int64_t)(r / a.rep_per_sample) * (N >> 4) : nullptr;
        const int64_t dym = y == 0 ? (LL - 1) * LL : -LL, dyp = y == L - 1 ? -(LL - 1) * LL : LL;
        const int64_t xl = x0 == 0 ? L - 1 : x0 - 1, xr = x0 + 16 == L ? 0 : x0 + 16;
        const ThrRow th = a.thr[r];
        int64_t i0 = ((int64_t)z0 * L + y) * LL + x0;
        uint4 rzm = *(const uint4 *)(S + (z0 == 0 ? i0 + (LL - 1) * P : i0 - P));
        uint4 own = *(const uint4 *)(S + i0);
        uint4 jzm = make_uint4(0u, 0u, 0u, 0u), jz = jzm;
        uint2 pzm = make_uint2(0u, 0u), pown = pzm;
        if constexpr (M == 1) {
            jzm = *(const uint4 *)(J + 2 * N + (z0 == 0 ? i0 + (LL - 1) * P : i0 - P));
            jz = *(const uint4 *)(J + 2 * N + i0);
        }
        if constexpr (M == 2) {
            pzm = PB[(z0 == 0 ? i0 + (LL - 1) * P : i0 - P) >> 4];
            pown = PB[i0 >> 4];
        }
#pragma unroll(Z < 4 ? Z : 4)
        for (int j = 0; j < Z; ++j) {
            const int z = z0 + j;
            const int64_t izp = z == L - 1 ? i0 - (LL - 1) * P : i0 + P;
            const uint4 rzp = *(const uint4 *)(S + izp);
            const uint4 rym = *(const uint4 *)(S + i0 + dym);
            const uint4 ryp = *(const uint4 *)(S + i0 + dyp);
            const int A = ((y + z) & 1) ^ a.c;
            const int64_t iex = i0 - x0 + (A ? xr : xl);
            const uint32_t eb = (uint8_t)S[iex];
            uint4 jzn = make_uint4(0u, 0u, 0u, 0u);
            uint2 pnext = make_uint2(0u, 0u);
            Bonds3 bd{};
            if constexpr (M == 1) {
                const uint4 jx = *(const uint4 *)(J + i0);
                const uint32_t jeb = ((uint32_t)(uint8_t)J[i0 - x0 + xl] >> 1) & 1u;
                const uint4 jy = *(const uint4 *)(J + N + i0);
                const uint4 jym = *(const uint4 *)(J + N + i0 + dym);
                if (j + 1 < Z) jzn = *(const uint4 *)(J + 2 * N + izp);
                bd = bonds_from_bytes(jx, jeb, jy, jym, jz, jzm, A);
            }
            if constexpr (M == 2) {
                // the bond entering the row from x0 - 1: the last odd-x bit of
                // the x mask of the segment to the left
                const uint32_t jeb = (PB[(i0 - x0 + xl) >> 4].x >> 15) & 1u;
                const uint2 pym = PB[(i0 + dym) >> 4];
                if (j + 1 < Z) pnext = PB[izp >> 4];
                bd = bonds_from_bits(pown.x & 0xFFFFu, jeb, pown.x >> 16, pym.x >> 16, pown.y, pzm.y, A);
            }
            const RowOut o = segment_update<EA>(own, rym, ryp, rzm, rzp, eb, A, bd, th, (uint32_t)(i0 >> 1),
                                                (uint32_t)a.c, a.t, (uint32_t)r, a.key, a.one2);
            if (o.F0 | o.F1) {
                const uint4 out = apply_flips(own, o, A);
                if constexpr (NT)
                    __builtin_nontemporal_store(v4u{out.x, out.y, out.z, out.w}, (v4u *)(S + i0));
                else
                    *(uint4 *)(S + i0) = out;
            }
            if (a.dE) dE += flip_energy(o);
            // next row: z + 1 is its own row, this row its z - 1 neighbour (only
            // the other colour's bytes are read from it, which did not change)
            rzm = own;
            own = rzp;
            if constexpr (M == 1) {
                jzm = jz;
                jz = jzn;
            }
            if constexpr (M == 2) {
                pzm = pown;
                pown = pnext;
            }
            i0 = izp;
        }
    }
    if (a.dE) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dE += __shfl_xor(dE, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dE;
        __syncthreads();
        if (threadIdx.x == 0) {
            const long long tot = red[0] + red[1] + red[2] + red[3];
            if (tot != 0) atomicAdd((unsigned long long *)&a.dE[r], (unsigned long long)tot);
        }
    }
}

// Bit-packed bonds: per sample and 16-site segment, x = (x mask) | (y mask
// << 16), y = z mask; a mask holds the even-x sites in bits 0..7 and the
// odd-x sites in bits 8..15, bit 1 where J = -1.
__global__ __launch_bounds__(kThreads) void k_pack_bonds3d(const int8_t *coup, uint2 *out, int64_t N, int64_t total) {
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;  // sample * (N / 16) + segment
    if (q >= total) return;
    const int64_t sample = q / (N >> 4), seg = q - sample * (N >> 4);
    const int8_t *J = coup + sample * 3 * N + (seg << 4);
    uint32_t m[3];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        const uint4 w = *(const uint4 *)(J + mu * N);
        const uint2 e = bits2(half_of(w, 0x06040200u)), o = bits2(half_of(w, 0x07050301u));
        m[mu] = gather4(e.x) | (gather4(e.y) << 4) | (gather4(o.x) << 8) | (gather4(o.y) << 12);
    }
    out[q] = make_uint2(m[0] | (m[1] << 16), m[2]);
}

}  // namespace

hipError_t launch_pack_bonds3d(const int8_t *coup, uint2 *out, int L, int n_samples, hipStream_t s) {
    if (L % 16 || n_samples < 1) return hipErrorInvalidValue;
    const int64_t N = (int64_t)L * L * L, total = (int64_t)n_samples * (N >> 4);
    SMC_LAUNCH(k_pack_bonds3d, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, coup,
                       out, N, total);
    return hipGetLastError();
}

bool sweep3d_supported(int L) { return L >= 16 && L % 16 == 0; }

namespace {

bool sweep3d_nt() {
    const char *env = getenv("SPINMC_SWEEP3D_NT");
    return !(env && env[0] == '0');
}

template <int M, int Z>
hipError_t launch_rows(bool nt, unsigned blocks, const Sweep3dArgs &a, hipStream_t s) {
    if (nt)
        SMC_LAUNCH((k_ising3d_half<M, Z, true>), dim3(blocks), dim3(kThreads), 0, s, a);
    else
        SMC_LAUNCH((k_ising3d_half<M, Z, false>), dim3(blocks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <int M>
hipError_t launch_model(int Z, bool nt, unsigned blocks, const Sweep3dArgs &a, hipStream_t s) {
    if (Z == 16) return launch_rows<M, 16>(nt, blocks, a, s);
    if (Z == 8) return launch_rows<M, 8>(nt, blocks, a, s);
    if (Z == 4) return launch_rows<M, 4>(nt, blocks, a, s);
    if (Z == 2) return launch_rows<M, 2>(nt, blocks, a, s);
    return launch_rows<M, 1>(nt, blocks, a, s);
}

}  // namespace

// Rows per thread along z: Z rows fetch Z + 2 row segments of every column
// instead of 3 Z, so a launch reads the lattice (Z + 2) / Z times.  Z = 4
// (the default) runs the Ising sweep at 512^3 and 1024^3 about 20 % faster
// than Z = 1; 8 and 16 fetch less but leave fewer threads and are no
// faster.  SPINMC_SWEEP3D_Z = 1, 2, 4, 8 or 16 sets it, else a value
// smc_autotune measured for the edge, model and replica count; non-temporal
// stores of the updated segments are on unless SPINMC_SWEEP3D_NT = 0.
int sweep3d_rows(int L, bool ea, int n_rep) {
    const char *env = getenv("SPINMC_SWEEP3D_Z");
    if (env && env[0]) {
        const int z = atoi(env);
        if (z == 1 || z == 2 || z == 4 || z == 8 || z == 16) return z;
    }
    Shape t;
    if (tuned_shape(kShapeHalf3d, L, ea ? 1 : 0, n_rep, &t)) {
        const int z = t.v[0];
        if (z == 1 || z == 2 || z == 4 || z == 8 || z == 16) return z;
    }
    return 4;
}

hipError_t launch_ising3d_half(int8_t *spins, const int8_t *coup, const uint2 *pbonds, int rep_per_sample,
                               const ThrRow *thr, int64_t *dE, int n_rep, int L, Key key, uint32_t t, int c,
                               hipStream_t s) {
    if (!sweep3d_supported(L) || rep_per_sample < 1 || n_rep < 1) return hipErrorInvalidValue;
    // a replica's (L / 16)^3 workgroups of one-row threads regroup into whole
    // workgroups of Z-row threads when Z divides (L / 16)^3
    const int B = L / 16;
    int Z = sweep3d_rows(L, coup != nullptr || pbonds != nullptr, n_rep);
    while ((B * B * B) % Z) Z >>= 1;
    const int64_t threads = (int64_t)L * L * L / (16 * Z);  // per replica
    Sweep3dArgs a;
    a.spins = spins;
    a.coup = coup;
    a.pbonds = pbonds;
    a.rep_per_sample = rep_per_sample;
    a.thr = thr;
    a.dE = dE;
    a.key = key;
    a.t = t;
    a.L = L;
    a.c = c;
    a.blocks_per_rep = (int)((threads + kThreads - 1) / kThreads);
    a.one2 = 0x00010001u;
    const int64_t blocks = (int64_t)n_rep * a.blocks_per_rep;
    if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
    if (pbonds) return launch_model<2>(Z, sweep3d_nt(), (unsigned)blocks, a, s);
    if (coup) return launch_model<1>(Z, sweep3d_nt(), (unsigned)blocks, a, s);
    return launch_model<0>(Z, sweep3d_nt(), (unsigned)blocks, a, s);
}

}  // namespace smc

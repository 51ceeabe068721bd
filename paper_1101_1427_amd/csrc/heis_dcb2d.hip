// Double checkerboard sweeps with multi-hit updates (Sec. 3.2, Sec. 3.4) of
// the 2D Heisenberg model (Sec. 4, Eq. 10) in three arithmetic modes, the
// implementations compared in Sec. 4:
//   fast:   float32 spins and arithmetic, hardware sin / cos / exp2 / sqrt
//           (the move of the plain Heisenberg sweep kernels, heis_math.hpp);
//   float:  float32 spins and arithmetic, accurate library functions
//           (sincospif, expf, correctly rounded square root and division);
//   double: float64 spins and arithmetic (sincospi, exp, sqrt).
// The update order is that of the Ising double checkerboard: one launch per
// tile colour; a workgroup stages its T x T tile and a one-site halo in LDS,
// gives the tile k hits (colour-0 sites, then colour-1 sites, the halo held
// fixed) and writes it back in place.  Hit j of sweep t takes the plain
// sweep's draws of sweep t*k + j: the move at in-colour site h uses words 0,
// 1 (proposal) and 2 (acceptance) of (h, t*k + j, r, 2*HEIS + c).  The
// proposal is a uniform re-orientation, or with cap > 0 a uniform point of
// the cap of that size around the current direction.
//
// A thread owns four consecutive sites of a tile row in registers for all k
// hits; per half-hit it updates the two of the current colour, reading their
// vertical neighbours and one horizontal neighbour from LDS (the others are
// its own sites), then writes them to LDS; one barrier per half-hit.
#include <type_traits>

#include "heis_math.hpp"
#include "internal.hpp"

namespace smc {
namespace {

template <int MODE>
struct HeisArith;

template <>
struct HeisArith<SMC_HEIS_FAST> {
    using R = float;
    __device__ static R uni(uint32_t w) { return unit23f(w); }
    __device__ static void propose(R u0, R u1, R &x, R &y, R &z) {
        const float3 p = heis_proposal(u0, u1);
        x = p.x;
        y = p.y;
        z = p.z;
    }
    __device__ static R boltzmann(R beta, R dE) { return heis_boltzmann(beta, dE); }
    __device__ static R sq(R x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static R dv(R a, R b) { return __fdividef(a, b); }
    __device__ static void sincos_rev(R u, R &sn, R &cs) {
        sn = __builtin_amdgcn_sinf(u);
        cs = __builtin_amdgcn_cosf(u);
    }
    __device__ static void unit(R &x, R &y, R &z) {
        const float3 u = heis_unit(x, y, z);
        x = u.x;
        y = u.y;
        z = u.z;
    }
};

template <>
struct HeisArith<SMC_HEIS_FLOAT> {
    using R = float;
    __device__ static R uni(uint32_t w) { return unit23f(w); }
    __device__ static void propose(R u0, R u1, R &x, R &y, R &z) {
        const float zz = 2.0f * u0 - 1.0f;
        const float rho = __fsqrt_rn(1.0f - zz * zz);
        float sn, cs;
        sincospif(2.0f * u1, &sn, &cs);  // sin and cos of 2 pi u1 (the argument 2 u1 is exact)
        x = rho * cs;
        y = rho * sn;
        z = zz;
    }
    __device__ static R boltzmann(R beta, R dE) { return expf(-beta * dE); }
    __device__ static R sq(R x) { return __fsqrt_rn(x); }
    __device__ static R dv(R a, R b) { return __fdiv_rn(a, b); }
    __device__ static void sincos_rev(R u, R &sn, R &cs) { sincospif(2.0f * u, &sn, &cs); }
    __device__ static void unit(R &x, R &y, R &z) {
        const float n = __fsqrt_rn(x * x + y * y + z * z);
        x = __fdiv_rn(x, n);
        y = __fdiv_rn(y, n);
        z = __fdiv_rn(z, n);
    }
};

template <>
struct HeisArith<SMC_HEIS_DOUBLE> {
    using R = double;
    __device__ static R uni(uint32_t w) { return (double)unit23f(w); }  // exact
    __device__ static void propose(R u0, R u1, R &x, R &y, R &z) {
        const double zz = 2.0 * u0 - 1.0;
        const double rho = sqrt(1.0 - zz * zz);
        double sn, cs;
        sincospi(2.0 * u1, &sn, &cs);
        x = rho * cs;
        y = rho * sn;
        z = zz;
    }
    __device__ static R boltzmann(R beta, R dE) { return exp(-beta * dE); }
    __device__ static R sq(R x) { return sqrt(x); }
    __device__ static R dv(R a, R b) { return a / b; }
    __device__ static void sincos_rev(R u, R &sn, R &cs) { sincospi(2.0 * u, &sn, &cs); }
    __device__ static void unit(R &x, R &y, R &z) {
        const double n = sqrt(x * x + y * y + z * z);
        x /= n;
        y /= n;
        z /= n;
    }
};

// Small-step proposal: s' uniform on the spherical cap {s' : 1 - a.s' <= cap}
// around a = s / |s| (a symmetric proposal density).  w = cap u0 gives the
// cosine 1 - w of the angle and the radius sqrt(w (2 - w)); the azimuth
// 2 pi u1 is taken in the frame (e1, e2): e1 perpendicular to a in the x-y
// plane when |a_x| > |a_z|, else in the y-z plane, and e2 = a x e1.
template <class A, typename R>
__device__ __forceinline__ void cap_proposal(R x, R y, R z, R cap, R u0, R u1, R &px, R &py, R &pz) {
    const R n = A::sq(x * x + y * y + z * z);
    const R ax = A::dv(x, n), ay = A::dv(y, n), az = A::dv(z, n);
    R e1x, e1y, e1z;
    if (fabs(ax) > fabs(az)) {
        const R m = A::sq(ax * ax + ay * ay);
        e1x = A::dv(-ay, m);
        e1y = A::dv(ax, m);
        e1z = R(0);
    } else {
        const R m = A::sq(ay * ay + az * az);
        e1x = R(0);
        e1y = A::dv(-az, m);
        e1z = A::dv(ay, m);
    }
    const R e2x = ay * e1z - az * e1y, e2y = az * e1x - ax * e1z, e2z = ax * e1y - ay * e1x;
    const R w = cap * u0;
    const R zc = R(1) - w, rc = A::sq(w * (R(2) - w));
    R sn, cs;
    A::sincos_rev(u1, sn, cs);
    px = zc * ax + rc * (cs * e1x + sn * e2x);
    py = zc * ay + rc * (cs * e1y + sn * e2y);
    pz = zc * az + rc * (cs * e1z + sn * e2z);
}

// One LDS cell: a spin and padding to 16 (float) or 32 (double) bytes.
template <typename R>
struct alignas(4 * sizeof(R)) Cell {
    R x, y, z, pad;
};

template <int T, int SPT>
struct HeisGeom {
    static constexpr int QPR = T / SPT;              // threads per tile row (SPT sites each)
    static constexpr int THREADS = T * T / SPT;
    static constexpr bool UNIFORM = THREADS >= 128;  // every wave holds rows of one parity
    static constexpr int W = T + 2;                  // staged square: tile and halo
};

struct HeisDcbArgs {
    void *spins;         // float or double [n_rep][N][3], updated in place
    const void *beta;    // float or double [n_rep]
    double cap;          // small-step cap (> 0 in the CAP kernels)
    int64_t *acc_slots;  // [n_rep][2 * tiles_per_colour] or nullptr
    Key key;
    uint32_t t;          // sweep index
    int k, L, B;
    int tile_colour, rev, tiles_per_colour;
};

template <int T, int SPT, int MODE, bool CAP>
__global__ __launch_bounds__((HeisGeom<T, SPT>::THREADS)) void k_heis_dcb2d(HeisDcbArgs a) {
    using A = HeisArith<MODE>;
    using R = typename A::R;
    using Gm = HeisGeom<T, SPT>;
    constexpr int QPR = Gm::QPR, W = Gm::W;
    __shared__ Cell<R> cell[W * W];
    __shared__ long long red[(Gm::THREADS + 63) / 64];

    const int lt = (int)threadIdx.x;
    int v, q;
    if constexpr (Gm::UNIFORM) {
        constexpr int RPW = 64 / QPR;  // rows per wave
        const int w = lt >> 6, lane = lt & 63;
        v = 2 * ((w >> 1) * RPW + lane / QPR) + (w & 1);
        q = lane % QPR;
    } else {
        v = lt / QPR;
        q = lt % QPR;
    }
    const int r = (int)blockIdx.x / a.tiles_per_colour;
    const int ti = (int)blockIdx.x % a.tiles_per_colour;
    int bx, by;
    if (a.B == 1) {
        bx = by = 0;
    } else {
        const int half = a.B / 2;
        by = ti / half;
        bx = 2 * (ti % half) + ((by + a.tile_colour) & 1);
    }
    const int L = a.L, x0 = bx * T, y0 = by * T, y = y0 + v, xq = x0 + SPT * q;
    const int64_t N = (int64_t)L * L;
    R *S = (R *)a.spins + (int64_t)r * N * 3;
    const R beta = ((const R *)a.beta)[r];
    const R cap = (R)a.cap;

    // own sites: columns xq .. xq + SPT - 1 of row y
    R sx[SPT], sy[SPT], sz[SPT];
    {
        const R *p = S + ((int64_t)y * L + xq) * 3;
#pragma unroll
        for (int m = 0; m < SPT; ++m) {
            sx[m] = p[3 * m];
            sy[m] = p[3 * m + 1];
            sz[m] = p[3 * m + 2];
            cell[(v + 1) * W + SPT * q + m + 1] = Cell<R>{sx[m], sy[m], sz[m], R(0)};
        }
    }
    if (a.B > 1) {
        auto stage = [&](int yy, int xx, int c) {
            const R *p = S + ((int64_t)yy * L + xx) * 3;
            cell[c] = Cell<R>{p[0], p[1], p[2], R(0)};
        };
        if (v == 0) {
            const int yy = y0 == 0 ? L - 1 : y0 - 1;
#pragma unroll
            for (int m = 0; m < SPT; ++m) stage(yy, xq + m, SPT * q + m + 1);
        }
        if (v == T - 1) {
            const int yy = y0 + T == L ? 0 : y0 + T;
#pragma unroll
            for (int m = 0; m < SPT; ++m) stage(yy, xq + m, (T + 1) * W + SPT * q + m + 1);
        }
        if (q == 0) stage(y, x0 == 0 ? L - 1 : x0 - 1, (v + 1) * W);
        if (q == QPR - 1) stage(y, x0 + T == L ? 0 : x0 + T, (v + 1) * W + T + 1);
    }
    // LDS rows of y - 1 and y + 1, columns of x - 1 for the first site and
    // x + 1 for the last (a single tile wraps onto itself)
    const bool one = a.B == 1;
    const int rowU = (v == 0 ? (one ? T : 0) : v) * W;
    const int rowD = (v == T - 1 ? (one ? 1 : T + 1) : v + 2) * W;
    const int rowO = (v + 1) * W;
    const int colL = q == 0 && one ? T : SPT * q;                // LDS column of x - 1 of site 0
    const int colR = q == QPR - 1 && one ? 1 : SPT * q + SPT + 1;  // LDS column of x + 1 of site SPT - 1
    const uint32_t hrow = (uint32_t)(((int64_t)y * L + xq) >> 1);  // in-colour index of the first own site pair
    __syncthreads();

    int n_acc = 0;
    // The move at own site m (of colour C) with neighbours right, left, down, up.
    auto move = [&](int m, int C, const Cell<R> &rt, const Cell<R> &lf, const Cell<R> &dn, const Cell<R> &up,
                    uint32_t tj) __attribute__((always_inline)) {
        R hx = rt.x, hy = rt.y, hz = rt.z;
        hx += lf.x;
        hy += lf.y;
        hz += lf.z;
        hx += dn.x;
        hy += dn.y;
        hz += dn.z;
        hx += up.x;
        hy += up.y;
        hz += up.z;
        const uint32_t h = hrow + (uint32_t)(m >> 1);
        const uint4 w = philox4x32_10(make_uint4(h, tj, (uint32_t)r, 2 * kTagHeis + (uint32_t)C), a.key);
        R px, py, pz;
        if constexpr (CAP)
            cap_proposal<A, R>(sx[m], sy[m], sz[m], cap, A::uni(w.x), A::uni(w.y), px, py, pz);
        else
            A::propose(A::uni(w.x), A::uni(w.y), px, py, pz);
        const R dE = -((px - sx[m]) * hx + (py - sy[m]) * hy + (pz - sz[m]) * hz);
        if (dE <= R(0) || A::uni(w.z) < A::boltzmann(beta, dE)) {
            sx[m] = px;
            sy[m] = py;
            sz[m] = pz;
            ++n_acc;
        }
    };
    auto own = [&](int m) { return Cell<R>{sx[m], sy[m], sz[m], R(0)}; };
    // Half-hit of colour C; P = 1 when the row's colour-C sites are the odd
    // columns.  The own sites of colour C are P, P + 2, ..; their horizontal
    // neighbours are own sites of the other colour except at the two ends.
    auto half = [&](auto cc, auto pp, uint32_t tj) __attribute__((always_inline)) {
        constexpr int C = decltype(cc)::value, P = decltype(pp)::value;
        constexpr int K = SPT / 2;
        Cell<R> up[K], dn[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            up[i] = cell[rowU + SPT * q + P + 2 * i + 1];
            dn[i] = cell[rowD + SPT * q + P + 2 * i + 1];
        }
        const Cell<R> edge = cell[rowO + (P == 0 ? colL : colR)];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int m = P + 2 * i;
            const Cell<R> lf = m == 0 ? edge : own(m == 0 ? 0 : m - 1);
            const Cell<R> rt = m == SPT - 1 ? edge : own(m == SPT - 1 ? 0 : m + 1);
            move(m, C, rt, lf, dn[i], up[i], tj);
        }
#pragma unroll
        for (int i = 0; i < K; ++i) cell[rowO + SPT * q + P + 2 * i + 1] = own(P + 2 * i);
        __syncthreads();
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    auto half_c = [&](auto cc, uint32_t tj) __attribute__((always_inline)) {
        constexpr int C = decltype(cc)::value;
        // (y + C) odd: the colour-C sites of the row sit at odd columns (x0 even)
        if (((v + C) & 1) != 0)
            half(cc, I1{}, tj);
        else
            half(cc, I0{}, tj);
    };
    for (int j = 0; j < a.k; ++j) {
        const uint32_t tj = a.t * (uint32_t)a.k + (uint32_t)j;
        if (a.rev) {
            half_c(I1{}, tj);
            half_c(I0{}, tj);
        } else {
            half_c(I0{}, tj);
            half_c(I1{}, tj);
        }
    }
    {
        R *p = S + ((int64_t)y * L + xq) * 3;
#pragma unroll
        for (int m = 0; m < SPT; ++m) {
            p[3 * m] = sx[m];
            p[3 * m + 1] = sy[m];
            p[3 * m + 2] = sz[m];
        }
    }
    if (a.acc_slots) {
        long long tot = n_acc;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
        if ((lt & 63) == 0) red[lt >> 6] = tot;
        __syncthreads();
        if (lt == 0) {
            long long sum = 0;
            for (int w = 0; w < (Gm::THREADS + 63) / 64; ++w) sum += red[w];
            a.acc_slots[(int64_t)r * 2 * a.tiles_per_colour + a.tile_colour * a.tiles_per_colour + ti] += sum;
        }
    }
}

// s / |s| for every spin of the batch, in the mode's arithmetic.
template <int MODE>
__global__ __launch_bounds__(256) void k_heis_dcb_renorm(void *spins, int64_t n_spins) {
    using A = HeisArith<MODE>;
    using R = typename A::R;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_spins) return;
    R *s = (R *)spins + 3 * i;
    R x = s[0], y = s[1], z = s[2];
    A::unit(x, y, z);
    s[0] = x;
    s[1] = y;
    s[2] = z;
}

template <int T, int SPT, int MODE>
hipError_t launch_t(const HeisDcbArgs &a, int n_rep, hipStream_t s) {
    const unsigned blocks = (unsigned)(n_rep * a.tiles_per_colour);
    constexpr unsigned threads = HeisGeom<T, SPT>::THREADS;
    if (a.cap > 0.0)
        SMC_LAUNCH((k_heis_dcb2d<T, SPT, MODE, true>), dim3(blocks), dim3(threads), 0, s, a);
    else
        SMC_LAUNCH((k_heis_dcb2d<T, SPT, MODE, false>), dim3(blocks), dim3(threads), 0, s, a);
    return hipGetLastError();
}

// Four sites per thread (eight were measured: 154 VGPRs, 3 % faster for one
// case and up to 1.8x slower for the others).
constexpr int kSpt = 4;

template <int MODE>
hipError_t launch_mode(const HeisDcbArgs &a, int T, int n_rep, hipStream_t s) {
    switch (T) {
        case 16: return launch_t<16, kSpt, MODE>(a, n_rep, s);
        case 32: return launch_t<32, kSpt, MODE>(a, n_rep, s);
        case 64:
            if constexpr (MODE != SMC_HEIS_DOUBLE) return launch_t<64, kSpt, MODE>(a, n_rep, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool heis_dcb2d_supported(int L, int T, int precision) {
    if (!(T == 16 || T == 32 || (T == 64 && precision != SMC_HEIS_DOUBLE))) return false;
    if (L % T) return false;
    const int B = L / T;
    return B == 1 || B % 2 == 0;
}

hipError_t launch_heis_dcb2d(void *spins, const void *beta, int64_t *acc_slots, int n_rep, int L, int T, int k,
                             int precision, double cap, Key key, uint32_t t, int tile_colour, bool rev,
                             hipStream_t s) {
    if (!heis_dcb2d_supported(L, T, precision) || k < 1) return hipErrorInvalidValue;
    const int B = L / T;
    if (B == 1 && tile_colour == 1) return hipSuccess;  // one tile, of tile colour 0
    HeisDcbArgs a;
    a.spins = spins;
    a.beta = beta;
    a.cap = cap;
    a.acc_slots = acc_slots;
    a.key = key;
    a.t = t;
    a.k = k;
    a.L = L;
    a.B = B;
    a.tile_colour = tile_colour;
    a.rev = rev ? 1 : 0;
    a.tiles_per_colour = dcb2d_tiles_per_colour(L, T);
    switch (precision) {
        case SMC_HEIS_FAST: return launch_mode<SMC_HEIS_FAST>(a, T, n_rep, s);
        case SMC_HEIS_FLOAT: return launch_mode<SMC_HEIS_FLOAT>(a, T, n_rep, s);
        case SMC_HEIS_DOUBLE: return launch_mode<SMC_HEIS_DOUBLE>(a, T, n_rep, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_heis_dcb_renorm(void *spins, int64_t n_spins, int precision, hipStream_t s) {
    if (n_spins <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n_spins + 255) / 256));
    switch (precision) {
        case SMC_HEIS_FAST: SMC_LAUNCH(k_heis_dcb_renorm<SMC_HEIS_FAST>, grid, dim3(256), 0, s, spins, n_spins); break;
        case SMC_HEIS_FLOAT: SMC_LAUNCH(k_heis_dcb_renorm<SMC_HEIS_FLOAT>, grid, dim3(256), 0, s, spins, n_spins); break;
        case SMC_HEIS_DOUBLE: SMC_LAUNCH(k_heis_dcb_renorm<SMC_HEIS_DOUBLE>, grid, dim3(256), 0, s, spins, n_spins); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace smc

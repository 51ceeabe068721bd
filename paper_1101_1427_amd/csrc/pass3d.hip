// One-pass checkerboard sweeps of uniform 3D Ising and +-J EA batches (Eq. 2
// on the simple cubic lattice; colour 0, then colour 1, Sec. 3.2) with an
// edge L that is a multiple of 16, reading each spin once and writing it
// once per sweep (plus halos).
//
// A workgroup owns a strip of TY rows (y in [Y0, Y0 + TY), all x) over a
// segment of D planes in z and streams down the planes.  At step z it
// updates colour 0 of plane z, then colour 1 of plane z - 1, whose six
// neighbours are then final, and writes plane z - 1 of the strip to the
// destination buffer (reads come from the source buffer, so strips never
// see each other's new values).  Colour 0 is also computed on the rows
// Y0 - 1 and Y0 + TY and on the planes Z0 - 1 and Z0 + D around the strip
// (recomputed identically by the neighbouring strips: every draw is keyed by
// the site), which needs the rows Y0 - 2 and Y0 + TY + 1 and the planes
// Z0 - 2 and Z0 + D + 1 as input.
//
// Layout on chip: a 16-site row segment is held "split", its eight even-x
// bytes (x0, x0 + 2, ..., x0 + 14) in words 0-1 and its eight odd-x bytes in
// words 2-3, so the eight sites of one colour, and their y and z neighbours,
// are two whole words; the caller's row-major bytes are split once when a
// plane arrives and joined once when it leaves.  A thread owns SEGS segments
// of one staged row (segments i TR + tl for TR threads per row, so that each
// load, store and LDS access of a wavefront covers consecutive segments) and
// keeps its column of segments along z in registers (planes z - 2 .. z + 3,
// the last two in flight from global memory), so z neighbours never leave
// the thread; the y neighbours and the sites beyond a segment's ends come
// from an LDS ring of three staged planes (TY + 4 rows, each row the even-x
// halves of its segments, then the odd-x halves, so that the halves of one
// parity of consecutive segments are consecutive words).
// One barrier per plane: plane z + 1 is staged into the slot of plane z - 2,
// colour 0 of plane z writes its half back to the slot of plane z, colour 1
// of plane z - 1 only reads.  EA bonds (bit-packed, 3 bits per site) travel
// with the spins: the row's masks in the register column, the x and y masks
// of every staged row in a second LDS ring.
//
// Threads are grouped by the parity of their row, so the colour's parity in
// x (which half of a split segment is updated) is uniform over a wavefront
// and fixed at compile time in each of two copies of the plane loop.
// Global loads and stores are buffer instructions issued by every lane at
// every step, with an offset past the end of the lattice where nothing is to
// be read or written (such loads return zeros, such stores are dropped), so
// the compiler's count of loads in flight stays exact and the wait before a
// plane is staged covers only that plane.
//
// Per site and sweep the update is the one of the half-sweep kernels
// (unsatisfied bonds counted four sites to a word, one Philox block per
// eight sites, packed 16-bit threshold comparisons, exact tail decisions
// on ties), so the results are theirs bit for bit.
#include <stdlib.h>

#include <type_traits>

#include "internal.hpp"
#include "segment3d.hpp"

namespace smc {
namespace {

using namespace seg3d;

constexpr int kRing = 3;                // staged planes
constexpr uint32_t kOob = 0x40000000u;  // a byte offset past every lattice (L^3 <= 2^30)

struct Pass3dArgs {
    const int8_t *src;     // replica r at r * L^3 (read)
    int8_t *dst;           // replica r at r * L^3 (written)
    const uint2 *pbonds;   // EA: bit-packed bonds [sample][L^3 / 16] (pack_bonds3d), else nullptr
    int rep_per_sample;
    const ThrRow *thr;     // per replica (high halves <= 0xFFFF)
    unsigned long long *dE;  // per replica, or nullptr
    Key key;
    uint32_t t;
    int L, D;              // edge; planes per z segment
    int strips, zsegs;     // per replica
    int np;                // threads per row-parity class (a multiple of 64)
    uint32_t one2;         // 0x00010001, opaque to the compiler
};

__device__ __forceinline__ int wrapi(int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); }

__device__ __forceinline__ uint4 ld16(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    const v4u v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 ld8(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    const v2u v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    return make_uint2(v.x, v.y);
}
// Non-temporal 16-byte store (aux bit 1).
__device__ __forceinline__ void st16(__amdgpu_buffer_rsrc_t rs, uint32_t off, const uint4 &w) {
    __builtin_amdgcn_raw_buffer_store_b128(v4u{w.x, w.y, w.z, w.w}, rs, off, 0, 2);
}

// Row-major segment bytes <-> split form.
__device__ __forceinline__ uint4 to_split(const uint4 &w) {
    return make_uint4(perm(w.y, w.x, 0x06040200u), perm(w.w, w.z, 0x06040200u), perm(w.y, w.x, 0x07050301u),
                      perm(w.w, w.z, 0x07050301u));
}
__device__ __forceinline__ uint4 from_split(const uint4 &q) {
    return make_uint4(perm(q.z, q.x, 0x05010400u), perm(q.z, q.x, 0x07030602u), perm(q.w, q.y, 0x05010400u),
                      perm(q.w, q.y, 0x07030602u));
}
template <int H>
__device__ __forceinline__ uint2 half(const uint4 &q) {
    return H ? make_uint2(q.z, q.w) : make_uint2(q.x, q.y);
}
template <int H>
__device__ __forceinline__ void set_half(uint4 &q, uint2 h) {
    if constexpr (H) {
        q.z = h.x;
        q.w = h.y;
    } else {
        q.x = h.x;
        q.y = h.y;
    }
}

// The eight sites of parity A of a split segment q, colour c: neighbours in
// the other half (x +- 1, with eb the raw byte of the site beyond the
// segment: x0 + 16 for odd-x sites, x0 - 1 for even-x), in rows y -+ 1 (ym,
// yp) and planes z -+ 1 (zm, zp), all as the parity-A halves.  Returns the
// new own half; adds the energy change to dE where count is set.
template <bool EA, int A, bool DE>
__device__ __forceinline__ uint2 update_half(const uint4 &q, uint2 ym, uint2 yp, uint2 zm, uint2 zp, uint32_t eb,
                                             const Bonds3 &bd, const Lut3 &K, const ThrRow &th, uint32_t h0,
                                             uint32_t c, uint32_t r, const Pass3dArgs &a, bool count, long long &dE) {
    const uint2 Sa = half<A>(q), Sb = half<1 - A>(q);
    uint2 sh;
    if constexpr (A) {
        sh.x = alignbyte(Sb.y, Sb.x, 1);
        sh.y = (Sb.y >> 8) | (eb << 24);
    } else {
        sh.x = (Sb.x << 8) | eb;
        sh.y = alignbyte(Sb.y, Sb.x, 3);
    }
    RowOut o;
    count_unsat<EA>(Sa, Sb, sh, ym, yp, zm, zp, bd, o.n0, o.n1);
    const uint4 w = philox4x32_10_wide(make_uint4(h0 >> 3, a.t, r, 2 * kTagHead + c), a.key);
    uint32_t eq = 0xFFFFFFFFu;
    o.F0 = decide4(o.n0, w.x, w.y, K, a.one2, eq);
    o.F1 = decide4(o.n1, w.z, w.w, K, a.one2, eq);
    if (__builtin_expect(__any(has_tie(eq)), 0)) exact_decisions(o, w, th, K, h0, c, a.t, r, a.key, has_tie(eq));
    if constexpr (DE) {
        if (count) dE += flip_energy(o);
    }
    return make_uint2(Sa.x ^ bytes_fe(o.F0), Sa.y ^ bytes_fe(o.F1));
}

// Largest workgroup of a launch shape (edges up to 1024).
constexpr int pass3d_max_threads(int ty, int segs) { return ty == 8 ? (segs == 1 ? 768 : 384) : 640; }

// TY rows per strip, SEGS segments per thread; DE: energy changes wanted.
template <int M, int TY, int SEGS, bool DE>
__global__ __launch_bounds__(pass3d_max_threads(TY, SEGS)) void k_ising3d_pass(Pass3dArgs a) {
    constexpr bool EA = M != 0;
    constexpr int kRows = TY + 4, kHalf = kRows / 2;
    // spins [kRing][kRows][L] (split segments), EA: x/y masks [kRing][kRows][L / 16]
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ long long red[16];
    const int L = a.L, nseg = L >> 4;
    const int TR = nseg / SEGS;  // threads per staged row
    // row-parity classes: threads [0, np) take the even staged rows, [np, 2 np) the odd ones
    const int tid = (int)threadIdx.x;
    const int par = tid >= a.np ? 1 : 0, idx = tid - par * a.np;
    const int rc = idx / TR, tl = idx % TR;
    const bool valid = rc < kHalf;  // lanes past the last row of the class only take part in the barriers
    const int ry = valid ? 2 * rc + par : par;
    // Workgroups go to the XCDs round-robin; consecutive logical blocks
    // (neighbouring strips of one z segment) run on one XCD, which then reads
    // the halo rows they share once into its L2.
    const uint32_t nblk = gridDim.x, b = blockIdx.x;
    const int lb = (int)((nblk & 7u) == 0 ? (b & 7u) * (nblk >> 3) + (b >> 3) : b);
    const int per_rep = a.strips * a.zsegs;
    const int r = lb / per_rep, rem = lb % per_rep;
    const int zs = rem / a.strips, st = rem % a.strips;
    const int Y0 = st * TY, Z0 = zs * a.D, Z1 = Z0 + a.D;
    const int y = wrapi(Y0 - 2 + ry, L);
    const uint32_t P = (uint32_t)L * (uint32_t)L, N = P * (uint32_t)L;
    const bool c0_row = valid && ry >= 1 && ry < kRows - 1;  // rows Y0-1 .. Y0+TY: colour 0
    const bool own_row = valid && ry >= 2 && ry < kRows - 2;  // rows Y0 .. Y0+TY-1: colour 1 and stores
    const ThrRow th = a.thr[r];
    const Lut3 K = lut_of(th);
    const __amdgpu_buffer_rsrc_t rs_src =
        __builtin_amdgcn_make_buffer_rsrc((void *)(a.src + (size_t)r * N), 0, (int)N, 0x00020000);
    const __amdgpu_buffer_rsrc_t rs_dst = __builtin_amdgcn_make_buffer_rsrc((void *)(a.dst + (size_t)r * N), 0, (int)N,
                                                                             0x00020000);
    __amdgpu_buffer_rsrc_t rs_b = rs_src;
    if constexpr (EA)
        rs_b = __builtin_amdgcn_make_buffer_rsrc((void *)(a.pbonds + (size_t)(r / a.rep_per_sample) * (N >> 4)), 0,
                                                 (int)(N >> 1), 0x00020000);
    const uint32_t row_off = (uint32_t)y * (uint32_t)L;
    const size_t plane_bytes = (size_t)kRows * (size_t)L;
    uint32_t off_ld[SEGS], off_st[SEGS];  // in-plane byte offsets of the thread's segments (kOob: none)
#pragma unroll
    for (int i = 0; i < SEGS; ++i) {
        const uint32_t o = row_off + 16u * (uint32_t)(i * TR + tl);
        off_ld[i] = valid ? o : kOob;
        off_st[i] = own_row ? o : kOob;
    }
    auto poff = [&](int z) -> uint32_t { return (uint32_t)wrapi(z, L) * P; };
    auto slot = [&](int z) -> int { return (z + 4 * kRing) % kRing; };
    uint8_t *const bring = lds + (size_t)kRing * plane_bytes;  // EA masks
    auto bmask = [&](int s, int row, int seg) -> uint32_t & {
        return ((uint32_t *)bring)[((size_t)s * kRows + row) * nseg + seg];
    };

    // Column registers: six planes in rotation, R[(k + j) % 6] holding plane
    // z - 2 + j at step k of a group of six steps (j = 0 .. 5: planes z-2 ..
    // z+3), raw bytes from the load until the plane is staged, split after.
    // The rotation is by name only (the loop body is unrolled six times), so
    // a plane in flight is never copied before it is used.
    uint4 R[6][SEGS];
    uint2 B[6][SEGS];  // EA: the row's bond masks, same rotation
    auto load_plane = [&](uint4 (&Rp)[SEGS], uint2 (&Bp)[SEGS], uint32_t pz) {
#pragma unroll
        for (int i = 0; i < SEGS; ++i) {
            Rp[i] = ld16(rs_src, pz + off_ld[i]);
            if constexpr (EA) Bp[i] = ld8(rs_b, (pz + off_ld[i]) >> 1);
        }
    };
    // byte offset of a plane's slot (uniform)
    auto soff = [&](int z) -> uint32_t {
        return __builtin_amdgcn_readfirstlane((uint32_t)slot(z) * (uint32_t)plane_bytes);
    };
    uint8_t *const my_row = lds + (size_t)ry * L;  // the thread's row in slot 0
    auto stage = [&](uint4 (&Rp)[SEGS], const uint2 (&Bp)[SEGS], int z) {
        uint8_t *p = my_row + soff(z);
#pragma unroll
        for (int i = 0; i < SEGS; ++i) {
            Rp[i] = to_split(Rp[i]);
            if (valid) {
                const int seg = i * TR + tl;
                *(uint2 *)(p + 8 * seg) = half<0>(Rp[i]);
                *(uint2 *)(p + (L >> 1) + 8 * seg) = half<1>(Rp[i]);
                if constexpr (EA) bmask(slot(z), ry, seg) = Bp[i].x;
            }
        }
    };

    // prologue: planes Z0-2 .. Z0+1 requested (roles z-1 .. z+2 of the first
    // step), Z0-2 split, Z0-1 staged
    load_plane(R[1], B[1], poff(Z0 - 2));
    load_plane(R[2], B[2], poff(Z0 - 1));
    load_plane(R[3], B[3], poff(Z0));
    load_plane(R[4], B[4], poff(Z0 + 1));
#pragma unroll
    for (int i = 0; i < SEGS; ++i) R[1][i] = to_split(R[1][i]);
    stage(R[2], B[2], Z0 - 1);
    __syncthreads();
    long long dE = 0;

    // One segment of plane z, colour c, parity A: its neighbours from the
    // staged plane s and the column registers zm / zp (bonds: own masks bo,
    // z masks of plane z - 1 in bzm).
    auto seg_update = [&](auto ac, const uint4 &q, const uint4 &qzm, const uint4 &qzp, const uint2 &bo, uint32_t bzm,
                          int z, int s, int seg, uint32_t c, bool count) -> uint2 {
        constexpr int A = decltype(ac)::value;
        const uint8_t *S = my_row + soff(z);  // the thread's row of plane z
        const int segn = seg + 1 == nseg ? 0 : seg + 1, segp = seg == 0 ? nseg - 1 : seg - 1;
        const uint8_t *H = S + A * (L >> 1);   // the parity-A halves of the row
        const uint2 ym = *(const uint2 *)(H - L + 8 * seg);
        const uint2 yp = *(const uint2 *)(H + L + 8 * seg);
        // x0 + 16 (even, first byte of the next segment) or x0 - 1 (odd, last
        // byte of the previous segment)
        const uint32_t eb = A ? S[8 * segn] : S[(L >> 1) + 8 * segp + 7];
        Bonds3 bd{};
        if constexpr (EA) {
            // masks: x (bits 0-15) and y (16-31) of the row and of row y - 1,
            // z of the row and of the row in plane z - 1, the bond entering
            // from x0 - 1 (last odd-x bit of the x mask to the left)
            const uint32_t jeb = (bmask(s, ry, segp) >> 15) & 1u;
            bd = bonds_from_bits(bo.x, jeb, bo.x >> 16, bmask(s, ry - 1, seg) >> 16, bo.y, bzm, A);
        }
        const uint32_t h0 = (poff(z) + row_off + 16u * (uint32_t)seg) >> 1;
        return update_half<EA, A, DE>(q, ym, yp, half<A>(qzm), half<A>(qzp), eb, bd, K, th, h0, c, (uint32_t)r, a,
                                      count, dE);
    };

    // step z (k = (z - Z0 + 1) mod 6, A = (y + z) & 1): stage plane z+1,
    // colour 0 of plane z, request plane z+3, colour 1 of plane z-1 and its
    // store, barrier
    auto step = [&](auto kc, auto ac, int z) {
        constexpr int k = decltype(kc)::value;
        uint4(&Pm2)[SEGS] = R[k % 6];
        uint4(&Pm1)[SEGS] = R[(k + 1) % 6];
        uint4(&Pz)[SEGS] = R[(k + 2) % 6];
        uint4(&Pp1)[SEGS] = R[(k + 3) % 6];
        uint4(&Pp3)[SEGS] = R[(k + 5) % 6];
        const uint2(&Bm2)[SEGS] = B[k % 6];
        const uint2(&Bm1)[SEGS] = B[(k + 1) % 6];
        const uint2(&Bz)[SEGS] = B[(k + 2) % 6];
        const uint2(&Bp1)[SEGS] = B[(k + 3) % 6];
        uint2(&Bp3)[SEGS] = B[(k + 5) % 6];
        constexpr int A = decltype(ac)::value;
        // plane z+1 (requested two steps ago) into the slot of plane z-2
        stage(Pp1, Bp1, z + 1);
        // colour 0 of plane z (rows Y0-1 .. Y0+TY), its half back into the slot
        if (c0_row) {
            const int s = slot(z);
            const bool count = own_row && z >= Z0 && z < Z1;
#pragma unroll
            for (int i = 0; i < SEGS; ++i) {
                const int seg = i * TR + tl;
                const uint2 nh = seg_update(ac, Pz[i], Pm1[i], Pp1[i], Bz[i], Bm1[i].y, z, s, seg, 0u, count);
                set_half<A>(Pz[i], nh);
                *(uint2 *)(my_row + soff(z) + A * (L >> 1) + 8 * seg) = nh;
            }
        }
        // request plane z+3 (the last plane read is Z1+1)
        load_plane(Pp3, Bp3, z + 3 <= Z1 + 1 ? poff(z + 3) : kOob);
        // colour 1 of plane z-1 (rows Y0 .. Y0+TY-1, planes Z0 .. Z1-1), then out
        if (own_row && z > Z0) {
            const int s = slot(z - 1);
#pragma unroll
            for (int i = 0; i < SEGS; ++i) {
                const int seg = i * TR + tl;
                set_half<A>(Pm1[i], seg_update(ac, Pm1[i], Pm2[i], Pz[i], Bm1[i], Bm2[i].y, z - 1, s, seg, 1u, true));
            }
        }
        const uint32_t pst = z > Z0 ? poff(z - 1) : kOob;
#pragma unroll
        for (int i = 0; i < SEGS; ++i) st16(rs_dst, pst + off_st[i], from_split(Pm1[i]));
        __syncthreads();
    };

    // A = (y + z) & 1 = (PP + 1 + k) & 1 with PP = (y + Z0) & 1, uniform over
    // a wavefront (rows of one parity)
    auto run = [&](auto pc) {
        constexpr int PP = decltype(pc)::value;
        using std::integral_constant;
        for (int z = Z0 - 1;; z += 6) {
            step(integral_constant<int, 0>{}, integral_constant<int, (PP + 1) & 1>{}, z);
            if (z + 1 > Z1) break;
            step(integral_constant<int, 1>{}, integral_constant<int, PP>{}, z + 1);
            if (z + 2 > Z1) break;
            step(integral_constant<int, 2>{}, integral_constant<int, (PP + 1) & 1>{}, z + 2);
            if (z + 3 > Z1) break;
            step(integral_constant<int, 3>{}, integral_constant<int, PP>{}, z + 3);
            if (z + 4 > Z1) break;
            step(integral_constant<int, 4>{}, integral_constant<int, (PP + 1) & 1>{}, z + 4);
            if (z + 5 > Z1) break;
            step(integral_constant<int, 5>{}, integral_constant<int, PP>{}, z + 5);
            if (z + 6 > Z1) break;
        }
    };
    if (__builtin_amdgcn_readfirstlane((y + Z0) & 1))
        run(std::integral_constant<int, 1>{});
    else
        run(std::integral_constant<int, 0>{});

    if constexpr (DE) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dE += __shfl_xor(dE, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dE;
        __syncthreads();
        if (threadIdx.x == 0) {
            long long tot = 0;
            for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) tot += red[w];
            if (tot != 0) atomicAdd(&a.dE[r], (unsigned long long)tot);
        }
    }
}

// Workgroup size: two row-parity classes of (TY + 4) / 2 rows, each padded
// to whole wavefronts.
int pass3d_threads(int L, int ty, int segs) {
    const int per_class = (ty + 4) / 2 * ((L / 16) / segs);
    return 2 * ((per_class + 63) / 64 * 64);
}

// Whether a launch shape fits: ty and D divide L, at most two segments per
// thread dividing the row's segments, the workgroup within the kernel's
// bound, and no EA kernel of 16 rows with two segments (it would not fit its
// registers).
bool shape_fits(int L, bool ea, int ty, int segs, int D, int *threads) {
    if (L < 32 || L > 1024 || L % 16 || (ty != 8 && ty != 16) || (segs != 1 && segs != 2)) return false;
    if ((L / 16) % segs || (ea && ty == 16 && segs == 2)) return false;
    if ((D != 16 && D != 32 && D != 64 && D != 128 && D != 256 && D != 512) || D > L || L % D || L % ty) return false;
    *threads = pass3d_threads(L, ty, segs);
    return *threads <= pass3d_max_threads(ty, segs);
}

// Launch shape for an edge: rows per strip, segments per thread, planes per
// z segment, workgroup size; false if the edge has none.  SPINMC_PASS3D_TY
// (8 or 16), SPINMC_PASS3D_SEGS (1 or 2) and SPINMC_PASS3D_D (16, 32, 64,
// 128, 256 or 512) override the first three; without them a shape smc_autotune
// measured for the edge, model and replica count is taken.  Results never
// depend on the shape.
bool pass3d_shape(int L, bool ea, int n_rep, int *ty, int *segs, int *D, int *threads) {
    if (L < 32 || L > 1024 || L % 16) return false;
    const char *ety = getenv("SPINMC_PASS3D_TY"), *esegs = getenv("SPINMC_PASS3D_SEGS"),
               *ed = getenv("SPINMC_PASS3D_D");
    Shape t;
    if (!(ety || esegs || ed) && tuned_shape(kShapePass3d, L, ea ? 1 : 0, n_rep, &t) &&
        shape_fits(L, ea, t.v[0], t.v[1], t.v[2], threads)) {
        *ty = t.v[0];
        *segs = t.v[1];
        *D = t.v[2];
        return true;
    }
    *ty = L >= 1024 ? 8 : 16;
    *segs = 1;
    if (ety && (atoi(ety) == 8 || atoi(ety) == 16)) *ty = atoi(ety);
    if (esegs && (atoi(esegs) == 1 || atoi(esegs) == 2)) *segs = atoi(esegs);
    if ((L / 16) % *segs) *segs = 1;
    if (*segs == 1 && pass3d_threads(L, *ty, 1) > pass3d_max_threads(*ty, 1) && (L / 16) % 2 == 0) *segs = 2;
    if (ea && *ty == 16 && *segs == 2) *ty = 8;  // the EA kernel of that shape would not fit its registers
    *D = L >= 1024 ? 128 : L >= 512 ? 32 : 16;
    if (ed && (atoi(ed) == 16 || atoi(ed) == 32 || atoi(ed) == 64 || atoi(ed) == 128 || atoi(ed) == 256 ||
               atoi(ed) == 512))
        *D = atoi(ed);
    return shape_fits(L, ea, *ty, *segs, *D, threads);
}

}  // namespace

bool pass3d_supported(int L) {
    int ty, segs, D, threads;
    return pass3d_shape(L, false, 1, &ty, &segs, &D, &threads) && pass3d_shape(L, true, 1, &ty, &segs, &D, &threads);
}

bool pass3d_launch_shape(int L, bool ea, int n_rep, Shape *out) {
    int threads;
    return pass3d_shape(L, ea, n_rep, &out->v[0], &out->v[1], &out->v[2], &threads);
}

bool pass3d_shape_valid(int L, bool ea, int ty, int segs, int D) {
    int threads;
    return shape_fits(L, ea, ty, segs, D, &threads);
}

hipError_t launch_ising3d_pass(const int8_t *src, int8_t *dst, const uint2 *pbonds, int rep_per_sample,
                               const ThrRow *thr, int64_t *dE, int n_rep, int L, Key key, uint32_t t,
                               hipStream_t s) {
    int ty, segs, D, threads;
    if (n_rep < 1 || src == dst || !pass3d_shape(L, pbonds != nullptr, n_rep, &ty, &segs, &D, &threads))
        return hipErrorInvalidValue;
    Pass3dArgs a;
    a.src = src;
    a.dst = dst;
    a.pbonds = pbonds;
    a.rep_per_sample = rep_per_sample;
    a.thr = thr;
    a.dE = (unsigned long long *)dE;
    a.key = key;
    a.t = t;
    a.L = L;
    a.D = D;
    a.strips = L / ty;
    a.zsegs = L / D;
    a.np = threads / 2;
    a.one2 = 0x00010001u;
    const size_t lds = (size_t)kRing * (size_t)(ty + 4) * (size_t)L * (pbonds ? 5 : 4) / 4;
    const dim3 grid((unsigned)((int64_t)n_rep * a.strips * a.zsegs));
#define SMC_PASS3D(MM, TT, SS, DD)                                                                          \
    if ((pbonds ? 2 : 0) == MM && ty == TT && segs == SS && (dE != nullptr) == DD) {                        \
        (void)hipFuncSetAttribute((const void *)k_ising3d_pass<MM, TT, SS, DD>,                             \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                    \
        SMC_LAUNCH((k_ising3d_pass<MM, TT, SS, DD>), grid, dim3(threads), lds, s, a);                       \
        return hipGetLastError();                                                                           \
    }
    SMC_PASS3D(0, 8, 1, false)
    SMC_PASS3D(0, 8, 2, false)
    SMC_PASS3D(0, 16, 1, false)
    SMC_PASS3D(0, 16, 2, false)
    SMC_PASS3D(2, 8, 1, false)
    SMC_PASS3D(2, 8, 2, false)
    SMC_PASS3D(2, 16, 1, false)
    SMC_PASS3D(0, 8, 1, true)
    SMC_PASS3D(0, 8, 2, true)
    SMC_PASS3D(0, 16, 1, true)
    SMC_PASS3D(0, 16, 2, true)
    SMC_PASS3D(2, 8, 1, true)
    SMC_PASS3D(2, 8, 2, true)
    SMC_PASS3D(2, 16, 1, true)
#undef SMC_PASS3D
    return hipErrorInvalidValue;
}

}  // namespace smc

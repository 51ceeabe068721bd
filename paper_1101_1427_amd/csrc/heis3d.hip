// Heisenberg half-sweeps of uniform 3D batches whose edge is a power of two
// (Sec. 4, Eq. 10): the same update as the generic kernel (same proposal
// and acceptance functions, same float32 arithmetic in the same order, same
// random numbers), with 32-bit shift/mask indexing instead of 64-bit
// divisions and one 12-byte load per neighbour.  A thread handles the
// colour-c sites of site pairs (2p, 2p+1), whose in-colour index is p.
#include <stdlib.h>

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

// ----------------------------------------------------------------------
// One-pass sweep (colour 0 then colour 1 in a single pass over the
// lattice).  A workgroup owns a tile of kTile x kTile sites in (x, y) over a
// segment of kSeg planes in z and streams down the planes: at step z it
// updates colour 0 of plane z on the tile plus a one-site ring, then colour 1
// of plane z-1 on the tile (its neighbours are then final), and writes plane
// z-1 of the tile.  The ring's colour-0 values are recomputed identically by
// the neighbouring tiles (every draw is keyed by the site), so tiles never
// exchange data; reads come from one buffer and writes go to the other.
// Planes live in LDS as structure-of-arrays float planes of
// (kTile+4) x (kTile+4) sites (two-site halo), five planes in a ring.
//
// Order within step z: request plane z+2 from global memory into
// registers, colour 0 of plane z, colour 1 of plane z-1, then wait for the
// requested plane, put it into the slot of plane z-3, and only then store
// the tile's plane z-1 to global memory.  Loads and stores share one
// completion counter on this target, so a wait for data also waits for
// every store issued before it; in this order the stores a wait covers were
// issued two update phases earlier and have completed.
constexpr int kTile = 32;
constexpr int kSeg = 32;
constexpr int kW = kTile + 4;       // staged width with the halo
constexpr int kPlane = kW * kW;     // sites per staged plane
constexpr int kRing = 5;
constexpr int kTiledThreads = 576;  // one colour-0 cell per thread (see update_colour0)
constexpr int kLoadsPerThread = (kPlane + kTiledThreads - 1) / kTiledThreads;

struct TiledArgs {
    const float *src;  // [n_rep][N][3]
    float *dst;
    const float *beta;
    int64_t *acc;
    Key key;
    uint32_t t;
    int lgL;
    int64_t N;
    int tiles, segs;   // tiles per row of tiles, segments per replica
    int xcd_remap;     // 1: consecutive tiles of a segment on one XCD (shared halo lines in its L2)
    int renorm;        // 1: the stored spins are renormalised (this sweep ends a renormalisation period)
};

struct PlaneRegs {
    F3 v[kLoadsPerThread];
};

__device__ __forceinline__ void load_plane(const float *src, int L, int lgL, int x0, int y0, int z, PlaneRegs &pr) {
    const uint32_t m = (uint32_t)L - 1u;
    const uint32_t zz = (uint32_t)z & m;
#pragma unroll
    for (int j = 0; j < kLoadsPerThread; ++j) {
        const int q = (int)threadIdx.x + j * kTiledThreads;
        if (q < kPlane) {
            const int v = q / kW, u = q - v * kW;
            const uint32_t x = (uint32_t)(x0 - 2 + u) & m, y = (uint32_t)(y0 - 2 + v) & m;
            pr.v[j] = ld(src, (((zz << lgL) + y) << lgL) + x);
        }
    }
}

__device__ __forceinline__ int slot_of(int z) { return (z + 2 * kRing) % kRing; }  // z >= -2 * kRing

__device__ __forceinline__ void store_plane(float *ring, int slot, const PlaneRegs &pr) {
    float *P = ring + slot * 3 * kPlane;
#pragma unroll
    for (int j = 0; j < kLoadsPerThread; ++j) {
        const int q = (int)threadIdx.x + j * kTiledThreads;
        if (q < kPlane) {
            P[q] = pr.v[j].x;
            P[kPlane + q] = pr.v[j].y;
            P[2 * kPlane + q] = pr.v[j].z;
        }
    }
}

__device__ __forceinline__ F3 lds3(const float *ring, int slot, int q) {
    const float *P = ring + slot * 3 * kPlane;
    F3 r;
    r.x = P[q];
    r.y = P[kPlane + q];
    r.z = P[2 * kPlane + q];
    return r;
}

// Update the colour-c site at staged cell (u, v) of plane z (ring slot sz);
// planes z-1 and z+1 sit in slots sm and sp.  Returns whether it moved.
__device__ __forceinline__ bool update_cell(float *ring, int sm, int sz, int sp, int u, int v, int c, int x0, int y0,
                                            int z, const TiledArgs &a, int r, float beta) {
    const uint32_t m = (1u << a.lgL) - 1u;
    const uint32_t zz = (uint32_t)z & m;
    const uint32_t x = (uint32_t)(x0 - 2 + u) & m, y = (uint32_t)(y0 - 2 + v) & m;
    const int q = v * kW + u;
    const F3 nx1 = lds3(ring, sz, q + 1), nx0 = lds3(ring, sz, q - 1);
    const F3 ny1 = lds3(ring, sz, q + kW), ny0 = lds3(ring, sz, q - kW);
    const F3 nz1 = lds3(ring, sp, q), nz0 = lds3(ring, sm, q);
    const F3 so = lds3(ring, sz, q);
    float3 hf = make_float3(0.f, 0.f, 0.f);
    hf.x += nx1.x; hf.y += nx1.y; hf.z += nx1.z;
    hf.x += nx0.x; hf.y += nx0.y; hf.z += nx0.z;
    hf.x += ny1.x; hf.y += ny1.y; hf.z += ny1.z;
    hf.x += ny0.x; hf.y += ny0.y; hf.z += ny0.z;
    hf.x += nz1.x; hf.y += nz1.y; hf.z += nz1.z;
    hf.x += nz0.x; hf.y += nz0.y; hf.z += nz0.z;
    const uint32_t i = (((zz << a.lgL) + y) << a.lgL) + x;
    const uint4 w = philox4x32_10_wide(make_uint4(i >> 1, a.t, (uint32_t)r, 2 * kTagHeis + (uint32_t)c), a.key);
    const float3 sp3 = heis_proposal(unit23f(w.x), unit23f(w.y));
    const float dE = -((sp3.x - so.x) * hf.x + (sp3.y - so.y) * hf.y + (sp3.z - so.z) * hf.z);
    if (dE <= 0.0f || unit23f(w.z) < heis_boltzmann(beta, dE)) {
        float *P = ring + sz * 3 * kPlane;
        P[q] = sp3.x;
        P[kPlane + q] = sp3.y;
        P[2 * kPlane + q] = sp3.z;
        return true;
    }
    return false;
}

// First staged column u >= lo of staged row v whose site has colour c in plane z.
__device__ __forceinline__ int first_cell(int lo, int v, int c, int x0, int y0, int z) {
    return lo + ((c - (x0 - 2 + lo) - (y0 - 2 + v) - z) & 1);
}

// Colour 0 of plane z on the tile and on the one-site ring around it without
// the ring's corners (no tile site neighbours them): staged rows 1 and kW-2
// over columns [2, kW-2), rows 2 .. kW-3 over columns [1, kW-1).  That is
// kTile/2 + kTile*(kTile/2 + 1) + kTile/2 cells, one per thread.
constexpr int kRingRowCells = kTile / 2;
constexpr int kMidRowCells = kTile / 2 + 1;
constexpr int kColour0Cells = 2 * kRingRowCells + kTile * kMidRowCells;
static_assert(kColour0Cells == kTiledThreads, "one colour-0 cell per thread");

__device__ __forceinline__ int update_colour0(float *ring, int sm, int sz, int sp, int x0, int y0, int z,
                                              const TiledArgs &a, int r, float beta, bool count) {
    const int k = (int)threadIdx.x;
    int v, lo, j;
    if (k < kRingRowCells) {
        v = 1, lo = 2, j = k;
    } else if (k < kRingRowCells + kTile * kMidRowCells) {
        const int kk = k - kRingRowCells;
        v = 2 + kk / kMidRowCells, lo = 1, j = kk % kMidRowCells;
    } else {
        v = kW - 2, lo = 2, j = k - kRingRowCells - kTile * kMidRowCells;
    }
    const int u = first_cell(lo, v, 0, x0, y0, z) + 2 * j;
    const bool moved = update_cell(ring, sm, sz, sp, u, v, 0, x0, y0, z, a, r, beta);
    return moved && count && u >= 2 && u < 2 + kTile && v >= 2 && v < 2 + kTile ? 1 : 0;
}

// Colour 1 of plane z on the tile: kTile * kTile / 2 cells, one per thread
// of the first kTile * kTile / 2.
__device__ __forceinline__ int update_colour1(float *ring, int sm, int sz, int sp, int x0, int y0, int z,
                                              const TiledArgs &a, int r, float beta) {
    const int k = (int)threadIdx.x;
    if (k >= kTile * kTile / 2) return 0;
    const int v = 2 + k / (kTile / 2), j = k % (kTile / 2);
    const int u = first_cell(2, v, 1, x0, y0, z) + 2 * j;
    return update_cell(ring, sm, sz, sp, u, v, 1, x0, y0, z, a, r, beta) ? 1 : 0;
}

__global__ __launch_bounds__(kTiledThreads) void k_heis3d_tiled(TiledArgs a) {
    extern __shared__ __align__(16) float ring[];  // [kRing][3][kPlane]
    __shared__ int red[kTiledThreads / 64];
    const int L = 1 << a.lgL;
    const int per_rep = a.tiles * a.tiles * a.segs;
    // Workgroups go to the XCDs round-robin; with the remap, XCD k runs a
    // contiguous range of logical blocks (whole segments), so the halo rows
    // and columns that neighbouring tiles share are fetched once into its L2.
    const uint32_t nblk = gridDim.x, b = blockIdx.x;
    const int lb = (int)((a.xcd_remap && (nblk & 7u) == 0) ? (b & 7u) * (nblk >> 3) + (b >> 3) : b);
    const int r = lb / per_rep;
    const int rem = lb % per_rep;
    const int seg = rem / (a.tiles * a.tiles), tile = rem % (a.tiles * a.tiles);
    const int x0 = (tile % a.tiles) * kTile, y0 = (tile / a.tiles) * kTile;
    const int z0 = seg * kSeg, z1 = z0 + (kSeg < L ? kSeg : L);
    const float *src = a.src + (size_t)r * 3 * (size_t)a.N;
    float *dst = a.dst + (size_t)r * 3 * (size_t)a.N;
    const float beta = a.beta[r];
    const uint32_t m = (uint32_t)L - 1u;

    // planes z0-2 .. z0 into their slots
    PlaneRegs pr;
    for (int z = z0 - 2; z <= z0; ++z) {
        load_plane(src, L, a.lgL, x0, y0, z, pr);
        store_plane(ring, slot_of(z), pr);
    }
    __syncthreads();
    int n_acc = 0;
    for (int z = z0 - 1; z <= z1; ++z) {
        const bool fetch = z + 2 <= z1 + 1;
        if (fetch) load_plane(src, L, a.lgL, x0, y0, z + 2, pr);
        // colour 0 of plane z on the tile and a one-site ring (planes z-1 .. z+1)
        n_acc += update_colour0(ring, slot_of(z - 1), slot_of(z), slot_of(z + 1), x0, y0, z, a, r, beta,
                                z >= z0 && z < z1);
        __syncthreads();
        // colour 1 of plane z-1 on the tile (planes z-2 .. z)
        if (z >= z0 + 1) n_acc += update_colour1(ring, slot_of(z - 2), slot_of(z - 1), slot_of(z), x0, y0, z - 1, a,
                                                 r, beta);
        // plane z+2 into the slot of plane z-3.  The wait is explicit and on
        // every path, so that no load is left pending across the loop (the
        // next step's request would otherwise wait behind this step's stores).
        __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));  // vmcnt(0)
        if (fetch) store_plane(ring, slot_of(z + 2), pr);
        __syncthreads();
        if (z >= z0 + 1) {
            // the tile's plane z-1 out
            const int zc = z - 1;
            const uint32_t zz = (uint32_t)zc & m;
            for (int k = threadIdx.x; k < kTile * kTile; k += kTiledThreads) {
                const int v = 2 + k / kTile, u = 2 + k % kTile;
                F3 val = lds3(ring, slot_of(zc), v * kW + u);
                if (a.renorm) {
                    const float3 n = heis_unit(val.x, val.y, val.z);
                    val.x = n.x;
                    val.y = n.y;
                    val.z = n.z;
                }
                const uint32_t x = (uint32_t)(x0 + u - 2) & m, y = (uint32_t)(y0 + v - 2) & m;
                *(F3 *)(dst + 3 * (size_t)((((zz << a.lgL) + y) << a.lgL) + x)) = val;
            }
        }
    }
    if (a.acc) {
        int v = n_acc;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            int tot = 0;
            for (int w = 0; w < kTiledThreads / 64; ++w) tot += red[w];
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
    SMC_LAUNCH(k_heis3d_half, dim3((unsigned)(a.bpr * n_rep)), dim3(kThreads), 0, s, a, c);
    return hipGetLastError();
}

bool heis3d_tiled_supported(int dim, int L) { return heis3d_supported(dim, L) && L >= kTile; }

size_t heis3d_tiled_lds_bytes() { return (size_t)kRing * 3 * kPlane * sizeof(float); }

hipError_t launch_heis3d_tiled(const float *src, float *dst, const float *beta, int64_t *acc, int n_rep, int L, Key key,
                               uint32_t t, bool renorm, hipStream_t s) {
    TiledArgs a;
    a.renorm = renorm ? 1 : 0;
    a.src = src;
    a.dst = dst;
    a.beta = beta;
    a.acc = acc;
    a.key = key;
    a.t = t;
    a.lgL = 0;
    while ((1 << a.lgL) < L) ++a.lgL;
    a.N = (int64_t)L * L * L;
    a.tiles = L / kTile;
    a.segs = L > kSeg ? L / kSeg : 1;
    {
        const char *e = getenv("SPINMC_XCD_REMAP");
        a.xcd_remap = (e && e[0] == '0') ? 0 : 1;
    }
    const size_t lds = heis3d_tiled_lds_bytes();
    (void)hipFuncSetAttribute((const void *)k_heis3d_tiled, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const unsigned blocks = (unsigned)(a.tiles * a.tiles * a.segs * n_rep);
    SMC_LAUNCH(k_heis3d_tiled, dim3(blocks), dim3(kTiledThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace smc

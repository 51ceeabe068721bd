// Sweeps of batches of small 2D lattices with each replica in LDS: parallel
// tempering of uneven batches (Sec. 6, Eq. 12; many independent instances at
// once) and plain sweeps of small uniform batches.
//
// A launch per lattice size runs one workgroup per replica: it holds the
// replica in LDS, runs `sweeps` sweeps (colour 0 then colour 1 each, sweep
// indices from the device counter *t_dev on) and writes it back, tracking
// the replica's energy.  Couplings are read from a
// colour-split copy made once per call; the replicas of one instance run
// next to each other on one XCD, so the copy is served from its L2 (keeping
// the couplings out of LDS leaves room for more workgroups per CU, which
// measured faster than staging them).  Results equal those of the generic
// per-site kernels step for step.
//
// LDS layout of a replica of edge L (L^2 bytes): row y holds the L/2 sites
// with even x (array E, x = 2i) and then the L/2 sites with odd x (array O),
// one byte per site, (1 - s)/2.  E sites of row y have colour y & 1.  The
// coupling copy has the same shape twice: plane X holds the bond from each
// site to its +x neighbour, plane Y the bond to its +y neighbour, as bytes
// (1 - J)/2.
#include <string.h>

#include "internal.hpp"
#include "intrin.hpp"

namespace smc {
namespace {

constexpr int kMaxThreads = 512;
constexpr int kBatch = 8;  // 16-byte spin loads in flight per thread while staging a replica


// Thresholds by the number n of unsatisfied bonds (Delta E = 8 - 4n): n = 0
// and 1 take the high halves of thr[2] and thr[1]; n >= 2 is always accepted
// (0xFFFF, a head of 0xFFFF goes through the exact path).
struct Lut2 {
    uint32_t lo, hi;
};

__device__ __forceinline__ Lut2 lut2(const ThrRow &row) {
    const uint32_t t2 = row.m[2].x, t1 = row.m[1].x;  // <= 0xFFFF (checked on the host)
    Lut2 k;
    k.lo = (t2 & 0xFFu) | ((t1 & 0xFFu) << 8) | 0xFFFF0000u;
    k.hi = (t2 >> 8) | ((t1 >> 8) << 8) | 0xFFFF0000u;
    return k;
}

// Flip flags of four sites from counts n (bytes) and heads wa (sites 0, 1),
// wb (sites 2, 3); eq collects threshold - head per 16-bit lane.
__device__ __forceinline__ uint32_t decide4(uint32_t n, uint32_t wa, uint32_t wb, Lut2 k, uint32_t one2,
                                            uint32_t &eq) {
    const uint32_t tl = perm(0xFFFFFFFFu, k.lo, n);
    const uint32_t th = perm(0xFFFFFFFFu, k.hi, n);
    const uint32_t ta = perm(th, tl, 0x05010400u);
    const uint32_t tb = perm(th, tl, 0x07030602u);
    const uint32_t ra = min16(sub_sat16(ta, wa), one2);
    const uint32_t rb = min16(sub_sat16(tb, wb), one2);
    eq = min16(eq, min16(sub16(ta, wa), sub16(tb, wb)));
    return perm(rb, ra, 0x06040200u);
}

// One colour-c group: the eight colour-c sites of row y with in-array
// indices 8k .. 8k+7 (one Philox draw).  S: spins, X/Y: coupling planes
// (either in LDS or in global memory), all with the row layout above.
// Offsets (in a row-layout plane) of the words a colour-c group reads.
struct GroupAt {
    uint32_t own, oth, ext, below, above;
};

// yL = y * L (kept by the caller as the rows advance, without multiplications).
__device__ __forceinline__ GroupAt group_at(int L, int yL, int y, int k, int c) {
    const int half = L >> 1, N = L * L;
    const int a = (y & 1) == c ? 0 : 1;
    const int ymL = yL == 0 ? N - L : yL - L, ypL = yL == N - L ? 0 : yL + L;
    GroupAt o;
    o.own = (uint32_t)(yL + a * half + 8 * k);
    o.oth = (uint32_t)(yL + (1 - a) * half + 8 * k);
    // the extra word of the other array: the word before (a = 0) or after (a = 1), wrapping in the row
    o.ext = (uint32_t)(yL + (1 - a) * half +
                       (a == 0 ? (k == 0 ? half - 4 : 8 * k - 4) : (8 * k + 8 == half ? 0 : 8 * k + 8)));
    o.below = (uint32_t)(ymL + a * half + 8 * k);
    o.above = (uint32_t)(ypL + a * half + 8 * k);
    return o;
}

// Coupling bytes of a group: +x bonds of the own sites (xo), of the other
// array (xt, with its extra word xe), +y bonds of the own sites (yo) and of
// the sites below (ym).
struct GroupCoup {
    uint2 xo, xt, yo, ym;
    uint32_t xe;
};

__device__ __forceinline__ GroupCoup group_coup(const uint8_t *X, const uint8_t *Yp, const GroupAt &o) {
    GroupCoup j;
    j.xo = *(const uint2 *)(X + o.own);
    j.xt = *(const uint2 *)(X + o.oth);
    j.xe = *(const uint32_t *)(X + o.ext);
    j.yo = *(const uint2 *)(Yp + o.own);
    j.ym = *(const uint2 *)(Yp + o.below);
    return j;
}

template <bool EA>
__device__ __forceinline__ void group(uint8_t *S, const GroupAt &o, const GroupCoup &J, int L, int y, int k, int c,
                                      uint32_t t, uint32_t r, Key key, Lut2 K, const ThrRow &th, uint32_t one2,
                                      uint32_t &cnt, uint32_t &nsum) {
    const int a = (y & 1) == c ? 0 : 1;
    const int o_own = o.own;
    const uint2 own = *(const uint2 *)(S + o.own);
    const uint2 oth = *(const uint2 *)(S + o.oth);
    const uint32_t ext = *(const uint32_t *)(S + o.ext);
    const uint2 vm = *(const uint2 *)(S + o.below);
    const uint2 vp = *(const uint2 *)(S + o.above);
    uint2 jxo = make_uint2(0u, 0u), jxt = jxo, jyo = jxo, jym = jxo;
    uint32_t jxe = 0u;
    if constexpr (EA) {
        jxo = J.xo;
        jxt = J.xt;
        jxe = J.xe;
        jyo = J.yo;
        jym = J.ym;
    }
    uint32_t xm0, xm1, xp0, xp1;  // unsatisfied flags of the -x and +x bonds
    if (a == 0) {
        // E site 2i: -x neighbour O[i-1] over its +x bond, +x neighbour O[i] over the own +x bond
        const uint32_t t0 = oth.x ^ jxt.x, t1 = oth.y ^ jxt.y, te = ext ^ jxe;
        xm0 = own.x ^ alignbyte(t0, te, 3);
        xm1 = own.y ^ alignbyte(t1, t0, 3);
        xp0 = own.x ^ oth.x ^ jxo.x;
        xp1 = own.y ^ oth.y ^ jxo.y;
    } else {
        // O site 2i+1: -x neighbour E[i] over its +x bond, +x neighbour E[i+1] over the own +x bond
        xm0 = own.x ^ oth.x ^ jxt.x;
        xm1 = own.y ^ oth.y ^ jxt.y;
        xp0 = own.x ^ alignbyte(oth.y, oth.x, 1) ^ jxo.x;
        xp1 = own.y ^ alignbyte(ext, oth.y, 1) ^ jxo.y;
    }
    const uint32_t n0 = (xm0 + xp0) + ((own.x ^ vm.x ^ jym.x) + (own.x ^ vp.x ^ jyo.x));
    const uint32_t n1 = (xm1 + xp1) + ((own.y ^ vm.y ^ jym.y) + (own.y ^ vp.y ^ jyo.y));
    const uint32_t g = (uint32_t)(y * (L >> 4) + k);
    const uint4 w = philox4x32_10(make_uint4(g, t, r, 2 * kTagHead + (uint32_t)c), key);
    uint32_t eq = 0xFFFFFFFFu;
    uint32_t F0 = decide4(n0, w.x, w.y, K, one2, eq);
    uint32_t F1 = decide4(n1, w.z, w.w, K, one2, eq);
    const bool tie = ((eq & 0xFFFFu) == 0u) || ((eq >> 16) == 0u);
    if (__builtin_expect(__any(tie), 0)) {
        // Exact decisions of the sites whose head equals the high half of the
        // threshold (probability 2^-16 each).  A wavefront that meets one
        // holds up its workgroup at the next barrier, so the path is short: a
        // mask of the tied sites, then one pass per tied site of the lane with
        // most of them (almost always one), each drawing the single tail it
        // needs.
        uint32_t tm = 0;  // bit s: site s (0 .. 7) is tied
        if (tie) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const uint32_t n = q ? n1 : n0;
                const uint32_t tl = perm(0xFFFFFFFFu, K.lo, n), thh = perm(0xFFFFFFFFu, K.hi, n);
                const uint32_t da = perm(thh, tl, 0x05010400u) ^ (q ? w.z : w.x);
                const uint32_t db = perm(thh, tl, 0x07030602u) ^ (q ? w.w : w.y);
                const uint32_t m4 = ((da & 0xFFFFu) == 0u ? 1u : 0u) | ((da >> 16) == 0u ? 2u : 0u) |
                                    ((db & 0xFFFFu) == 0u ? 4u : 0u) | ((db >> 16) == 0u ? 8u : 0u);
                tm |= m4 << (4 * q);
            }
        }
        while (__any(tm != 0u)) {
            if (tm != 0u) {
                const uint32_t s = __builtin_ctz(tm), b = 8u * (s & 3u);
                tm &= tm - 1u;
                const uint32_t ns = ((s < 4u ? n0 : n1) >> b) & 0xFFu;
                uint32_t flip = 1u;  // a head of 0xFFFF at a site with Delta E <= 0
                if (ns < 2u) {
                    // the head equals the threshold's high half: compare the tail
                    const uint32_t lo = ns == 0u ? th.m[2].y : th.m[1].y;
                    flip = tail16(g * 8u + s, t, r, (uint32_t)c, key) < lo ? 1u : 0u;
                }
                const uint32_t keep = ~(0xFFu << b), set = flip << b;
                if (s < 4u)
                    F0 = (F0 & keep) | set;
                else
                    F1 = (F1 & keep) | set;
            }
        }
    }
    *(uint2 *)(S + o_own) = make_uint2(own.x ^ F0, own.y ^ F1);
    // Delta E of a flip with n unsatisfied bonds is 4 (2 - n)
    const uint32_t m0 = bytes_ff(F0), m1 = bytes_ff(F1);
    cnt = __builtin_amdgcn_sad_u8(F0, 0u, __builtin_amdgcn_sad_u8(F1, 0u, cnt));
    nsum = __builtin_amdgcn_sad_u8(n0 & m0, 0u, __builtin_amdgcn_sad_u8(n1 & m1, 0u, nsum));
}

// One workgroup per replica of the work list (EA: with couplings).
template <bool EA>
__global__ __launch_bounds__(kMaxThreads) void k_uneven2d_sweep(Uneven2dArgs a, const int32_t *work, int L) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ long long red[kMaxThreads / 64];
    const uint32_t nblk = gridDim.x, b = blockIdx.x;
    // consecutive work items (the replicas of one chain) on one XCD, sharing its L2
    const uint32_t logical = (nblk & 7u) ? b : (b & 7u) * (nblk >> 3) + (b >> 3);
    const int r = work[logical];
    const int row = a.row_of_rep[r];
    if (row < 0) return;  // chain without a valid permutation: unchanged
    const smc_inst g = a.inst[r];
    const int N = L * L, half = L >> 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    uint8_t *S = smem;
    const uint8_t *X = nullptr, *Yp = nullptr;
    int8_t *gs = a.spins + g.spin_off;

    // (row, 16-byte piece) of index i = tid + j*nt, advanced without divisions
    const int G = L >> 4;  // pieces per row = draw groups per row and colour
    const int dy = nt / G, dk = nt % G;
    const int y0 = tid / G, k0 = tid % G;

    // row-major +-1 -> split 0/1 bytes; up to kBatch 16-byte loads per
    // thread are in flight before the first is converted
    for (int i0 = tid, y = y0, m = k0; i0 < N / 16; i0 += kBatch * nt) {
        uint4 v[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            const int i = i0 + j * nt;
            if (i < N / 16) v[j] = *(const uint4 *)(gs + (int64_t)i * 16);
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
            if (i0 + j * nt < N / 16) {
                const uint32_t mm = 0x01010101u;
                const uint32_t b0 = (v[j].x >> 1) & mm, b1 = (v[j].y >> 1) & mm, b2 = (v[j].z >> 1) & mm,
                               b3 = (v[j].w >> 1) & mm;
                *(uint2 *)(S + y * L + 8 * m) = make_uint2(perm(b1, b0, 0x06040200u), perm(b3, b2, 0x06040200u));
                *(uint2 *)(S + y * L + half + 8 * m) =
                    make_uint2(perm(b1, b0, 0x07050301u), perm(b3, b2, 0x07050301u));
            }
            y += dy;
            m += dk;
            if (m >= G) {
                m -= G;
                ++y;
            }
        }
    }
    if constexpr (EA) {
        X = a.csplit + g.coup_off;
        Yp = X + N;
    }
    const ThrRow &th = a.thr[row];
    const Lut2 K = lut2(th);
    const uint32_t t0 = *a.t_dev;
    __syncthreads();

    uint32_t cnt = 0u, nsum = 0u;
    const int groups = N >> 4;  // per colour
    // The couplings of the next group are requested before this one is
    // computed; the loop body handles two groups with alternating register
    // sets, so nothing is copied from one iteration to the next.
    struct Pos {
        int y, yL, k;
    };
    auto advance = [&](Pos p) {
        p.y += dy;
        p.yL += dy * L;
        p.k += dk;
        if (p.k >= G) {
            p.k -= G;
            ++p.y;
            p.yL += L;
        }
        return p;
    };
#pragma unroll 1
    for (int sw = 0; sw < a.sweeps; ++sw) {
        const uint32_t t = t0 + (uint32_t)sw;
#pragma unroll 1
        for (int c = 0; c < 2; ++c) {
            // (past the last group the position is clamped to row 0, so every
            // coupling load stays inside the sample and none is conditional)
            Pos pa{y0 < L ? y0 : 0, y0 < L ? y0 * L : 0, k0};
            GroupAt ata = group_at(L, pa.yL, pa.y, pa.k, c);
            GroupCoup Ja{};
            if (EA) Ja = group_coup(X, Yp, ata);
#pragma unroll 1
            for (int q = tid; q < groups;) {
                const Pos pb = advance(pa);
                const bool hb = q + nt < groups;
                const GroupAt atb = group_at(L, hb ? pb.yL : 0, hb ? pb.y : 0, pb.k, c);
                GroupCoup Jb{};
                if (EA) Jb = group_coup(X, Yp, atb);
                group<EA>(S, ata, Ja, L, pa.y, pa.k, c, t, (uint32_t)r, a.key, K, th, a.one2, cnt, nsum);
                q += nt;
                if (!hb) break;
                pa = advance(pb);
                const bool ha = q + nt < groups;
                ata = group_at(L, ha ? pa.yL : 0, ha ? pa.y : 0, pa.k, c);
                if (EA) Ja = group_coup(X, Yp, ata);
                group<EA>(S, atb, Jb, L, pb.y, pb.k, c, t, (uint32_t)r, a.key, K, th, a.one2, cnt, nsum);
                q += nt;
            }
            __syncthreads();
        }
    }

    // split 0/1 bytes -> row-major +-1
    for (int i = tid, y = y0, m = k0; i < N / 16; i += nt) {
        const uint2 e = *(const uint2 *)(S + y * L + 8 * m);
        const uint2 o = *(const uint2 *)(S + y * L + half + 8 * m);
        const uint32_t w0 = perm(o.x, e.x, 0x05010400u), w1 = perm(o.x, e.x, 0x07030602u);
        const uint32_t w2 = perm(o.y, e.y, 0x05010400u), w3 = perm(o.y, e.y, 0x07030602u);
        *(uint4 *)(gs + (int64_t)i * 16) = make_uint4(bytes_pm1(w0), bytes_pm1(w1), bytes_pm1(w2), bytes_pm1(w3));
        y += dy;
        m += dk;
        if (m >= G) {
            m -= G;
            ++y;
        }
    }
    // energy: sum over flips of 4 (2 - n)
    long long v = 2ll * (long long)cnt - (long long)nsum;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
        long long tot = 0;
        for (int w = 0; w < (nt >> 6); ++w) tot += red[w];
        a.E[r] += 4 * tot;
    }
}

// Couplings of every sample into the colour-split planes (one thread per 16
// sites of a row): X[y][a][i] = (1 - J_x(site))/2, Y likewise.
__global__ __launch_bounds__(256) void k_coup_split2d(const int8_t *coup, uint8_t *out, const smc_inst *samples,
                                                     int n_samples, int64_t chunks_total, const int64_t *chunk_start) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= chunks_total) return;
    // sample by binary search over its first chunk
    int lo = 0, hi = n_samples - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_start[mid] <= gid) lo = mid; else hi = mid - 1;
    }
    const smc_inst g = samples[lo];
    const int L = g.L, half = L >> 1;
    const int64_t N = (int64_t)L * L;
    const int64_t i = gid - chunk_start[lo];  // chunk within the sample: plane, row, 16-site piece
    const int per_plane = (int)(N / 16);
    const int plane = (int)(i / per_plane), rem = (int)(i % per_plane);
    const int y = rem / (L >> 4), m = rem % (L >> 4);
    const uint4 v = *(const uint4 *)(coup + g.coup_off + plane * N + (int64_t)y * L + 16 * m);
    const uint32_t mm = 0x01010101u;
    const uint32_t b0 = (v.x >> 1) & mm, b1 = (v.y >> 1) & mm, b2 = (v.z >> 1) & mm, b3 = (v.w >> 1) & mm;
    uint8_t *o = out + g.coup_off + plane * N + (int64_t)y * L;
    *(uint2 *)(o + 8 * m) = make_uint2(perm(b1, b0, 0x06040200u), perm(b3, b2, 0x06040200u));
    *(uint2 *)(o + half + 8 * m) = make_uint2(perm(b1, b0, 0x07050301u), perm(b3, b2, 0x07050301u));
}

__global__ void k_set_step(uint32_t *t_dev, uint32_t t) { *t_dev = t; }
__global__ void k_advance_step(uint32_t *t_dev, uint32_t inc) { *t_dev += inc; }

}  // namespace

bool uneven2d_edge_supported(int L) { return L >= 16 && L <= 256 && L % 16 == 0; }

size_t uneven2d_lds_bytes(int L) { return (size_t)L * L; }

const void *uneven2d_kernel(bool ea) {
    return ea ? (const void *)k_uneven2d_sweep<true> : (const void *)k_uneven2d_sweep<false>;
}

hipError_t uneven2d_prepare_kernel(bool ea, int L) {
    return hipFuncSetAttribute(uneven2d_kernel(ea), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)uneven2d_lds_bytes(L));
}

Uneven2dArgs make_uneven2d_args(int8_t *spins, const smc_inst *inst, const uint8_t *csplit, const int32_t *row_of_rep,
                                const ThrRow *thr, int64_t *E, const uint32_t *t_dev, Key key) {
    Uneven2dArgs a;
    a.spins = spins;
    a.inst = inst;
    a.csplit = csplit;
    a.row_of_rep = row_of_rep;
    a.thr = thr;
    a.E = E;
    a.t_dev = t_dev;
    a.sweeps = 1;
    a.key = key;
    a.one2 = 0x00010001u;
    return a;
}

hipError_t launch_coup_split2d(const int8_t *coup, uint8_t *out, const smc_inst *samples, int n_samples,
                               int64_t chunks_total, const int64_t *chunk_start, hipStream_t s) {
    if (chunks_total == 0) return hipSuccess;
    SMC_LAUNCH(k_coup_split2d, dim3((unsigned)((chunks_total + 255) / 256)), dim3(256), 0, s, coup, out,
                       samples, n_samples, chunks_total, chunk_start);
    return hipGetLastError();
}

hipError_t launch_set_step(uint32_t *t_dev, uint32_t t, hipStream_t s) {
    SMC_LAUNCH(k_set_step, dim3(1), dim3(1), 0, s, t_dev, t);
    return hipGetLastError();
}

// ---- graph nodes ----
hipError_t add_uneven2d_sweep_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, size_t n_deps,
                                   const Uneven2dArgs &a, const int32_t *work, int n_work, int L, bool ea,
                                   int threads) {
    Uneven2dArgs args = a;
    const int32_t *w = work;
    int edge = L;
    void *params[] = {&args, &w, &edge};
    hipKernelNodeParams p;
    memset(&p, 0, sizeof p);
    p.func = const_cast<void *>(uneven2d_kernel(ea));
    p.gridDim = dim3((unsigned)n_work);
    p.blockDim = dim3((unsigned)threads);
    p.sharedMemBytes = (unsigned)uneven2d_lds_bytes(L);
    p.kernelParams = params;
    p.extra = nullptr;
    if (const char *why = launch_config_error((uint64_t)n_work, (uint64_t)threads, p.sharedMemBytes))
        return reject_launch("k_uneven2d_sweep (graph node)", (uint64_t)n_work, (uint64_t)threads, p.sharedMemBytes,
                             why);
    return hipGraphAddKernelNode(node, g, deps, n_deps, &p);
}

hipError_t add_advance_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, size_t n_deps,
                            uint32_t *t_dev, uint32_t inc) {
    uint32_t *tp = t_dev;
    uint32_t by = inc;
    void *params[] = {&tp, &by};
    hipKernelNodeParams p;
    memset(&p, 0, sizeof p);
    p.func = (void *)k_advance_step;
    p.gridDim = dim3(1);
    p.blockDim = dim3(1);
    p.kernelParams = params;
    return hipGraphAddKernelNode(node, g, deps, n_deps, &p);
}

hipError_t launch_uneven2d_sweep(const Uneven2dArgs &a, const int32_t *work, int n_work, int L, bool ea, int threads,
                                 hipStream_t s) {
    const size_t lds = uneven2d_lds_bytes(L);
    if (ea)
        SMC_LAUNCH(k_uneven2d_sweep<true>, dim3(n_work), dim3(threads), lds, s, a, work, L);
    else
        SMC_LAUNCH(k_uneven2d_sweep<false>, dim3(n_work), dim3(threads), lds, s, a, work, L);
    return hipGetLastError();
}

hipError_t launch_advance_step(uint32_t *t_dev, hipStream_t s, uint32_t inc) {
    SMC_LAUNCH(k_advance_step, dim3(1), dim3(1), 0, s, t_dev, inc);
    return hipGetLastError();
}

}  // namespace smc

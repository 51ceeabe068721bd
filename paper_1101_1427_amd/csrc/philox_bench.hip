// Throughput of the counter-based generator alone (Sec. 3.3 measures its
// generators the same way, Fig. 4): every thread draws Philox4x32-10 blocks
// and folds their words into one XOR, so the kernel does no memory traffic
// beyond one word per thread and runs at the VALU rate of the generator.
// The draws are advanced four at a time, as in the sweep kernels.
#include "internal.hpp"

namespace smc {
namespace {

constexpr int kBenchBlock = 256;

__global__ __launch_bounds__(kBenchBlock) void k_philox_bench(Key key, uint32_t t, uint32_t r, uint32_t tag,
                                                              uint32_t n_threads, int per_thread, uint32_t *out) {
    const uint32_t i = blockIdx.x * kBenchBlock + threadIdx.x;
    if (i >= n_threads) return;
    uint32_t acc = 0;
    int k = 0;
    for (; k + 4 <= per_thread; k += 4) {
        uint4 w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = make_uint4(i + (uint32_t)(k + q) * n_threads, t, r, tag);
        philox4x32_10_multi<4>(w, key);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc ^= w[q].x ^ w[q].y ^ w[q].z ^ w[q].w;
    }
    for (; k < per_thread; ++k) {
        const uint4 w = philox4x32_10(make_uint4(i + (uint32_t)k * n_threads, t, r, tag), key);
        acc ^= w.x ^ w.y ^ w.z ^ w.w;
    }
    out[i] = acc;
}

}  // namespace

hipError_t launch_philox_bench(Key key, uint32_t t, uint32_t r, uint32_t tag, uint32_t n_threads, int per_thread,
                               uint32_t *out, hipStream_t s) {
    const unsigned blocks = (n_threads + kBenchBlock - 1) / kBenchBlock;
    SMC_LAUNCH(k_philox_bench, dim3(blocks), dim3(kBenchBlock), 0, s, key, t, r, tag, n_threads, per_thread,
                       out);
    return hipGetLastError();
}

}  // namespace smc

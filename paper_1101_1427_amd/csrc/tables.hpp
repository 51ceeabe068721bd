// Acceptance tables shared by the sweep kernels and the C-ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

// One row of the acceptance table: entry m (1..3) is the threshold of
// Delta E = 4m split as (hi, lo) = (thr >> 16, thr & 0xffff) with
// thr = floor(2^32 exp(-4 m beta)); entry 0 is unused.
struct ThrRow {
    uint2 m[4];
};

}  // namespace smc

// Host-side validation of a kernel launch configuration on gfx950, applied to
// every launch and graph kernel node the library issues, before it reaches
// the runtime.  Plain C++ (no HIP types) so that the check itself can be
// compiled and unit-tested on a machine without a GPU.
#pragma once
#include <stdint.h>

namespace smc {

constexpr uint64_t kMaxWorkgroup = 1024;           // work-items per workgroup
constexpr uint64_t kMaxLdsBytes = 160u * 1024u;    // LDS per workgroup (CDNA4)
constexpr uint64_t kMaxGridX = 0x7FFFFFFFull;      // workgroups along x

// nullptr if `grid` workgroups of `block` work-items with `lds` bytes of
// dynamic LDS are a configuration this library may launch, else a static
// description of the first limit it breaks: at least one workgroup, at most
// 2^31 - 1 of them, a workgroup of 1 .. 1024 work-items, dynamic LDS within
// the 160 KiB of a compute unit, and fewer than 2^32 work-items in the grid
// (the dispatch packet holds the grid size in work-items as a 32-bit word).
inline const char *launch_config_error(uint64_t grid, uint64_t block, uint64_t lds) {
    if (grid < 1) return "empty grid";
    if (grid > kMaxGridX) return "more than 2^31-1 workgroups";
    if (block < 1 || block > kMaxWorkgroup) return "workgroup size outside 1..1024";
    if (lds > kMaxLdsBytes) return "dynamic LDS above 160 KiB";
    if (grid * block >= (1ull << 32)) return "2^32 or more work-items in the grid";
    return nullptr;
}

}  // namespace smc

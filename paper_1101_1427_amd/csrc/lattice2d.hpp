// Large 2D Ising lattices on the colour-split layout (lattice2d.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "philox.hpp"
#include "tables.hpp"

namespace smc {

bool lattice2d_supported(int L);
size_t lattice2d_split_bytes(int L);  // bytes of one replica in the split layout
hipError_t launch_to_split(const int8_t *src, uint8_t *dst, int L, int n_rep, hipStream_t s);
hipError_t launch_from_split(const uint8_t *src, int8_t *dst, int L, int n_rep, hipStream_t s);
hipError_t launch_ising2d_split(const uint8_t *src, uint8_t *dst, int L, int n_rep, const ThrRow *thr, int64_t *dE,
                                Key key, uint32_t t, hipStream_t s);

}  // namespace smc

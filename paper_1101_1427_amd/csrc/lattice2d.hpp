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
int lattice2d_band_height(int L, int n_rep);  // rows per band of the next sweep of this batch
hipError_t launch_to_split(const int8_t *src, uint8_t *dst, int L, int n_rep, hipStream_t s);
hipError_t launch_from_split(const uint8_t *src, int8_t *dst, int L, int n_rep, hipStream_t s);
// One sweep from src to dst (distinct buffers).  Each is either the split
// layout (lattice2d_split_bytes per replica) or, with src_rows / dst_rows,
// the caller's row-major int8 +-1 lattice (L*L bytes per replica).  With
// dE_part != nullptr every compute wave writes (dE_first) or adds its share
// of the energy change to its own slot of dE_part (lattice2d_de_slots
// entries); launch_lattice2d_de_collect then adds each replica's slots to
// dE[r].
hipError_t launch_ising2d_split(const void *src, bool src_rows, void *dst, bool dst_rows, int L, int n_rep,
                                const ThrRow *thr, int64_t *dE_part, bool dE_first, Key key, uint32_t t,
                                hipStream_t s);
size_t lattice2d_de_slots(int L, int n_rep);
hipError_t launch_lattice2d_de_collect(const int64_t *part, int64_t *dE, int L, int n_rep, hipStream_t s);

}  // namespace smc

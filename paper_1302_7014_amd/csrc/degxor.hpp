// Degrees and edge-id XORs of a hypergraph, for the CSR-free k = 2 peel.
//
// For every vertex v < n: deg[v] = its number of incidences (a row listing v
// twice counts twice) and xr[v] = the XOR of the ids of its incident edges
// (with the same multiplicity).  Built by the same binned counting sort as
// hg_build, with the bucket kernel accumulating in LDS instead of placing the
// edge lists; for n > 2^26 by one device atomic per incidence.  Ids >= n set
// PEEL_FLAG_ERANGE in info[0] (info[0..1] zeroed by the caller).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "peel.h"

namespace peel {

size_t degxor_ws_bytes(uint32_t n, uint64_t m, uint32_t r);
peel_status degxor_build(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n, uint32_t *deg,
                         uint32_t *xr, uint32_t *info, void *ws, hipStream_t s);

}  // namespace peel

// Device-wide exclusive scan of a uint32 array, shared by the CSR build and
// the binned IBLT update.
#pragma once
#include "common.hpp"

namespace peel {
namespace {

constexpr int kScanItems = 8;                   // values per thread in the scans
constexpr int kScanTile = kBlock * kScanItems;  // 2048 values per workgroup

inline uint64_t scan_tiles(uint64_t count) { return (count + kScanTile - 1) / kScanTile; }

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of a uint32 array (three passes).

// part[b] = sum of in over tile b; pmax[b] (if given) = its maximum.
__global__ void __launch_bounds__(kBlock)
    k_scan_tiles(const uint32_t *__restrict__ in, uint64_t count, uint32_t *part, uint32_t *pmax) {
  __shared__ uint32_t lds[kBlock / kWave + 1];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t s = 0, mx = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < count) {
      const uint32_t d = in[base + i];
      s += d;
      mx = d > mx ? d : mx;
    }
  }
  const uint32_t tot = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
  if (pmax) {
    const uint32_t bmax = block_max(mx, lds);
    if (threadIdx.x == 0) pmax[blockIdx.x] = bmax;
  }
}

// Exclusive scan of part[0..tiles) in place (one workgroup); *total = the sum;
// *max_out (if given) = maximum of pmax.
__global__ void __launch_bounds__(kBlock)
    k_scan_parts(uint32_t *part, const uint32_t *pmax, uint64_t tiles, uint32_t *total,
                 uint32_t *max_out) {
  __shared__ uint32_t lds[kBlock / kWave + 1];
  if (max_out) {
    uint32_t mx = 0;
    for (uint64_t b = threadIdx.x; b < tiles; b += kBlock) mx = pmax[b] > mx ? pmax[b] : mx;
    mx = block_max(mx, lds);
    if (threadIdx.x == 0) *max_out = mx;
  }
  uint32_t carry = 0;
  for (uint64_t b0 = 0; b0 < tiles; b0 += (uint64_t)kBlock * kScanItems) {
    const uint64_t base = b0 + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      v[i] = (base + i < tiles) ? part[base + i] : 0u;
      s += v[i];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan(s, &tot, lds);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      if (base + i < tiles) part[base + i] = run;
      run += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// out[i] = part[tile] + prefix of in inside the tile; out2 (if given) gets a copy.
__global__ void __launch_bounds__(kBlock)
    k_scan_apply(const uint32_t *in, uint64_t count, const uint32_t *__restrict__ part,
                 uint32_t *out, uint32_t *out2) {
  __shared__ uint32_t lds[kBlock / kWave + 1];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < count) ? in[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = part[blockIdx.x] + block_exclusive_scan(s, &tot, lds);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < count) {
      out[base + i] = run;
      if (out2) out2[base + i] = run;
    }
    run += v[i];
  }
}

// Enqueues the exclusive scan of in[0..count) into out (may alias in).
void scan_u32(const uint32_t *in, uint64_t count, uint32_t *out, uint32_t *out2, uint32_t *part,
              uint32_t *pmax, uint32_t *total, uint32_t *max_out, hipStream_t s) {
  const uint64_t tiles = scan_tiles(count);
  if (tiles == 0) return;
  hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kBlock), 0, s, in, count, part, pmax);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBlock), 0, s, part, pmax, tiles, total, max_out);
  hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(kBlock), 0, s, in, count, part, out, out2);
}

}  // namespace
}  // namespace peel

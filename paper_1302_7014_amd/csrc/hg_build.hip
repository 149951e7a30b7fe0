// hg_build: vertex -> incident-edge lists (CSR) by counting sort.
//
// The peeling process removes each peeled vertex "together with its incident
// edges" (paper, Section 1), so the peel needs each vertex's edge list.  Three
// passes: degree histogram (one atomic per incidence), exclusive scan of the
// degrees into offsets, and scatter of edge ids through per-vertex cursors.
#include "common.hpp"
#include "host.hpp"

namespace peel {
namespace {

constexpr int kScanItems = 8;                      // degrees per thread in the scan
constexpr int kScanTile = kBlock * kScanItems;     // 2048 degrees per workgroup

struct BuildWs {
  uint32_t *cursor;  // n
  uint32_t *part;    // tiles: degree sum per tile, then its exclusive prefix
  uint32_t *pmax;    // tiles: maximum degree per tile
};

inline size_t scan_tiles(uint32_t n) { return (n + kScanTile - 1) / kScanTile; }

// deg[v] += 1 for every incidence; ids >= n raise PEEL_FLAG_ERANGE and are skipped.
template <int R>
__global__ void __launch_bounds__(kBlock)
    k_count(const uint32_t *__restrict__ edges, uint64_t m, uint32_t n, uint32_t *deg,
            uint32_t *info) {
  for (uint64_t e = blockIdx.x * (uint64_t)kBlock + threadIdx.x; e < m;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint32_t *row = edges + e * R;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint32_t v = row[j];
      if (v < n)
        atomicAdd(&deg[v], 1u);
      else
        atomicOr(&info[0], PEEL_FLAG_ERANGE);
    }
  }
}

// part[b] = sum of deg over tile b; pmax[b] = its maximum.
__global__ void __launch_bounds__(kBlock)
    k_tile_sums(const uint32_t *__restrict__ deg, uint32_t n, uint32_t *part, uint32_t *pmax) {
  __shared__ uint32_t lds[kBlock / kWave + 1];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t s = 0, mx = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const uint64_t v = base + i;
    if (v < n) {
      const uint32_t d = deg[v];
      s += d;
      mx = d > mx ? d : mx;
    }
  }
  const uint32_t tot = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
  const uint32_t bmax = block_max(mx, lds);
  if (threadIdx.x == 0) pmax[blockIdx.x] = bmax;
}

// Exclusive scan of part[0..tiles) in place by one workgroup; offsets[n] =
// total; info[1] = maximum of pmax.
__global__ void __launch_bounds__(kBlock)
    k_scan_parts(uint32_t *part, const uint32_t *pmax, uint64_t tiles, uint32_t *offsets,
                 uint32_t n, uint32_t *info) {
  __shared__ uint32_t lds[kBlock / kWave + 1];
  uint32_t carry = 0, mx = 0;
  for (uint64_t b = threadIdx.x; b < tiles; b += kBlock) mx = pmax[b] > mx ? pmax[b] : mx;
  mx = block_max(mx, lds);
  if (threadIdx.x == 0) info[1] = mx;
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
  if (threadIdx.x == 0) offsets[n] = carry;
}

// offsets[v] = part[tile] + prefix of deg inside the tile; cursor[v] = offsets[v].
__global__ void __launch_bounds__(kBlock)
    k_tile_scan(const uint32_t *__restrict__ deg, uint32_t n, const uint32_t *__restrict__ part,
                uint32_t *offsets, uint32_t *cursor) {
  __shared__ uint32_t lds[kBlock / kWave + 1];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? deg[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = part[blockIdx.x] + block_exclusive_scan(s, &tot, lds);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) {
      offsets[base + i] = run;
      cursor[base + i] = run;
    }
    run += v[i];
  }
}

// inc[cursor[v]++] = e for every incidence (e, v) with v < n.
template <int R>
__global__ void __launch_bounds__(kBlock)
    k_scatter(const uint32_t *__restrict__ edges, uint64_t m, uint32_t n, uint32_t *cursor,
              uint32_t *inc) {
  for (uint64_t e = blockIdx.x * (uint64_t)kBlock + threadIdx.x; e < m;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint32_t *row = edges + e * R;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint32_t v = row[j];
      if (v < n) {
        const uint32_t pos = atomicAdd(&cursor[v], 1u);
        inc[pos] = static_cast<uint32_t>(e);
      }
    }
  }
}

template <int R>
peel_status launch_edges(bool scatter, const uint32_t *edges, uint64_t m, uint32_t n,
                         uint32_t *a, uint32_t *b, hipStream_t s) {
  if (m == 0) return PEEL_OK;
  const unsigned grid = grid_for(m, kBlock, 1u << 16);
  if (scatter)
    hipLaunchKernelGGL(k_scatter<R>, dim3(grid), dim3(kBlock), 0, s, edges, m, n, a, b);
  else
    hipLaunchKernelGGL(k_count<R>, dim3(grid), dim3(kBlock), 0, s, edges, m, n, a, b);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

peel_status dispatch_edges(uint32_t r, bool scatter, const uint32_t *edges, uint64_t m,
                           uint32_t n, uint32_t *a, uint32_t *b, hipStream_t s) {
  switch (r) {
    case 2: return launch_edges<2>(scatter, edges, m, n, a, b, s);
    case 3: return launch_edges<3>(scatter, edges, m, n, a, b, s);
    case 4: return launch_edges<4>(scatter, edges, m, n, a, b, s);
    case 5: return launch_edges<5>(scatter, edges, m, n, a, b, s);
    case 6: return launch_edges<6>(scatter, edges, m, n, a, b, s);
    case 7: return launch_edges<7>(scatter, edges, m, n, a, b, s);
    case 8: return launch_edges<8>(scatter, edges, m, n, a, b, s);
    default: return PEEL_EINVAL;
  }
}

size_t build_ws_bytes(uint32_t n) {
  return align_up((size_t)n * 4) + 2 * align_up(scan_tiles(n) * 4) + 256;
}

}  // namespace
}  // namespace peel

using namespace peel;

extern "C" size_t hg_build_workspace(uint32_t n, uint64_t m, uint32_t r) {
  (void)m;
  (void)r;
  return build_ws_bytes(n);
}

extern "C" peel_status hg_build(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n,
                                uint32_t *offsets, uint32_t *inc, uint32_t *deg, uint32_t *info,
                                void *ws, size_t ws_bytes, void *stream) {
  if (r < 2 || r > 8 || n == 0) return PEEL_EINVAL;
  if (m * (uint64_t)r >= (1ull << 32)) return PEEL_EINVAL;
  if ((m && (!edges || !inc)) || !offsets || !deg || !info || !ws) return PEEL_EINVAL;
  if (ws_bytes < build_ws_bytes(n)) return PEEL_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  BuildWs w{c.take<uint32_t>(n), c.take<uint32_t>(scan_tiles(n)), c.take<uint32_t>(scan_tiles(n))};
  const uint64_t tiles = scan_tiles(n);

  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, kBlock * 4, 4096)), dim3(kBlock), 0, s,
                     deg, (uint64_t)n, 0u);
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(kBlock), 0, s, info, (uint64_t)2, 0u);
  PEEL_HIP_TRY(hipGetLastError());
  peel_status st = dispatch_edges(r, false, edges, m, n, deg, info, s);
  if (st) return st;
  hipLaunchKernelGGL(k_tile_sums, dim3(tiles), dim3(kBlock), 0, s, deg, n, w.part, w.pmax);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBlock), 0, s, w.part, w.pmax, tiles, offsets,
                     n, info);
  hipLaunchKernelGGL(k_tile_scan, dim3(tiles), dim3(kBlock), 0, s, deg, n, w.part, offsets,
                     w.cursor);
  PEEL_HIP_TRY(hipGetLastError());
  return dispatch_edges(r, true, edges, m, n, w.cursor, inc, s);
}

// hg_build: vertex -> incident-edge lists (CSR) by counting sort.
//
// The peeling process removes each peeled vertex "together with its incident
// edges" (paper, Section 1), so the peel needs each vertex's edge list.
//
// Device-scope atomics run at a fixed rate far below HBM bandwidth on this
// GPU, so the build keeps them out of the per-incidence work.  It is a
// three-level counting sort that keeps every write stream it opens short
// enough for L2 to fill whole lines:
//   1. bin count    each workgroup takes a tile of edges and counts, in LDS,
//                   its incidences per bucket of 8192 vertices (and so per
//                   super-bucket of 65536);
//   2. scans        exclusive scans of the (super-bucket, tile) counts and of
//                   the (bucket, tile) counts, both bucket-major: the second
//                   gives every (bucket, tile) run its final place;
//   3. bin scatter  each tile writes its (vertex, edge) pairs into its slice of
//                   every super-bucket: 8192 pairs at a time are sorted by
//                   super-bucket in LDS and stored as contiguous runs;
//   4. split        one workgroup per (super-bucket, group of tiles) moves its
//                   pairs to their (bucket, tile) runs (LDS cursors);
//   5. bucket build one workgroup per bucket counts degrees in LDS, scans them
//                   into offsets, places the edge ids with LDS cursors into an
//                   LDS copy of the bucket's lists and writes that out in one
//                   coalesced pass (a bucket too large for LDS is placed
//                   directly in device memory instead).
// Above 1024 super-buckets (n > 2^26) the LDS histograms do not fit and the
// build falls back to one device atomic per incidence for the degrees and
// another for the cursors.
#include "common.hpp"
#include "degxor.hpp"
#include "host.hpp"
#include "scan.hpp"

namespace peel {
namespace {

constexpr int kBinShift = 13;                   // 8192 vertices per bucket
constexpr int kBinV = 1 << kBinShift;
constexpr int kSupShift = 16;                   // 65536 vertices per super-bucket
constexpr int kSubPer = 1 << (kSupShift - kBinShift);  // buckets per super-bucket
constexpr int kMaxSuper = 1024;
constexpr int kSplitU = 8;                      // pairs per thread in flight in the split
constexpr int kSplitTiles = 32;                 // tiles per split workgroup
constexpr uint32_t kStageCap = 28672;           // incidences of a bucket staged in LDS
constexpr uint64_t kTileEdges = 16384;          // edges per bin tile
constexpr int kBT = 1024;                       // threads per workgroup in the bin kernels
constexpr int kRowsU = 4;                       // edge rows per thread in flight in the count
constexpr int kCT = 512;                        // threads per count workgroup: every tile resident at once
constexpr uint32_t kSortPairs = 8192;           // pairs sorted in LDS per scatter chunk
constexpr int kPairsU = 4;                      // pairs per thread in flight in the bucket build
constexpr uint32_t kNone = ~0u;
constexpr uint32_t kSort4 = 16384;              // 4-byte pairs sorted in LDS per flat-scatter chunk
constexpr uint32_t kMaxB4 = 2048;               // buckets of the flat scatter (n <= 2^24)
constexpr uint32_t kMaxTiles4 = 1024;           // tiles of the flat scatter (m <= 2^24)
constexpr uint32_t kBlk = 32;                   // places per entry of the bucket build's tile table

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
__device__ inline uint64_t ceil_div_dev(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline bool binned(uint32_t n) { return ceil_div(n, 1u << kSupShift) <= kMaxSuper; }

// ---------------------------------------------------------------------------
// Binned build.

// LDS index with one pad word per 32, so that a thread walking 64 consecutive
// counters does not hit the same bank as its neighbours.
__device__ inline uint32_t pad(uint32_t i) { return i + (i >> 5); }

// hist8[b * ntiles + tile] = incidences of this edge tile whose vertex is in bucket b;
// hist[s * ntiles + tile] = the same per super-bucket s.
template <int R>
__global__ void __launch_bounds__(kCT)
    k_bin_count(const uint32_t *__restrict__ edges, uint64_t m, uint32_t n, uint32_t nb,
                uint32_t nsb, uint64_t ntiles, uint32_t *hist, uint32_t *hist8, uint32_t *info) {
  __shared__ uint32_t h[kMaxSuper * kSubPer];
  for (uint32_t b = threadIdx.x; b < nsb * kSubPer; b += kCT) h[b] = 0;
  __syncthreads();
  const uint32_t tile = xcd_item(blockIdx.x, static_cast<uint32_t>(ntiles));
  const uint64_t e0 = (uint64_t)tile * kTileEdges;
  const uint64_t e1 = e0 + kTileEdges < m ? e0 + kTileEdges : m;
  bool bad = false;
  for (uint64_t eb = e0 + threadIdx.x; eb < e1; eb += kRowsU * kCT) {
    uint32_t ids[kRowsU][R];
#pragma unroll
    for (int u = 0; u < kRowsU; ++u) {
      const uint64_t e = eb + (uint64_t)u * kCT;
#pragma unroll
      for (int j = 0; j < R; ++j) ids[u][j] = e < e1 ? edges[e * R + j] : kNone;
    }
#pragma unroll
    for (int u = 0; u < kRowsU; ++u) {
      if (eb + (uint64_t)u * kCT >= e1) continue;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t v = ids[u][j];
        if (v < n)
          atomicAdd(&h[v >> kBinShift], 1u);
        else
          bad = true;
      }
    }
  }
  if (bad) atomicOr(&info[0], PEEL_FLAG_ERANGE);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nb; b += kCT) hist8[(uint64_t)b * ntiles + tile] = h[b];
  for (uint32_t sb = threadIdx.x; sb < nsb; sb += kCT) {
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < kSubPer; ++q) c += h[sb * kSubPer + q];
    hist[(uint64_t)sb * ntiles + tile] = c;
  }
}

// pairs[...] = (edge << 32 | vertex) grouped by super-bucket, each tile in its own
// slice of every super-bucket.  A tile is taken kSortPairs incidences at a time:
// they are ranked per super-bucket and sorted in LDS, then written out as one
// run per super-bucket, so neighbouring lanes store to neighbouring addresses.
template <int R>
__global__ void __launch_bounds__(kBT)
    k_bin_scatter(const uint32_t *__restrict__ edges, uint64_t m, uint32_t n, uint32_t nsb,
                  uint64_t ntiles, const uint32_t *__restrict__ hist, uint64_t *pairs) {
  constexpr uint32_t kCE = kSortPairs / R;            // edges per chunk
  constexpr int kEPT = (int)((kCE + kBT - 1) / kBT);  // edges per thread per chunk
  __shared__ uint64_t sp[kSortPairs];
  __shared__ uint32_t cur[kMaxSuper];  // next place of this tile in each super-bucket
  __shared__ uint32_t cnt[kMaxSuper];  // this chunk's pairs per super-bucket
  __shared__ uint32_t st[kMaxSuper];   // their exclusive scan
  __shared__ uint32_t lds[kBT / kWave + 1];
  const uint32_t tid = threadIdx.x;
  const uint32_t tile = xcd_item(blockIdx.x, static_cast<uint32_t>(ntiles));
  for (uint32_t b = tid; b < nsb; b += kBT) cur[b] = hist[(uint64_t)b * ntiles + tile];
  const uint64_t e0 = (uint64_t)tile * kTileEdges;
  const uint64_t e1 = e0 + kTileEdges < m ? e0 + kTileEdges : m;
  for (uint64_t c0 = e0; c0 < e1; c0 += kCE) {
    const uint64_t c1 = c0 + kCE < e1 ? c0 + kCE : e1;
    for (uint32_t b = tid; b < nsb; b += kBT) cnt[b] = 0;
    __syncthreads();
    uint32_t ids[kEPT][R], rk[kEPT][R];
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
      const uint64_t e = c0 + (uint64_t)u * kBT + tid;
#pragma unroll
      for (int j = 0; j < R; ++j) ids[u][j] = e < c1 ? edges[e * R + j] : kNone;
    }
#pragma unroll
    for (int u = 0; u < kEPT; ++u)
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (ids[u][j] < n) rk[u][j] = atomicAdd(&cnt[ids[u][j] >> kSupShift], 1u);
    __syncthreads();
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kBT>(tid < nsb ? cnt[tid] : 0u, &tot, lds);
    if (tid < nsb) st[tid] = ex;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
      const uint64_t e = c0 + (uint64_t)u * kBT + tid;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t v = ids[u][j];
        if (v < n) sp[st[v >> kSupShift] + rk[u][j]] = (e << 32) | v;
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < tot; i += kBT) {
      const uint64_t pr = sp[i];
      const uint32_t b = static_cast<uint32_t>(pr) >> kSupShift;
      pairs[cur[b] + (i - st[b])] = pr;
    }
    __syncthreads();
    for (uint32_t b = tid; b < nsb; b += kBT) cur[b] += cnt[b];
  }
}

// Up to 2048 buckets and 2048 tiles (n <= 2^24): each tile writes its pairs
// straight to their (bucket, tile) runs, whose starts are the scanned hist8,
// as 4-byte pairs (edge - e0) << kBinShift | (vertex - first vertex of the
// bucket), with e0 the tile's first edge.  kSort4 pairs at a time are ranked
// per bucket and sorted in LDS, then stored in sorted order, so neighbouring
// lanes store to neighbouring addresses within each run.
template <int R>
__global__ void __launch_bounds__(kBT)
    k_bin_scatter4(const uint32_t *__restrict__ edges, uint64_t m, uint32_t n, uint32_t nb,
                   uint64_t ntiles, const uint32_t *__restrict__ hist8, uint32_t *pairs) {
  constexpr int kEPT = (kSort4 / kBT) / R;            // edges per thread per chunk
  constexpr uint32_t kCE = (uint32_t)kEPT * kBT;      // edges per chunk: <= kSort4 pairs
  static_assert(kCE * R <= kSort4, "a chunk's pairs fit in LDS");
  __shared__ uint32_t sp[kSort4];
  __shared__ uint16_t sb[kSort4];   // the bucket of each sorted pair
  __shared__ uint32_t cur[kMaxB4];  // next place of this tile in each bucket
  __shared__ uint32_t cnt[kMaxB4];  // this chunk's pairs per bucket
  __shared__ uint32_t st[kMaxB4];   // their exclusive scan
  __shared__ uint32_t lds[kBT / kWave + 1];
  const uint32_t tid = threadIdx.x;
  const uint32_t tile = xcd_item(blockIdx.x, static_cast<uint32_t>(ntiles));
  for (uint32_t b = tid; b < nb; b += kBT) cur[b] = hist8[(uint64_t)b * ntiles + tile];
  const uint64_t e0 = (uint64_t)tile * kTileEdges;
  const uint64_t e1 = e0 + kTileEdges < m ? e0 + kTileEdges : m;
  for (uint64_t c0 = e0; c0 < e1; c0 += kCE) {
    const uint64_t c1 = c0 + kCE < e1 ? c0 + kCE : e1;
    for (uint32_t b = tid; b < nb; b += kBT) cnt[b] = 0;
    __syncthreads();
    uint32_t ids[kEPT][R], rk[kEPT][R];
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
      const uint64_t e = c0 + (uint64_t)u * kBT + tid;
#pragma unroll
      for (int j = 0; j < R; ++j) ids[u][j] = e < c1 ? edges[e * R + j] : kNone;
    }
#pragma unroll
    for (int u = 0; u < kEPT; ++u)
#pragma unroll
      for (int j = 0; j < R; ++j)
        if (ids[u][j] < n) rk[u][j] = atomicAdd(&cnt[ids[u][j] >> kBinShift], 1u);
    __syncthreads();
    // exclusive scan of cnt[0..nb), two buckets per thread
    const uint32_t b2 = 2 * tid;
    const uint32_t x0 = b2 < nb ? cnt[b2] : 0u, x1 = b2 + 1 < nb ? cnt[b2 + 1] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kBT>(x0 + x1, &tot, lds);
    if (b2 < nb) st[b2] = ex;
    if (b2 + 1 < nb) st[b2 + 1] = ex + x0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kEPT; ++u) {
      const uint32_t el = static_cast<uint32_t>(c0 - e0) + (uint32_t)u * kBT + tid;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t v = ids[u][j];
        if (v < n) {
          const uint32_t b = v >> kBinShift;
          const uint32_t i = st[b] + rk[u][j];
          sp[i] = (el << kBinShift) | (v & (uint32_t)(kBinV - 1));
          sb[i] = static_cast<uint16_t>(b);
        }
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < tot; i += kBT) {
      const uint32_t b = sb[i];
      pairs[cur[b] + (i - st[b])] = sp[i];
    }
    __syncthreads();
    for (uint32_t b = tid; b < nb; b += kBT) cur[b] += cnt[b];
  }
}

// One workgroup per (super-bucket sb, group of kSplitTiles tiles): the pairs of
// those tiles in sb's slice of pairs_in go to their (bucket, tile) runs in
// pairs_out, whose starts are the scanned hist8.  A pair's tile is its edge id's.
__global__ void __launch_bounds__(kBT)
    k_bin_split(const uint64_t *__restrict__ pairs_in, uint32_t nb, uint32_t nsb,
                uint64_t ntiles, const uint32_t *__restrict__ hist, const uint32_t *total,
                const uint32_t *__restrict__ hist8, uint64_t *pairs_out) {
  __shared__ uint32_t cur[kSubPer * kSplitTiles];
  const uint64_t ngroups = ceil_div_dev(ntiles, kSplitTiles);
  const uint32_t sb = static_cast<uint32_t>(blockIdx.x / ngroups);
  const uint64_t t0 = (blockIdx.x % ngroups) * kSplitTiles;
  const uint64_t t1 = t0 + kSplitTiles < ntiles ? t0 + kSplitTiles : ntiles;
  const uint32_t base = hist[(uint64_t)sb * ntiles + t0];
  const uint32_t end = t1 < ntiles                 ? hist[(uint64_t)sb * ntiles + t1]
                       : (sb + 1 < nsb)             ? hist[(uint64_t)(sb + 1) * ntiles]
                                                    : *total;
  const uint32_t b0 = sb * kSubPer;
  for (uint32_t i = threadIdx.x; i < (uint32_t)(kSubPer * kSplitTiles); i += kBT) {
    const uint32_t q = i / kSplitTiles, g = i % kSplitTiles;
    cur[i] = (b0 + q < nb && t0 + g < t1) ? hist8[(uint64_t)(b0 + q) * ntiles + t0 + g] : 0u;
  }
  __syncthreads();
  for (uint32_t p0 = base; p0 < end; p0 += kSplitU * kBT) {
    uint64_t pr[kSplitU];
#pragma unroll
    for (int u = 0; u < kSplitU; ++u) {
      const uint32_t p = p0 + u * kBT + threadIdx.x;
      pr[u] = p < end ? pairs_in[p] : ~0ull;
    }
#pragma unroll
    for (int u = 0; u < kSplitU; ++u) {
      if (pr[u] == ~0ull) continue;
      const uint32_t q = (static_cast<uint32_t>(pr[u]) >> kBinShift) - b0;
      const uint32_t g = static_cast<uint32_t>((pr[u] >> 32) / kTileEdges - t0);
      pairs_out[atomicAdd(&cur[q * kSplitTiles + g], 1u)] = pr[u];
    }
  }
}

// One workgroup per bucket: degrees, offsets and edge lists of its vertices.
// P = uint64_t: pairs are (edge << 32 | vertex).  P = uint32_t: pairs are
// (edge - first edge of its tile) << kBinShift | (vertex - first vertex of the
// bucket), and the bucket's runs are in tile order, so a pair's tile is the
// last tile whose run starts at or before the pair's place.
// XOR: degrees and, in place of the lists, the XOR of each vertex's incident
// edge ids (written to inc[v], n entries); offsets and maxdeg are not used.
template <typename P, bool XOR = false>
__global__ void __launch_bounds__(kBT)
    k_bin_build(const P *__restrict__ pairs, uint32_t n, uint32_t nb, uint64_t ntiles,
                const uint32_t *__restrict__ hist8, const uint32_t *total, uint32_t *offsets,
                uint32_t *inc, uint32_t *deg, uint32_t *maxdeg) {
  constexpr bool kP4 = sizeof(P) == 4;
  __shared__ uint32_t cnt[kBinV + kBinV / 32];
  __shared__ uint32_t stage[XOR ? kBinV : kStageCap];  // XOR: the bucket's edge-id XORs
  __shared__ uint32_t bnd[kP4 ? kMaxTiles4 + 1 : 1];           // start of each tile's run
  __shared__ uint16_t blk[kP4 ? kStageCap / kBlk : 1];         // tile of every kBlk-th place
  __shared__ uint32_t lds[kBT / kWave + 1];
  const uint32_t b = xcd_item(blockIdx.x, nb);
  const uint32_t base = hist8[(uint64_t)b * ntiles];
  const uint32_t end = (b + 1 < nb) ? hist8[(uint64_t)(b + 1) * ntiles] : *total;
  const uint32_t v0 = b << kBinShift;
  const uint32_t nv = (n - v0) < (uint32_t)kBinV ? (n - v0) : (uint32_t)kBinV;
  for (uint32_t i = threadIdx.x; i < (uint32_t)(kBinV + kBinV / 32); i += kBT) cnt[i] = 0;
  if constexpr (XOR)
    for (uint32_t i = threadIdx.x; i < (uint32_t)kBinV; i += kBT) stage[i] = 0;
  if (kP4) {
    for (uint32_t t = threadIdx.x; t < (uint32_t)ntiles; t += kBT) bnd[t] = hist8[(uint64_t)b * ntiles + t];
    if (threadIdx.x == 0) bnd[ntiles] = end;
  }
  __syncthreads();
  // the last tile whose run starts at or before place p (p in [base, end))
  auto tile_search = [&](uint32_t p) -> uint32_t {
    uint32_t lo = 0, hi = static_cast<uint32_t>(ntiles);
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (bnd[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
  };
  const bool staged = end - base <= kStageCap;
  if (kP4 && staged) {
    for (uint32_t j = threadIdx.x; j * kBlk < end - base; j += kBT)
      blk[j] = static_cast<uint16_t>(tile_search(base + j * kBlk));
  }
  auto vloc = [&](P x) -> uint32_t {
    if constexpr (kP4) return x & (uint32_t)(kBinV - 1);
    else return static_cast<uint32_t>(x) - v0;
  };
  auto edge = [&](uint32_t p, P x) -> uint32_t {
    if constexpr (kP4) {
      uint32_t t;
      if (staged) {
        t = blk[(p - base) / kBlk];
        while (bnd[t + 1] <= p) ++t;
      } else {
        t = tile_search(p);
      }
      return t * static_cast<uint32_t>(kTileEdges) + (x >> kBinShift);
    } else {
      return static_cast<uint32_t>(x >> 32);
    }
  };
  // f(place, pair) for every pair of [base, end), kPairsU loads per thread in
  // flight.  4-byte pairs are read 16 bytes at a time; the pair buffer is sized
  // for 8-byte pairs, so the vector holding the last pair stays inside it.
  auto for_pairs = [&](auto f) {
    if constexpr (kP4) {
      const uint4 *p4 = reinterpret_cast<const uint4 *>(pairs);
      const uint32_t q_lo = base / 4, q_hi = (end + 3) / 4;
      for (uint32_t q0 = q_lo + threadIdx.x; q0 < q_hi; q0 += kPairsU * kBT) {
        uint4 x[kPairsU];
#pragma unroll
        for (int u = 0; u < kPairsU; ++u) {
          const uint32_t q = q0 + u * kBT;
          if (q < q_hi) x[u] = p4[q];
        }
#pragma unroll
        for (int u = 0; u < kPairsU; ++u) {
          const uint32_t q = q0 + u * kBT;
          if (q >= q_hi) continue;
          const uint32_t w[4] = {x[u].x, x[u].y, x[u].z, x[u].w};
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const uint32_t p = 4 * q + c;
            if (p >= base && p < end) f(p, w[c]);
          }
        }
      }
    } else {
      for (uint32_t p0 = base + threadIdx.x; p0 < end; p0 += kPairsU * kBT) {
        P pr[kPairsU];
#pragma unroll
        for (int u = 0; u < kPairsU; ++u) {
          const uint32_t p = p0 + u * kBT;
          pr[u] = p < end ? pairs[p] : P(0);
        }
#pragma unroll
        for (int u = 0; u < kPairsU; ++u) {
          const uint32_t p = p0 + u * kBT;
          if (p < end) f(p, pr[u]);
        }
      }
    }
  };
  if constexpr (XOR) {
    __syncthreads();  // the tile table is complete before edge() reads it
    for_pairs([&](uint32_t p, P x) {
      const uint32_t v = vloc(x);
      atomicAdd(&cnt[pad(v)], 1u);
      atomicXor(&stage[v], edge(p, x));
    });
    __syncthreads();
    for (uint32_t v = threadIdx.x; v < nv; v += kBT) {
      deg[v0 + v] = cnt[pad(v)];
      inc[v0 + v] = stage[v];
    }
    return;
  }
  for_pairs([&](uint32_t, P x) { atomicAdd(&cnt[pad(vloc(x))], 1u); });
  __syncthreads();
  // exclusive scan of cnt[0..kBinV): kPer consecutive counts per thread
  constexpr int kPer = kBinV / kBT;
  const uint32_t i0 = threadIdx.x * kPer;
  uint32_t s = 0, mx = 0;
  for (int i = 0; i < kPer; ++i) {
    const uint32_t d = cnt[pad(i0 + i)];
    s += d;
    mx = d > mx ? d : mx;
  }
  uint32_t tot;
  uint32_t run = block_exclusive_scan<kBT>(s, &tot, lds);
  for (int i = 0; i < kPer; ++i) {
    const uint32_t v = i0 + i;
    const uint32_t d = cnt[pad(v)];
    if (v < nv) {
      offsets[v0 + v] = base + run;
      deg[v0 + v] = d;
    }
    cnt[pad(v)] = run;  // becomes the cursor
    run += d;
  }
  const uint32_t bmax = block_max<kBT>(mx, lds);
  if (threadIdx.x == 0) {
    if (bmax) atomicMax(maxdeg, bmax);  // *maxdeg starts at 0
    if (b == nb - 1) offsets[n] = end;
  }
  __syncthreads();
  const uint32_t total_b = end - base;
  if (staged) {
    for_pairs([&](uint32_t p, P x) {
      const uint32_t pos = atomicAdd(&cnt[pad(vloc(x))], 1u);
      stage[pos] = edge(p, x);
    });
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < total_b; i += kBT) inc[base + i] = stage[i];
  } else {
    for (uint32_t p = base + threadIdx.x; p < end; p += kBT) {
      const P pr = pairs[p];
      const uint32_t pos = atomicAdd(&cnt[pad(vloc(pr))], 1u);
      inc[base + pos] = edge(p, pr);
    }
  }
}

// ---------------------------------------------------------------------------
// Fallback for n > 2^26: one device atomic per incidence.

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

// ---------------------------------------------------------------------------
struct Sizes {
  uint64_t ntiles, nb, nsb, hist, hist8, pairs;
};

Sizes sizes(uint32_t n, uint64_t m, uint32_t r) {
  Sizes z{};
  if (binned(n)) {
    z.ntiles = ceil_div(m, kTileEdges);
    z.nb = ceil_div(n, kBinV);
    z.nsb = ceil_div(n, 1u << kSupShift);
    z.hist = (z.ntiles ? z.ntiles : 1) * z.nsb;
    z.hist8 = (z.ntiles ? z.ntiles : 1) * z.nb;
    z.pairs = m * r;
  } else {
    z.hist = (uint64_t)n + 1;  // degrees then cursors
  }
  return z;
}

size_t build_ws_bytes(uint32_t n, uint64_t m, uint32_t r) {
  const Sizes z = sizes(n, m, r);
  const uint64_t scan_n = z.hist8 > n ? z.hist8 : n;
  return align_up(z.hist * 4) + align_up(z.hist8 * 4) + 3 * align_up(scan_tiles(scan_n) * 4 + 4) +
         2 * align_up((z.pairs ? z.pairs : 1) * 8) + align_up((z.nb + 4) * 4) + 512;
}

template <int R, bool XOR = false>
peel_status build_binned(const uint32_t *edges, uint64_t m, uint32_t n, uint32_t *offsets,
                         uint32_t *inc, uint32_t *deg, uint32_t *info, Carver &c, hipStream_t s) {
  const Sizes z = sizes(n, m, R);
  uint32_t *hist = c.take<uint32_t>(z.hist);
  uint32_t *hist8 = c.take<uint32_t>(z.hist8);
  uint32_t *part = c.take<uint32_t>(scan_tiles(z.hist) + 1);
  uint32_t *part8 = c.take<uint32_t>(scan_tiles(z.hist8) + 1);
  uint64_t *pairs = c.take<uint64_t>(z.pairs ? z.pairs : 1);
  uint64_t *pairs2 = c.take<uint64_t>(z.pairs ? z.pairs : 1);
  uint32_t *sums = c.take<uint32_t>(z.nb + 4);
  uint32_t *total = sums + z.nb;      // pairs, from the super-bucket scan
  uint32_t *total8 = sums + z.nb + 1; // the same, from the bucket scan
  const bool flat = z.ntiles && z.nb <= kMaxB4 && z.ntiles <= kMaxTiles4;
  if (flat) {
    // two levels: tiles to (bucket, tile) runs of 4-byte pairs, then buckets
    hipLaunchKernelGGL(k_bin_count<R>, dim3(z.ntiles), dim3(kCT), 0, s, edges, m, n,
                       (uint32_t)z.nb, (uint32_t)z.nsb, z.ntiles, hist, hist8, info);
    scan_u32(hist8, z.hist8, hist8, nullptr, part8, nullptr, total8, nullptr, s);
    uint32_t *pairs4 = reinterpret_cast<uint32_t *>(pairs);
    hipLaunchKernelGGL(k_bin_scatter4<R>, dim3(z.ntiles), dim3(kBT), 0, s, edges, m, n,
                       (uint32_t)z.nb, z.ntiles, hist8, pairs4);
    hipLaunchKernelGGL((k_bin_build<uint32_t, XOR>), dim3(z.nb), dim3(kBT), 0, s, pairs4, n,
                       (uint32_t)z.nb, z.ntiles, hist8, total8, offsets, inc, deg, info + 1);
    PEEL_HIP_TRY(hipGetLastError());
    return PEEL_OK;
  }
  if (z.ntiles) {
    hipLaunchKernelGGL(k_bin_count<R>, dim3(z.ntiles), dim3(kCT), 0, s, edges, m, n,
                       (uint32_t)z.nb, (uint32_t)z.nsb, z.ntiles, hist, hist8, info);
    scan_u32(hist, z.hist, hist, nullptr, part, nullptr, total, nullptr, s);
    scan_u32(hist8, z.hist8, hist8, nullptr, part8, nullptr, total8, nullptr, s);
    hipLaunchKernelGGL(k_bin_scatter<R>, dim3(z.ntiles), dim3(kBT), 0, s, edges, m, n,
                       (uint32_t)z.nsb, z.ntiles, hist, pairs);
    const uint64_t groups = ceil_div(z.ntiles, kSplitTiles);
    hipLaunchKernelGGL(k_bin_split, dim3(z.nsb * groups), dim3(kBT), 0, s, pairs,
                       (uint32_t)z.nb, (uint32_t)z.nsb, z.ntiles, hist, total, hist8, pairs2);
  } else {
    // no edges: every bucket is empty
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(z.nb, kBlock, 4096)), dim3(kBlock), 0, s,
                       hist8, z.nb, 0u);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(kBlock), 0, s, total8, (uint64_t)1, 0u);
  }
  hipLaunchKernelGGL((k_bin_build<uint64_t, XOR>), dim3(z.nb), dim3(kBT), 0, s, pairs2, n, (uint32_t)z.nb,
                     z.ntiles ? z.ntiles : 1, hist8, total8, offsets, inc, deg, info + 1);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

template <int R>
peel_status build_atomic(const uint32_t *edges, uint64_t m, uint32_t n, uint32_t *offsets,
                         uint32_t *inc, uint32_t *deg, uint32_t *info, Carver &c, hipStream_t s) {
  uint32_t *cursor = c.take<uint32_t>((uint64_t)n + 1);
  uint32_t *part = c.take<uint32_t>(scan_tiles(n) + 1);
  uint32_t *pmax = c.take<uint32_t>(scan_tiles(n) + 1);
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, kBlock * 4, 4096)), dim3(kBlock), 0, s,
                     deg, (uint64_t)n, 0u);
  if (m) {
    hipLaunchKernelGGL(k_count<R>, dim3(grid_for(m, kBlock, 1u << 16)), dim3(kBlock), 0, s,
                       edges, m, n, deg, info);
  }
  scan_u32(deg, n, offsets, cursor, part, pmax, offsets + n, info + 1, s);
  if (m) {
    hipLaunchKernelGGL(k_scatter<R>, dim3(grid_for(m, kBlock, 1u << 16)), dim3(kBlock), 0, s,
                       edges, m, n, cursor, inc);
  }
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

template <int R>
peel_status build(const uint32_t *edges, uint64_t m, uint32_t n, uint32_t *offsets, uint32_t *inc,
                  uint32_t *deg, uint32_t *info, Carver &c, hipStream_t s) {
  return binned(n) ? build_binned<R>(edges, m, n, offsets, inc, deg, info, c, s)
                   : build_atomic<R>(edges, m, n, offsets, inc, deg, info, c, s);
}

// deg[v] += 1 and xr[v] ^= e for every incidence (e, v) with v < n (n > 2^26).
template <int R>
__global__ void __launch_bounds__(kBlock)
    k_count_xor(const uint32_t *__restrict__ edges, uint64_t m, uint32_t n, uint32_t *deg,
                uint32_t *xr, uint32_t *info) {
  for (uint64_t e = blockIdx.x * (uint64_t)kBlock + threadIdx.x; e < m;
       e += (uint64_t)gridDim.x * kBlock) {
    const uint32_t *row = edges + e * R;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint32_t v = row[j];
      if (v < n) {
        atomicAdd(&deg[v], 1u);
        atomicXor(&xr[v], static_cast<uint32_t>(e));
      } else {
        atomicOr(&info[0], PEEL_FLAG_ERANGE);
      }
    }
  }
}

template <int R>
peel_status degxor(const uint32_t *edges, uint64_t m, uint32_t n, uint32_t *deg, uint32_t *xr,
                   uint32_t *info, Carver &c, hipStream_t s) {
  if (binned(n)) return build_binned<R, true>(edges, m, n, nullptr, xr, deg, info, c, s);
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, kBlock * 4, 4096)), dim3(kBlock), 0, s,
                     deg, (uint64_t)n, 0u);
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, kBlock * 4, 4096)), dim3(kBlock), 0, s,
                     xr, (uint64_t)n, 0u);
  if (m)
    hipLaunchKernelGGL(k_count_xor<R>, dim3(grid_for(m, kBlock, 1u << 16)), dim3(kBlock), 0, s,
                       edges, m, n, deg, xr, info);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

}  // namespace

size_t degxor_ws_bytes(uint32_t n, uint64_t m, uint32_t r) { return build_ws_bytes(n, m, r); }

peel_status degxor_build(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n, uint32_t *deg,
                         uint32_t *xr, uint32_t *info, void *ws, hipStream_t s) {
  Carver c(ws);
  switch (r) {
    case 2: return degxor<2>(edges, m, n, deg, xr, info, c, s);
    case 3: return degxor<3>(edges, m, n, deg, xr, info, c, s);
    case 4: return degxor<4>(edges, m, n, deg, xr, info, c, s);
    case 5: return degxor<5>(edges, m, n, deg, xr, info, c, s);
    case 6: return degxor<6>(edges, m, n, deg, xr, info, c, s);
    case 7: return degxor<7>(edges, m, n, deg, xr, info, c, s);
    default: return degxor<8>(edges, m, n, deg, xr, info, c, s);
  }
}

}  // namespace peel

using namespace peel;

extern "C" size_t hg_build_workspace(uint32_t n, uint64_t m, uint32_t r) {
  return build_ws_bytes(n, m, r);
}

extern "C" peel_status hg_build(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n,
                                uint32_t *offsets, uint32_t *inc, uint32_t *deg, uint32_t *info,
                                void *ws, size_t ws_bytes, void *stream) {
  if (r < 2 || r > 8 || n == 0) return PEEL_EINVAL;
  if (m * (uint64_t)r >= (1ull << 32)) return PEEL_EINVAL;
  if ((m && (!edges || !inc)) || !offsets || !deg || !info || !ws) return PEEL_EINVAL;
  if (ws_bytes < build_ws_bytes(n, m, r)) return PEEL_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(kBlock), 0, s, info, (uint64_t)2, 0u);
  PEEL_HIP_TRY(hipGetLastError());
  switch (r) {
    case 2: return build<2>(edges, m, n, offsets, inc, deg, info, c, s);
    case 3: return build<3>(edges, m, n, offsets, inc, deg, info, c, s);
    case 4: return build<4>(edges, m, n, offsets, inc, deg, info, c, s);
    case 5: return build<5>(edges, m, n, offsets, inc, deg, info, c, s);
    case 6: return build<6>(edges, m, n, offsets, inc, deg, info, c, s);
    case 7: return build<7>(edges, m, n, offsets, inc, deg, info, c, s);
    default: return build<8>(edges, m, n, offsets, inc, deg, info, c, s);
  }
}

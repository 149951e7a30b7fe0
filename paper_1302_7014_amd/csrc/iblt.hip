// IBLT insert and round-synchronous listing (paper, Section 5).
//
// Insert: one lane per key; the key is XORed into the key field and its
// checksum into the checksum field of its r cells, one per subtable, with
// device-scope atomics (several keys may share a cell), and the cell's count
// moves by one ("Implementation Details").
//
// List: the table is a hypergraph whose vertices are cells and whose edges are
// keys; a pure cell is a vertex of degree 1, and each round lists every key
// that has a pure cell at the start of the round, then deletes it from its r
// cells.  A key pure in several cells must be listed once; instead of the
// paper's r serial subrounds per round (Appendix B), ownership decides: the
// key's pure cell in the lowest-numbered subtable lists it.  Each round runs
// in two phases separated by device-wide barriers, because ownership must
// read the cells as they were at the start of the round:
//   detect  for each candidate cell that is pure, check the key's cells in
//           the lower subtables; if none of them is a pure cell of the same
//           key, append the key to out_keys (block prefix + one atomic);
//   apply   for each key listed this round, delete it from its r cells
//           (atomic count decrement and 64-bit XORs); a cell whose count goes
//           2 -> 1 becomes a candidate for the next round.
// Round 1's candidates are all cells (one dense pass, which also sums the
// counts).  Every cell pure at the start of round t+1 went 2 -> 1 during
// round t, so the candidate lists miss none.
#include "common.hpp"
#include "host.hpp"

namespace peel {
namespace {

#ifndef PEEL_LDS_QUEUE
#define PEEL_LDS_QUEUE 4096
#endif
constexpr int kQueue = PEEL_LDS_QUEUE;
constexpr int kDenseItems = 4;  // cells per thread in the dense pass
constexpr int kDenseTile = kBlock * kDenseItems;

struct Hash {
  uint64_t base[8];
  uint64_t size[8];
  uint64_t salt[8];
  uint64_t salt_c;
  uint32_t r;
};

Hash make_hash(const iblt_desc &d) {
  Hash h{};
  uint64_t acc = 0;
  h.r = d.r;
  for (uint32_t j = 0; j < d.r; ++j) {
    h.size[j] = d.ncells / d.r + (j < d.ncells % d.r ? 1 : 0);
    h.base[j] = acc;
    acc += h.size[j];
    h.salt[j] = splitmix64(d.seed, j);
  }
  h.salt_c = splitmix64(d.seed, 8);
  return h;
}

__device__ inline uint32_t cell_of(const Hash &h, uint32_t j, uint64_t x) {
  return static_cast<uint32_t>(h.base[j] + mulhi64(mix64(x ^ h.salt[j]), h.size[j]));
}

__device__ inline uint64_t check_of(const Hash &h, uint64_t x) { return mix64(x ^ h.salt_c); }

__device__ inline uint32_t subtable_of(const Hash &h, uint32_t c) {
  uint32_t j = 0;
#pragma unroll
  for (int i = 1; i < 8; ++i)
    if (i < (int)h.r && c >= h.base[i]) j = i;
  return j;
}

// ---------------------------------------------------------------------------
template <int R>
__global__ void __launch_bounds__(kBlock)
    k_insert(Hash h, iblt_cell *cells, const uint64_t *__restrict__ keys, uint64_t nkeys) {
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < nkeys;
       i += (uint64_t)gridDim.x * kBlock) {
    const uint64_t x = keys[i];
    const uint64_t c = check_of(h, x);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      iblt_cell *cell = cells + cell_of(h, j, x);
      atomicAdd(&cell->count, 1);
      atomicXor(reinterpret_cast<unsigned long long *>(&cell->key_sum), (unsigned long long)x);
      atomicXor(reinterpret_cast<unsigned long long *>(&cell->hash_sum), (unsigned long long)c);
    }
  }
}

// ---------------------------------------------------------------------------
struct ListCtrl {
  GridSync sync;
  Team team;
  uint32_t own[3];   // keys owned in the detect phase feeding round t: own[t % 3]
  uint32_t cand[2];  // candidates pushed in round t: cand[t % 2]
  uint32_t flags;
  uint32_t rounds;
  uint64_t listed;
  unsigned long long count_sum;  // sum of all counts at the start (two's complement)
  uint64_t stamp[256];           // wall clock at each barrier generation (diagnostic)
};

struct ListArgs {
  Hash h;
  iblt_cell *cells;
  uint64_t *out;
  uint64_t out_cap;
  uint64_t *stats;
  uint32_t *ca;  // candidate lists
  uint32_t *cb;
  ListCtrl *ctrl;
  uint64_t limit;
  uint64_t quiet;
  uint32_t ncells;
  uint32_t max_rounds;
};

__global__ void k_list_init(ListCtrl *ctrl) {
  if (threadIdx.x == 0) {
    ctrl->sync.count = ctrl->sync.gen = ctrl->sync.abort = ctrl->sync.pad = 0;
    ctrl->team.join = ctrl->team.size = 0;
    ctrl->own[0] = ctrl->own[1] = ctrl->own[2] = 0;
    ctrl->cand[0] = ctrl->cand[1] = 0;
    ctrl->flags = 0;
    ctrl->rounds = 0;
    ctrl->listed = 0;
    ctrl->count_sum = 0;
  }
}

// True when cell c (already read as cnt/ks/hs) is pure and it is the owner of
// its key: no cell of the key in a lower subtable is a pure cell of that key.
template <int R>
__device__ inline bool owns(const ListArgs &a, uint32_t c, int32_t cnt, uint64_t ks, uint64_t hs,
                            uint32_t *flags_bad) {
  if (cnt != 1) return false;
  const uint64_t hx = check_of(a.h, ks);
  if (hs != hx) {
    *flags_bad = 1;
    return false;
  }
  const uint32_t j = subtable_of(a.h, c);
#pragma unroll
  for (int i = 0; i < R - 1; ++i) {
    if (i >= (int)j) break;
    const iblt_cell *o = a.cells + cell_of(a.h, i, ks);
    if (o->count == 1 && o->key_sum == ks && o->hash_sum == hx) return false;
  }
  return true;
}

// Appends `x` (when take) to out[listed_base + ...] with one global atomic per workgroup.
__device__ inline void append_owned(const ListArgs &a, uint32_t *own_ctr, uint64_t listed_base,
                                    bool take, uint64_t x, uint32_t *lds, uint32_t *s_base) {
  uint32_t tot;
  const uint32_t off = block_exclusive_scan(take ? 1u : 0u, &tot, lds);
  if (threadIdx.x == 0) *s_base = tot ? atomicAdd(own_ctr, tot) : 0u;
  __syncthreads();
  if (take) {
    const uint64_t pos = listed_base + *s_base + off;
    if (pos < a.out_cap)
      a.out[pos] = x;
    else
      atomicOr(&a.ctrl->flags, PEEL_FLAG_ENOSPC);
  }
  __syncthreads();
}

template <int R>
__global__ void __launch_bounds__(kBlock) k_list_persistent(ListArgs a) {
  __shared__ uint32_t q[kQueue];
  __shared__ uint32_t qn;
  __shared__ uint32_t s_base;
  __shared__ uint32_t lds[kBlock / kWave + 1];
  __shared__ unsigned long long s_sum;

  ListCtrl *ctrl = a.ctrl;
  uint32_t slot, nblocks;
  if (!team_join(&ctrl->team, a.quiet, a.limit, &slot, &nblocks)) return;
  const uint64_t gtid = (uint64_t)slot * kBlock + threadIdx.x;
  const uint64_t gsize = (uint64_t)nblocks * kBlock;
  uint32_t bad = 0;

  // ---- round-1 detect over every cell -------------------------------------
  for (uint64_t i = gtid; i < a.max_rounds; i += gsize) a.stats[i] = 0;
  if (threadIdx.x == 0) s_sum = 0;
  __syncthreads();
  long long local_sum = 0;
  for (uint64_t t0 = (uint64_t)slot * kDenseTile; t0 < a.ncells;
       t0 += (uint64_t)nblocks * kDenseTile) {
#pragma unroll
    for (int it = 0; it < kDenseItems; ++it) {
      const uint64_t c = t0 + (uint64_t)it * kBlock + threadIdx.x;
      bool take = false;
      uint64_t x = 0;
      if (c < a.ncells) {
        const iblt_cell cell = a.cells[c];
        local_sum += cell.count;
        take = owns<R>(a, static_cast<uint32_t>(c), cell.count, cell.key_sum, cell.hash_sum, &bad);
        x = cell.key_sum;
      }
      append_owned(a, &ctrl->own[1], 0, take, x, lds, &s_base);
    }
  }
  atomicAdd(&s_sum, (unsigned long long)local_sum);
  __syncthreads();
  if (threadIdx.x == 0 && s_sum) atomicAdd(&ctrl->count_sum, s_sum);
  if (bad) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
  bad = 0;
  if (!grid_barrier(&ctrl->sync, nblocks, a.limit, ctrl->stamp)) return;

  // ---- rounds ---------------------------------------------------------------
  uint64_t listed = 0;
  uint32_t t = 1;
  for (;; ++t) {
    const uint32_t K = atomic_load_u32(&ctrl->own[t % 3]);
    const uint32_t flags = atomic_load_u32(&ctrl->flags);
    if (K == 0) break;
    if (t > a.max_rounds) {
      if (gtid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_EROUNDS);
      break;
    }
    if (flags & PEEL_FLAG_ENOSPC) break;
    uint32_t *cand = (t & 1u) ? a.ca : a.cb;
    uint32_t *cctr = &ctrl->cand[t % 2];
    if (gtid == 0) {
      a.stats[t - 1] = K;
      ctrl->own[(t + 2) % 3] = 0;
      ctrl->cand[(t + 1) % 2] = 0;
    }
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();

    // apply: delete every key listed this round from its r cells
    for (uint64_t i = gtid; i < K; i += gsize) {
      const uint64_t x = a.out[listed + i];
      const uint64_t hx = check_of(a.h, x);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t c = cell_of(a.h, j, x);
        iblt_cell *cell = a.cells + c;
        const int32_t old = atomicSub(&cell->count, 1);
        atomicXor(reinterpret_cast<unsigned long long *>(&cell->key_sum), (unsigned long long)x);
        atomicXor(reinterpret_cast<unsigned long long *>(&cell->hash_sum), (unsigned long long)hx);
        if (old == 2) {
          const uint32_t slot = atomicAdd(&qn, 1u);
          if (slot < kQueue)
            q[slot] = c;
          else
            cand[atomicAdd(cctr, 1u)] = c;
        }
      }
    }
    __syncthreads();
    const uint32_t nq = qn < kQueue ? qn : kQueue;
    if (threadIdx.x == 0) s_base = nq ? atomicAdd(cctr, nq) : 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nq; i += kBlock) cand[s_base + i] = q[i];
    if (!grid_barrier(&ctrl->sync, nblocks, a.limit, ctrl->stamp)) return;

    // detect for round t+1 over this round's candidates
    listed += K;
    const uint32_t nc = atomic_load_u32(cctr);
    const uint64_t span = (nc + gsize - 1) / gsize * gsize;  // uniform trip count
    for (uint64_t i = gtid; i < span; i += gsize) {
      bool take = false;
      uint64_t x = 0;
      if (i < nc) {
        const uint32_t c = cand[i];
        const iblt_cell cell = a.cells[c];
        take = owns<R>(a, c, cell.count, cell.key_sum, cell.hash_sum, &bad);
        x = cell.key_sum;
      }
      append_owned(a, &ctrl->own[(t + 1) % 3], listed, take, x, lds, &s_base);
    }
    if (bad) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
    bad = 0;
    if (!grid_barrier(&ctrl->sync, nblocks, a.limit, ctrl->stamp)) return;
  }
  if (gtid == 0) {
    ctrl->rounds = t - 1 < a.max_rounds ? t - 1 : a.max_rounds;
    ctrl->listed = listed;
  }
}

// summary = [listed, rounds, keys left, flags, workgroups in the persistent team, 0, 0, 0].
__global__ void k_list_finish(const ListCtrl *ctrl, uint32_t r, uint64_t *summary) {
  if (threadIdx.x != 0) return;
  const long long total = (long long)ctrl->count_sum;
  const long long keys = total / (long long)r;
  uint32_t flags = ctrl->flags;
  if (ctrl->sync.abort) flags |= PEEL_FLAG_TIMEOUT;
  summary[0] = ctrl->listed;
  summary[1] = ctrl->rounds;
  summary[2] = (uint64_t)(keys - (long long)ctrl->listed);
  summary[3] = flags;
  summary[4] = ctrl->team.size;
  summary[5] = summary[6] = summary[7] = 0;
}

size_t list_ws_bytes(uint64_t ncells) {
  return align_up(sizeof(ListCtrl)) + 2 * align_up((size_t)ncells * 4);
}

bool desc_ok(const iblt_desc *d) {
  return d && d->r >= 2 && d->r <= 8 && d->ncells >= d->r && d->ncells < (1ull << 32);
}

template <int R>
peel_status launch_insert(const Hash &h, iblt_cell *cells, const uint64_t *keys, uint64_t nkeys,
                          hipStream_t s) {
  const unsigned grid = grid_for(nkeys, kBlock, 1u << 16);
  hipLaunchKernelGGL(k_insert<R>, dim3(grid), dim3(kBlock), 0, s, h, cells, keys, nkeys);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

template <int R>
peel_status launch_list(ListArgs &a, hipStream_t s) {
  const void *fn = reinterpret_cast<const void *>(&k_list_persistent<R>);
  const int cap = coresident_blocks(fn, kBlock, 0);
  uint64_t want = ((uint64_t)a.ncells + kDenseTile - 1) / kDenseTile;
  if (want < 1) want = 1;
  const unsigned grid = static_cast<unsigned>(want < (uint64_t)cap ? want : (uint64_t)cap);
  if (device_info().debug) std::fprintf(stderr, "[peel] persistent grid %u (cap %d)\n", grid, cap);
  // A plain launch: the kernel forms its team of resident workgroups itself.
  hipLaunchKernelGGL(k_list_persistent<R>, dim3(grid), dim3(kBlock), 0, s, a);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

}  // namespace
}  // namespace peel

using namespace peel;

extern "C" peel_status iblt_insert(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                                   uint64_t nkeys, void *stream) {
  if (!desc_ok(desc) || !cells || (nkeys && !keys)) return PEEL_EINVAL;
  if (nkeys == 0) return PEEL_OK;
  const Hash h = make_hash(*desc);
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (desc->r) {
    case 2: return launch_insert<2>(h, cells, keys, nkeys, s);
    case 3: return launch_insert<3>(h, cells, keys, nkeys, s);
    case 4: return launch_insert<4>(h, cells, keys, nkeys, s);
    case 5: return launch_insert<5>(h, cells, keys, nkeys, s);
    case 6: return launch_insert<6>(h, cells, keys, nkeys, s);
    case 7: return launch_insert<7>(h, cells, keys, nkeys, s);
    default: return launch_insert<8>(h, cells, keys, nkeys, s);
  }
}

extern "C" size_t iblt_list_workspace(const iblt_desc *desc) {
  return desc_ok(desc) ? list_ws_bytes(desc->ncells) : 0;
}

extern "C" peel_status iblt_list(const iblt_desc *desc, iblt_cell *cells, uint64_t *out_keys,
                                 uint64_t out_cap, uint64_t *round_stats, uint32_t max_rounds,
                                 uint64_t *summary, void *ws, size_t ws_bytes, void *stream) {
  if (!desc_ok(desc) || !cells || (out_cap && !out_keys) || !round_stats || !summary || !ws ||
      max_rounds == 0)
    return PEEL_EINVAL;
  if (ws_bytes < list_ws_bytes(desc->ncells)) return PEEL_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  ListArgs a;
  a.h = make_hash(*desc);
  a.ctrl = c.take<ListCtrl>(1);
  a.ca = c.take<uint32_t>(desc->ncells);
  a.cb = c.take<uint32_t>(desc->ncells);
  a.cells = cells;
  a.out = out_keys;
  a.out_cap = out_cap;
  a.stats = round_stats;
  a.limit = device_info().barrier_limit_ticks;
  a.quiet = device_info().team_quiet_ticks;
  a.ncells = static_cast<uint32_t>(desc->ncells);
  a.max_rounds = max_rounds;
  hipLaunchKernelGGL(k_list_init, dim3(1), dim3(64), 0, s, a.ctrl);
  PEEL_HIP_TRY(hipGetLastError());
  peel_status st;
  switch (desc->r) {
    case 2: st = launch_list<2>(a, s); break;
    case 3: st = launch_list<3>(a, s); break;
    case 4: st = launch_list<4>(a, s); break;
    case 5: st = launch_list<5>(a, s); break;
    case 6: st = launch_list<6>(a, s); break;
    case 7: st = launch_list<7>(a, s); break;
    default: st = launch_list<8>(a, s); break;
  }
  if (st) return st;
  hipLaunchKernelGGL(k_list_finish, dim3(1), dim3(64), 0, s, a.ctrl, desc->r, summary);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

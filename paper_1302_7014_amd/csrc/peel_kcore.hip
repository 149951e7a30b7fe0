// peel_kcore: round-synchronous parallel peeling to the k-core.
//
// Paper, Section 1 and Section 3: in round t every vertex whose degree is
// below k at the start of the round is removed at once, together with every
// edge still holding it; the run ends at the first round with nothing to
// remove.  Section 5 ("Implementation Details") notes that a parallel peel
// must never peel one edge twice; here the edge's round word is claimed by
// compare-and-swap (0 -> t), so exactly one of the peeled vertices that share
// an edge removes it.
//
// One persistent kernel (a run-time team of resident workgroups) runs every round, with a
// device-wide barrier between rounds and no host round trip:
//   phase 0   dense pass: zero edge rounds and stats, mark vertex_round = 1 and
//             compact F_1 = {v : deg(v) < k} (block prefix sum, one atomic per
//             2048-vertex tile, so F_1 comes out in ascending tiles);
//   round t   for v in F_t and each incidence e of v still alive: CAS the
//             edge's round word 0 -> t; the winner lowers the degree of each of
//             e's r slots.  A decrement that takes a degree from k to k-1
//             marks that vertex for round t+1 (vertex_round = t+1) and pushes
//             it onto F_{t+1} through a per-workgroup LDS queue.
//
// Why this is exact: a vertex alive at the start of round t with degree >= k
// crosses k -> k-1 at most once, so F_{t+1} is exactly the set of alive
// vertices whose degree dropped below k during round t; vertices of F_t start
// below k and never trigger a push.  Every slot of a removed edge is
// decremented, so removed vertices end at degree 0 and core vertices at their
// core degree, independent of which thread wins a CAS.
#include "common.hpp"
#include "host.hpp"

namespace peel {
namespace {

#ifndef PEEL_LDS_QUEUE
#define PEEL_LDS_QUEUE 4096
#endif
constexpr int kQueue = PEEL_LDS_QUEUE;          // LDS push-queue entries per workgroup
constexpr int kDenseItems = 8;        // vertices per thread in the dense pass
constexpr int kDenseTile = kBlock * kDenseItems;

struct PeelCtrl {
  GridSync sync;
  Team team;
  uint32_t fcount[3];  // |F_t| lives in fcount[t % 3]
  uint32_t flags;
  uint32_t rounds;
  uint32_t pad;
  uint64_t removed;
  uint64_t stamp[256];  // wall clock at each barrier generation (diagnostic)
};

struct PeelArgs {
  const uint32_t *edges;
  const uint32_t *offsets;
  const uint32_t *inc;
  uint32_t *deg;
  uint32_t *vr;
  uint32_t *er;
  uint64_t *stats;
  uint32_t *fa;
  uint32_t *fb;
  PeelCtrl *ctrl;
  uint64_t m;
  uint64_t limit;
  uint64_t quiet;
  uint32_t n;
  uint32_t k;
  uint32_t max_rounds;
};

__global__ void k_peel_init(PeelCtrl *ctrl) {
  if (threadIdx.x == 0) {
    ctrl->sync.count = 0;
    ctrl->sync.gen = 0;
    ctrl->sync.abort = 0;
    ctrl->sync.pad = 0;
    ctrl->team.join = 0;
    ctrl->team.size = 0;
    ctrl->fcount[0] = ctrl->fcount[1] = ctrl->fcount[2] = 0;
    ctrl->flags = 0;
    ctrl->rounds = 0;
    ctrl->pad = 0;
    ctrl->removed = 0;
  }
}

template <int R>
__global__ void __launch_bounds__(kBlock) k_peel_persistent(PeelArgs a) {
  __shared__ uint32_t q[kQueue];
  __shared__ uint32_t qn;
  __shared__ uint32_t s_base;
  __shared__ uint32_t lds[kBlock / kWave + 1];

  PeelCtrl *ctrl = a.ctrl;
  uint32_t slot, nblocks;
  if (!team_join(&ctrl->team, a.quiet, a.limit, &slot, &nblocks)) return;
  const uint64_t gtid = (uint64_t)slot * kBlock + threadIdx.x;
  const uint64_t gsize = (uint64_t)nblocks * kBlock;

  // ---- phase 0 ------------------------------------------------------------
  for (uint64_t e = gtid; e < a.m; e += gsize) a.er[e] = 0;
  for (uint64_t i = gtid; i < 2ull * a.max_rounds; i += gsize) a.stats[i] = 0;
  for (uint64_t t0 = (uint64_t)slot * kDenseTile; t0 < a.n;
       t0 += (uint64_t)nblocks * kDenseTile) {
    const uint64_t base = t0 + (uint64_t)threadIdx.x * kDenseItems;
    uint32_t low = 0, cnt = 0;
#pragma unroll
    for (int i = 0; i < kDenseItems; ++i) {
      const uint64_t v = base + i;
      if (v < a.n) {
        const uint32_t is_low = a.deg[v] < a.k ? 1u : 0u;
        a.vr[v] = is_low;
        low |= is_low << i;
        cnt += is_low;
      }
    }
    uint32_t tot;
    const uint32_t off = block_exclusive_scan(cnt, &tot, lds);
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(&ctrl->fcount[1], tot) : 0u;
    __syncthreads();
    uint32_t pos = s_base + off;
#pragma unroll
    for (int i = 0; i < kDenseItems; ++i)
      if (low >> i & 1u) a.fa[pos++] = static_cast<uint32_t>(base + i);
    __syncthreads();
  }
  if (!grid_barrier(&ctrl->sync, nblocks, a.limit, ctrl->stamp)) return;

  // ---- rounds -------------------------------------------------------------
  uint32_t t = 1;
  uint64_t removed = 0;
  for (;; ++t) {
    const uint32_t size = atomic_load_u32(&ctrl->fcount[t % 3]);
    const uint32_t *cur = (t & 1u) ? a.fa : a.fb;
    if (size == 0) break;
    if (t > a.max_rounds) {
      // Leave the state after max_rounds rounds: F_t stays in the graph.
      for (uint64_t i = gtid; i < size; i += gsize) a.vr[cur[i]] = 0;
      if (gtid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_EROUNDS);
      break;
    }
    removed += size;
    uint32_t *nxt = (t & 1u) ? a.fb : a.fa;
    uint32_t *ncount = &ctrl->fcount[(t + 1) % 3];
    if (gtid == 0) {
      a.stats[2ull * (t - 1)] = size;
      ctrl->fcount[(t + 2) % 3] = 0;
    }
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();

    uint32_t wins = 0;
    for (uint64_t i = gtid; i < size; i += gsize) {
      const uint32_t v = cur[i];
      const uint32_t beg = a.offsets[v];
      const uint32_t end = a.offsets[v + 1];
      for (uint32_t p = beg; p < end; ++p) {
        const uint32_t e = a.inc[p];
        // A plain read may be stale only towards 0 (a claim it has not seen yet);
        // the compare-and-swap below settles those.
        if (e >= a.m || a.er[e] != 0u) continue;
        if (atomicCAS(&a.er[e], 0u, t) != 0u) continue;
        ++wins;
        const uint32_t *row = a.edges + (uint64_t)e * R;
        uint32_t ids[R];
#pragma unroll
        for (int j = 0; j < R; ++j) ids[j] = row[j];
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t u = ids[j];
          if (u >= a.n) continue;  // ids >= n are reported by hg_build and skipped here
          const uint32_t old = atomicSub(&a.deg[u], 1u);
          if (old == a.k) {
            a.vr[u] = t + 1;
            const uint32_t slot = atomicAdd(&qn, 1u);
            if (slot < kQueue) {
              q[slot] = u;
            } else {
              nxt[atomicAdd(ncount, 1u)] = u;
            }
          }
        }
      }
    }
    __syncthreads();
    const uint32_t nq = qn < kQueue ? qn : kQueue;
    if (threadIdx.x == 0) s_base = nq ? atomicAdd(ncount, nq) : 0u;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nq; i += kBlock) nxt[s_base + i] = q[i];
    const uint32_t bw = block_sum(wins, lds);
    if (threadIdx.x == 0 && bw) atomicAdd(&a.stats[2ull * (t - 1) + 1], (uint64_t)bw);
    if (!grid_barrier(&ctrl->sync, nblocks, a.limit, ctrl->stamp)) return;
  }
  if (gtid == 0) {
    ctrl->rounds = t - 1 < a.max_rounds ? t - 1 : a.max_rounds;
    ctrl->removed = removed;
  }
}

// summary = [rounds, last round that removed an edge, flags, core vertices,
//            workgroups in the persistent team, 0, 0, 0].
__global__ void k_peel_finish(const PeelCtrl *ctrl, const uint64_t *stats, uint32_t n,
                              uint32_t *summary) {
  if (threadIdx.x != 0) return;
  const uint32_t rounds = ctrl->rounds;
  uint32_t last_e = 0;
  for (uint32_t t = rounds; t >= 1; --t)
    if (stats[2ull * (t - 1) + 1]) {
      last_e = t;
      break;
    }
  uint32_t flags = ctrl->flags;
  if (ctrl->sync.abort) flags |= PEEL_FLAG_TIMEOUT;
  summary[0] = rounds;
  summary[1] = last_e;
  summary[2] = flags;
  summary[3] = static_cast<uint32_t>(n - ctrl->removed);
  summary[4] = ctrl->team.size;
  summary[5] = summary[6] = summary[7] = 0;
}

size_t peel_ws_bytes(uint32_t n) { return align_up(sizeof(PeelCtrl)) + 2 * align_up((size_t)n * 4); }

template <int R>
peel_status launch(PeelArgs &a, hipStream_t s) {
  const void *fn = reinterpret_cast<const void *>(&k_peel_persistent<R>);
  const int cap = coresident_blocks(fn, kBlock, 0);
  uint64_t want = ((uint64_t)a.n + kDenseTile - 1) / kDenseTile;
  const uint64_t want_m = (a.m + 4ull * kBlock - 1) / (4ull * kBlock);
  if (want_m > want) want = want_m;
  if (want < 1) want = 1;
  const unsigned grid = static_cast<unsigned>(want < (uint64_t)cap ? want : (uint64_t)cap);
  if (device_info().debug) std::fprintf(stderr, "[peel] persistent grid %u (cap %d)\n", grid, cap);
  // A plain launch: the kernel forms its team of resident workgroups itself.
  hipLaunchKernelGGL(k_peel_persistent<R>, dim3(grid), dim3(kBlock), 0, s, a);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

}  // namespace
}  // namespace peel

using namespace peel;

extern "C" size_t peel_kcore_workspace(uint32_t n, uint64_t m, uint32_t r) {
  (void)m;
  (void)r;
  return peel_ws_bytes(n);
}

extern "C" peel_status peel_kcore(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n,
                                  uint32_t k, const uint32_t *offsets, const uint32_t *inc,
                                  uint32_t *deg, uint32_t *vertex_round, uint32_t *edge_round,
                                  uint64_t *round_stats, uint32_t max_rounds, uint32_t *summary,
                                  void *ws, size_t ws_bytes, void *stream) {
  if (r < 2 || r > 8 || n == 0 || k == 0 || max_rounds == 0) return PEEL_EINVAL;
  if (m * (uint64_t)r >= (1ull << 32)) return PEEL_EINVAL;
  if ((m && (!edges || !inc || !edge_round)) || !offsets || !deg || !vertex_round ||
      !round_stats || !summary || !ws)
    return PEEL_EINVAL;
  if (ws_bytes < peel_ws_bytes(n)) return PEEL_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  PeelArgs a;
  a.ctrl = c.take<PeelCtrl>(1);
  a.fa = c.take<uint32_t>(n);
  a.fb = c.take<uint32_t>(n);
  a.edges = edges;
  a.offsets = offsets;
  a.inc = inc;
  a.deg = deg;
  a.vr = vertex_round;
  a.er = edge_round;
  a.stats = round_stats;
  a.m = m;
  a.n = n;
  a.k = k;
  a.max_rounds = max_rounds;
  a.limit = device_info().barrier_limit_ticks;
  a.quiet = device_info().team_quiet_ticks;

  hipLaunchKernelGGL(k_peel_init, dim3(1), dim3(64), 0, s, a.ctrl);
  PEEL_HIP_TRY(hipGetLastError());
  peel_status st;
  switch (r) {
    case 2: st = launch<2>(a, s); break;
    case 3: st = launch<3>(a, s); break;
    case 4: st = launch<4>(a, s); break;
    case 5: st = launch<5>(a, s); break;
    case 6: st = launch<6>(a, s); break;
    case 7: st = launch<7>(a, s); break;
    default: st = launch<8>(a, s); break;
  }
  if (st) return st;
  hipLaunchKernelGGL(k_peel_finish, dim3(1), dim3(64), 0, s, a.ctrl, round_stats, n, summary);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

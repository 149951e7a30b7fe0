// peel_k2_xor: the round-synchronous peel to the 2-core without a CSR.
//
// Paper, Section 5 ("Motivation"): listing an IBLT is peeling the hypergraph
// whose vertices are the cells and whose edges are the keys; a pure cell is a
// vertex of degree one, and its key sum names its one item.  Here the same
// equivalence is run the other way: every vertex keeps its degree and the XOR
// of the ids of its alive incident edges, so at k = 2 a vertex of the round's
// set F_t (degree < 2 at the start of round t, Section 1) that still holds an
// edge names that edge directly, with no vertex -> edge lists to read.  Same
// rounds, removal sets and outputs as peel_kcore with k = 2.
//
// One persistent kernel, its team of resident workgroups formed at run time.
// Each of T workgroups owns a range of Vb vertices and holds their degrees
// (then removal rounds) as four-bit fields in LDS; the XORs live in device
// memory, written only by the owner.  A round is:
//   send   each owner walks its part of F_t in vertex order.  A vertex of
//          degree 1 reads its edge e from its XOR and e's row.  F_t is
//          published as a bitmap, so the edge is taken by exactly one of its
//          vertices in F_t: the one in the lowest slot (the rule that makes an
//          IBLT key listed once by its lowest pure cell).  That vertex stamps
//          e's round and sends (u, e) to the owner of every other vertex u of
//          e that is not in F_t.
//   apply  each owner lowers the degree of u and XORs e out of u's word; a
//          degree that falls from 2 to 1 puts u into F_{t+1}.  F_{t+1} is
//          then published.
// A hierarchical barrier ends each phase and sums the round's counts.  An edge
// is alive at the start of round t exactly when none of its vertices has left,
// so a vertex of F_t in an alive edge has degree 1 and names that edge: every
// edge that dies in round t is taken once.
#include "common.hpp"
#include "degxor.hpp"
#include "host.hpp"

namespace peel {
namespace {

constexpr int kXT = 1024;             // threads per workgroup
constexpr uint32_t kXMaxV = 98304;    // owned vertices (LDS four-bit fields)
constexpr uint32_t kXMaxT = 1024;     // workgroups (LDS per-destination counters)
constexpr uint32_t kNib = 15;         // escape value of the four-bit fields
constexpr int kSendU = 4;             // messages per thread in one sorted send chunk
constexpr uint32_t kSendChunk = kSendU * kXT;
constexpr uint32_t kNone = 0xffffffffu;
constexpr int kAU = 2;                // queued messages per thread in one apply chunk
constexpr uint32_t kAC = kAU * kXT;   // messages combined in LDS at a time
constexpr uint32_t kHSBits = 12;
constexpr uint32_t kHS = 1u << kHSBits;  // LDS hash slots for one chunk's vertices
static_assert(2 * kHS * sizeof(uint32_t) <= kSendChunk * sizeof(uint64_t),
              "the apply's hash table fits in the send buffer");
static_assert(kAC * 2 <= kHS, "the hash table stays at most half full");

struct XorCtrl {
  SumBar bar;
  Team team;
  uint32_t flags;
  uint32_t rounds;
  uint32_t team_size;
  uint32_t done;
  uint64_t removed;
  uint32_t qh[kXMaxT];    // message count per destination this round
  uint32_t dsum[kXMaxT];  // incidences of each workgroup's vertices (its queue's size)
  uint64_t stamp[256];
};

struct XorArgs {
  const uint32_t *edges;
  uint32_t *deg;    // initial degrees in, final degrees out
  uint32_t *xr;     // XOR of the alive incident edge ids
  uint32_t *vr;
  uint32_t *er;     // zeroed before the kernel
  uint64_t *stats;
  uint32_t *fbits;  // F_t as a bitmap over the vertices
  uint32_t *flist;  // F_t in vertex order, n entries (each owner its range)
  uint64_t *q;      // messages (vertex | edge << 32), one region per owner
  uint64_t *stage;  // each owner's outgoing messages of the round
  const uint32_t *info;  // [0]: flags of the degree build
  XorCtrl *ctrl;
  uint64_t m;
  uint64_t limit;
  uint64_t quiet;
  uint64_t team_limit;
  uint32_t n;
  uint32_t max_rounds;
};

__global__ void k_xor_init(XorCtrl *ctrl, uint32_t slot_groups) {
  uint32_t *w = reinterpret_cast<uint32_t *>(ctrl);
  for (uint32_t i = threadIdx.x; i < sizeof(XorCtrl) / 4; i += blockDim.x) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) bar_force_slot_groups(&ctrl->bar, slot_groups != 0);
}

__device__ inline bool bit_of(const uint32_t *bits, uint32_t v) {
  return (bits[v >> 5] >> (v & 31)) & 1u;
}

template <int R>
__global__ void __launch_bounds__(kXT) k_peel_xor(XorArgs a) {
  constexpr int kFU = R <= 4 ? 4 : 2;  // frontier vertices per thread whose loads overlap
  __shared__ uint32_t deg4[kXMaxV / 8];  // degree while alive, round once removed
  __shared__ uint32_t gone[kXMaxV / 32];
  __shared__ uint32_t fbl[kXMaxV / 32];  // F_{t+1} as bits over my vertices
  __shared__ uint32_t qb[kXMaxT];        // start of each owner's queue region
  __shared__ uint32_t cnt[kXMaxT];
  __shared__ uint32_t cur[kXMaxT];
  __shared__ uint32_t sst[kXMaxT];
  __shared__ uint64_t sbuf[kSendChunk];
  __shared__ uint32_t scan_lds[kXT / kWave + 1];
  __shared__ uint32_t s_w, s_bad;

  XorCtrl *ctrl = a.ctrl;
  uint32_t slot, T;
  if (!team_join(&ctrl->team, a.quiet, a.team_limit, &slot, &T)) return;
  const uint32_t n = a.n;
  const uint32_t Vb = ((n + T - 1) / T + 31u) & ~31u;
  if (T > kXMaxT || Vb > kXMaxV) {
    // the team that formed cannot hold the vertices in LDS: nothing is peeled
    if (slot == 0 && threadIdx.x == 0) atomicOr(&ctrl->flags, PEEL_FLAG_ETEAM);
    return;
  }
  const uint32_t tid = threadIdx.x;
  const uint32_t v0 = slot * Vb < n ? slot * Vb : n;
  const uint32_t v1 = v0 + Vb < n ? v0 + Vb : n;
  const uint32_t nw = (v1 - v0 + 31) / 32;  // bitmap words of my range
  uint32_t *myF = a.flist + v0;
  // at most R - 1 messages per vertex of mine in a round
  uint64_t *myStage = a.stage + (uint64_t)slot * (R - 1) * Vb;

  // ---- init: LDS degrees, F_1, my queue size ---------------------------------
  if (tid == 0) s_bad = 0;
  for (uint32_t w = tid; w < (Vb + 31) / 32; w += kXT) {
    gone[w] = 0;
    fbl[w] = 0;
  }
  __syncthreads();
  uint32_t dsum = 0;
  for (uint32_t w = tid; w < (Vb + 7) / 8; w += kXT) {
    uint32_t word = 0, low = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t v = v0 + 8 * w + i;
      if (v < v1) {
        const uint32_t d = a.deg[v];
        dsum += d;
        word |= (d >= kNib ? kNib : d) << (4 * i);
        if (d < 2) low |= 1u << i;
      }
    }
    deg4[w] = word;
    if (low) atomicOr(&fbl[w >> 2], low << (8 * (w & 3)));
  }
  {
    uint32_t tot;
    (void)block_exclusive_scan<kXT>(dsum, &tot, scan_lds);
    if (tid == 0) ctrl->dsum[slot] = tot;
  }
  if (slot == 0)
    for (uint64_t i = tid; i < 2ull * a.max_rounds; i += kXT) a.stats[i] = 0;
  // publish F_1
  uint32_t fnext = 0;
  for (uint32_t w = tid; w < nw; w += kXT) {
    a.fbits[v0 / 32 + w] = fbl[w];
    fnext += __popc(fbl[w]);
  }
  uint32_t epoch = 0;
  uint64_t vt;
  {
    uint32_t tot;
    (void)block_exclusive_scan<kXT>(fnext, &tot, scan_lds);
    if (!sum_barrier(&ctrl->bar, T, slot, tot, &epoch, a.limit, &vt, ctrl->stamp)) return;
  }
  // every owner's queue region: the incidences of its vertices bound the
  // messages it can receive in one round
  {
    uint32_t base = 0;
    for (uint32_t d0 = 0; d0 < T; d0 += kXT) {
      const uint32_t d = d0 + tid;
      const uint32_t x = d < T ? atomic_load_u32(&ctrl->dsum[d]) : 0u;
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan<kXT>(x, &tot, scan_lds);
      if (d < T) qb[d] = base + ex;
      base += tot;
    }
    __syncthreads();
  }

  // v leaves in round t: its nibble now keeps the round (vertex_round is
  // written at the end; a round >= kNib is written at once)
  auto mark_removed = [&](uint32_t v, uint32_t lv, uint32_t t) {
    const uint32_t sh = 4 * (lv & 7);
    atomicOr(&gone[lv >> 5], 1u << (lv & 31));
    atomicAnd(&deg4[lv >> 3], ~(kNib << sh));
    if (t < kNib) {
      atomicOr(&deg4[lv >> 3], t << sh);
    } else {
      atomicOr(&deg4[lv >> 3], kNib << sh);
      a.vr[v] = t;
    }
  };
  // Sends src[0, total) to the owners' queues at cur[d] onwards (cur[] already
  // reserved; it advances).  kSendChunk messages at a time are ranked per
  // destination in LDS, sorted there and stored in sorted order, so
  // neighbouring lanes store into one destination's run.  Every thread calls it.
  auto sorted_send = [&](const uint64_t *src, uint32_t total) {
    for (uint32_t c0 = 0; c0 < total; c0 += kSendChunk) {
      const uint32_t cn = total - c0 < kSendChunk ? total - c0 : kSendChunk;
      for (uint32_t d = tid; d < T; d += kXT) cnt[d] = 0;
      __syncthreads();
      uint64_t x[kSendU];
      uint32_t rk[kSendU];
#pragma unroll
      for (int u = 0; u < kSendU; ++u) {
        const uint32_t i = (uint32_t)u * kXT + tid;
        x[u] = i < cn ? src[c0 + i] : ~0ull;
      }
#pragma unroll
      for (int u = 0; u < kSendU; ++u)
        if (x[u] != ~0ull) rk[u] = atomicAdd(&cnt[static_cast<uint32_t>(x[u]) / Vb], 1u);
      __syncthreads();
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan<kXT>(tid < T ? cnt[tid] : 0u, &tot, scan_lds);
      if (tid < T) sst[tid] = ex;
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kSendU; ++u)
        if (x[u] != ~0ull) sbuf[sst[static_cast<uint32_t>(x[u]) / Vb] + rk[u]] = x[u];
      __syncthreads();
      for (uint32_t i = tid; i < tot; i += kXT) {
        const uint64_t msg = sbuf[i];
        const uint32_t d = static_cast<uint32_t>(msg) / Vb;
        a.q[cur[d] + (i - sst[d])] = msg;
      }
      __syncthreads();
      for (uint32_t d = tid; d < T; d += kXT) cur[d] += cnt[d];
    }
  };

  uint64_t removed = 0;
  uint32_t last = 0;
  uint32_t t = 1;
  for (;; ++t) {
    if (vt == 0) break;
    if (t > a.max_rounds) {
      // F_t stays in the graph: the outputs hold the state after max_rounds rounds
      if (slot == 0 && tid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_EROUNDS);
      break;
    }
    last = t;
    removed += vt;
    if (slot == 0 && tid == 0) a.stats[2ull * (t - 1)] = vt;

    // ---- send: F_t in vertex order; each edge taken by its lowest-slot vertex
    uint32_t fcnt = 0;
    for (uint32_t w0 = 0; w0 < nw; w0 += kXT) {
      const uint32_t w = w0 + tid;
      uint32_t bits = 0;
      if (w < nw) {
        bits = fbl[w];
        fbl[w] = 0;
      }
      uint32_t tot;
      uint32_t pos = fcnt + block_exclusive_scan<kXT>(__popc(bits), &tot, scan_lds);
      while (bits) {
        myF[pos++] = v0 + 32 * w + (__ffs(bits) - 1);
        bits &= bits - 1;
      }
      fcnt += tot;
    }
    for (uint32_t d = tid; d < T; d += kXT) cnt[d] = 0;
    if (tid == 0) s_w = 0;
    __syncthreads();
    uint32_t won = 0;  // edges taken by this thread
    uint32_t bad = 0;
    // kFU frontier vertices per thread at a time, so that the three dependent
    // random loads of each (its XOR, its edge's row, the bitmap words of the
    // row's vertices) overlap across them
    for (uint32_t i0 = tid; i0 < fcnt; i0 += kFU * kXT) {
      uint32_t v[kFU], e[kFU], ids[kFU][R], fb[kFU][R];
#pragma unroll
      for (int u = 0; u < kFU; ++u) {
        const uint32_t i = i0 + (uint32_t)u * kXT;
        v[u] = i < fcnt ? myF[i] : kNone;
      }
#pragma unroll
      for (int u = 0; u < kFU; ++u) {
        e[u] = kNone;
        if (v[u] == kNone) continue;
        const uint32_t lv = v[u] - v0;
        const uint32_t d4 = (deg4[lv >> 3] >> (4 * (lv & 7))) & kNib;
        const uint32_t d = d4 == kNib ? a.deg[v[u]] : d4;  // an escaped degree lives in deg
        mark_removed(v[u], lv, t);
        if (d != 0) e[u] = a.xr[v[u]];  // a vertex of degree 0 holds no edge
      }
#pragma unroll
      for (int u = 0; u < kFU; ++u) {
        if (e[u] != kNone && e[u] >= a.m) {  // cannot happen for a consistent XOR
          bad = 1;
          e[u] = kNone;
        }
        const uint32_t *row = a.edges + (uint64_t)(e[u] == kNone ? 0u : e[u]) * R;
#pragma unroll
        for (int j = 0; j < R; ++j) ids[u][j] = e[u] != kNone ? row[j] : kNone;
      }
#pragma unroll
      for (int u = 0; u < kFU; ++u)
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t x = ids[u][j];
          fb[u][j] = (x < n && x != v[u]) ? a.fbits[x >> 5] : 0u;
        }
#pragma unroll
      for (int u = 0; u < kFU; ++u) {
        if (e[u] == kNone) continue;
        // v's slot, and whether a vertex of F_t sits in a lower one
        bool mine = true, seen = false;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t x = ids[u][j];
          if (x == v[u]) {
            seen = true;
          } else if (x < n && ((fb[u][j] >> (x & 31)) & 1u)) {
            if (!seen) mine = false;
            ids[u][j] = kNone;  // leaves in this round too: no decrement
          }
        }
        if (!seen) {
          bad = 1;
          continue;
        }
        if (!mine) continue;
        ++won;
        a.er[e[u]] = t;
        uint32_t nm = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) nm += (ids[u][j] != v[u] && ids[u][j] < n) ? 1u : 0u;
        const uint32_t p = atomicAdd(&s_w, nm);
        uint32_t k = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
          const uint32_t x = ids[u][j];
          if (x == v[u] || x >= n) continue;
          myStage[p + k] = (uint64_t)x | ((uint64_t)e[u] << 32);
          atomicAdd(&cnt[x / Vb], 1u);
          ++k;
        }
      }
    }
    if (bad) s_bad = 1;
    __syncthreads();
    const uint32_t nmsg = s_w;
    for (uint32_t d = tid; d < T; d += kXT) {
      const uint32_t c = cnt[d];
      cur[d] = c ? qb[d] + atomicAdd(&ctrl->qh[d], c) : 0u;
    }
    __syncthreads();
    sorted_send(myStage, nmsg);
    uint32_t wtot;
    (void)block_exclusive_scan<kXT>(won, &wtot, scan_lds);
    uint64_t et;
    if (!sum_barrier(&ctrl->bar, T, slot, wtot, &epoch, a.limit, &et, ctrl->stamp)) return;
    if (slot == 0 && tid == 0) a.stats[2ull * (t - 1) + 1] = et;

    // ---- apply: lower degrees, XOR the dead edges out, collect F_{t+1} ----------
    if (tid == 0) {
      s_w = ctrl->qh[slot];
      ctrl->qh[slot] = 0;
    }
    __syncthreads();
    const uint32_t nin = s_w;
    const uint64_t *myQ = a.q + qb[slot];
    // kAC messages at a time: the edge ids bound for one vertex are XORed
    // together in an LDS hash table (the send buffer's space), then each
    // vertex's word takes them with one plain read-modify-write: this
    // workgroup is its only writer, so no device atomic is needed.
    uint32_t *hkey = reinterpret_cast<uint32_t *>(sbuf);
    uint32_t *hacc = hkey + kHS;
    for (uint32_t c0 = 0; c0 < nin; c0 += kAC) {
      for (uint32_t i = tid; i < kHS; i += kXT) {
        hkey[i] = kNone;
        hacc[i] = 0;
      }
      __syncthreads();
      uint64_t msg[kAU];
      uint32_t hs[kAU];
#pragma unroll
      for (int q = 0; q < kAU; ++q) {
        const uint32_t i = c0 + (uint32_t)q * kXT + tid;
        msg[q] = i < nin ? myQ[i] : ~0ull;
      }
#pragma unroll
      for (int q = 0; q < kAU; ++q) {
        hs[q] = kNone;
        if (msg[q] == ~0ull) continue;
        const uint32_t u = static_cast<uint32_t>(msg[q]);
        const uint32_t e = static_cast<uint32_t>(msg[q] >> 32);
        const uint32_t lv = u - v0;
        if ((gone[lv >> 5] >> (lv & 31)) & 1u) continue;
        const uint32_t sh = 4 * (lv & 7);
        uint32_t old;
        if (((deg4[lv >> 3] >> sh) & kNib) == kNib)
          old = atomicSub(&a.deg[u], 1u);
        else
          old = (atomicSub(&deg4[lv >> 3], 1u << sh) >> sh) & kNib;
        if (old == 2) atomicOr(&fbl[lv >> 5], 1u << (lv & 31));
        // lv's slot (linear probing; at most kAC keys in kHS slots)
        uint32_t h = (lv * 0x9e3779b1u) >> (32 - kHSBits);
        for (;;) {
          const uint32_t k = atomicCAS(&hkey[h], kNone, lv);
          if (k == kNone) {
            hs[q] = h;  // the first message of lv in this chunk applies them all
            break;
          }
          if (k == lv) break;
          h = (h + 1) & (kHS - 1);
        }
        atomicXor(&hacc[h], e);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kAU; ++q) {
        if (hs[q] == kNone) continue;
        uint32_t *w = a.xr + v0 + hkey[hs[q]];
        *w = atomic_load_u32(w) ^ hacc[hs[q]];
      }
      __syncthreads();
    }
    // publish F_{t+1}
    fnext = 0;
    for (uint32_t w = tid; w < nw; w += kXT) {
      a.fbits[v0 / 32 + w] = fbl[w];
      fnext += __popc(fbl[w]);
    }
    uint32_t ftot;
    (void)block_exclusive_scan<kXT>(fnext, &ftot, scan_lds);
    if (!sum_barrier(&ctrl->bar, T, slot, ftot, &epoch, a.limit, &vt, ctrl->stamp)) return;
  }

  // ---- epilogue: removal rounds and final degrees, written in order ------------
  for (uint32_t v = v0 + tid; v < v1; v += kXT) {
    const uint32_t lv = v - v0;
    const uint32_t b = (deg4[lv >> 3] >> (4 * (lv & 7))) & kNib;
    if ((gone[lv >> 5] >> (lv & 31)) & 1u) {
      a.deg[v] = 0;
      if (b != kNib) a.vr[v] = b;
    } else {
      a.vr[v] = 0;
      if (b != kNib) a.deg[v] = b;
    }
  }
  if (s_bad && tid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
  if (slot == 0 && tid == 0) {
    ctrl->rounds = last;
    ctrl->removed = removed;
    ctrl->team_size = T;
    ctrl->done = 1;
  }
}

__global__ void k_xor_finish(const XorCtrl *ctrl, const uint64_t *stats, const uint32_t *info,
                             uint32_t n, uint32_t *summary) {
  if (threadIdx.x != 0) return;
  const uint32_t rounds = ctrl->rounds;
  uint32_t last_e = 0;
  for (uint32_t t = rounds; t >= 1; --t)
    if (stats[2ull * (t - 1) + 1]) {
      last_e = t;
      break;
    }
  uint32_t flags = ctrl->flags | info[0];
  if (ctrl->bar.abort || (!ctrl->done && !(flags & PEEL_FLAG_ETEAM))) flags |= PEEL_FLAG_TIMEOUT;
  summary[0] = rounds;
  summary[1] = last_e;
  summary[2] = flags;
  summary[3] = static_cast<uint32_t>(n - ctrl->removed);
  summary[4] = ctrl->team_size;
  summary[5] = summary[6] = summary[7] = 0;
}

struct XLayout {
  size_t ctrl, xr, fbits, flist, q, stage, info, build, total;
};

XLayout xlayout(uint32_t n, uint64_t m, uint32_t r) {
  const uint64_t g = (uint64_t)device_info().cus + 64;  // team size upper bound
  XLayout L{};
  L.ctrl = align_up(sizeof(XorCtrl));
  L.xr = align_up((size_t)n * 4);
  L.fbits = align_up(((size_t)n + 31) / 32 * 4 + 4);
  L.flist = align_up((size_t)n * 4);
  L.q = align_up((size_t)r * m * 8 + 8);
  // T stages of (r - 1) Vb messages, with T Vb <= n + 32 T
  L.stage = align_up((size_t)(r - 1) * ((uint64_t)n + 32 * g) * 8);
  L.info = align_up(16);
  L.build = align_up(degxor_ws_bytes(n, m, r));
  L.total = L.ctrl + L.xr + L.fbits + L.flist + L.q + L.stage + L.info + L.build;
  return L;
}

template <int R>
peel_status launch_xor(XorArgs &a, hipStream_t s) {
  const DeviceInfo &dev = device_info();
  const unsigned grid = static_cast<unsigned>(dev.cus < (int)kXMaxT ? dev.cus : (int)kXMaxT);
  if (dev.debug) std::fprintf(stderr, "[peel] xor grid %u\n", grid);
  hipLaunchKernelGGL(k_peel_xor<R>, dim3(grid), dim3(kXT), 0, s, a);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

}  // namespace
}  // namespace peel

using namespace peel;

extern "C" size_t peel_k2_xor_workspace(uint32_t n, uint64_t m, uint32_t r) {
  if (r < 2 || r > 8 || n == 0) return 0;
  return xlayout(n, m, r).total;
}

extern "C" peel_status peel_k2_xor(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n,
                                   uint32_t *deg, uint32_t *vertex_round, uint32_t *edge_round,
                                   uint64_t *round_stats, uint32_t max_rounds, uint32_t *summary,
                                   void *ws, size_t ws_bytes, void *stream) {
  if (r < 2 || r > 8 || n == 0 || max_rounds == 0) return PEEL_EINVAL;
  if (m * (uint64_t)r >= (1ull << 32)) return PEEL_EINVAL;
  if ((m && (!edges || !edge_round)) || !deg || !vertex_round || !round_stats || !summary || !ws)
    return PEEL_EINVAL;
  const XLayout L = xlayout(n, m, r);
  if (ws_bytes < L.total) return PEEL_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ws);
  XorArgs a{};
  a.ctrl = reinterpret_cast<XorCtrl *>(base);
  base += L.ctrl;
  a.xr = reinterpret_cast<uint32_t *>(base);
  base += L.xr;
  a.fbits = reinterpret_cast<uint32_t *>(base);
  base += L.fbits;
  a.flist = reinterpret_cast<uint32_t *>(base);
  base += L.flist;
  a.q = reinterpret_cast<uint64_t *>(base);
  base += L.q;
  a.stage = reinterpret_cast<uint64_t *>(base);
  base += L.stage;
  uint32_t *info = reinterpret_cast<uint32_t *>(base);
  base += L.info;
  void *bws = base;
  a.info = info;
  a.edges = edges;
  a.deg = deg;
  a.vr = vertex_round;
  a.er = edge_round;
  a.stats = round_stats;
  a.m = m;
  a.n = n;
  a.max_rounds = max_rounds;
  a.limit = barrier_limit_ticks();
  a.team_limit = device_info().team_limit_ticks;
  a.quiet = device_info().team_quiet_ticks;
  hipLaunchKernelGGL(k_xor_init, dim3(1), dim3(256), 0, s, a.ctrl,
                     barrier_slots() ? 1u : 0u);
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(kBlock), 0, s, info, (uint64_t)4, 0u);
  if (m)
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(m, kBlock * 4, 4096)), dim3(kBlock), 0, s,
                       edge_round, m, 0u);
  PEEL_HIP_TRY(hipGetLastError());
  peel_status st = degxor_build(edges, m, r, n, deg, a.xr, info, bws, s);
  if (st) return st;
  switch (r) {
    case 2: st = launch_xor<2>(a, s); break;
    case 3: st = launch_xor<3>(a, s); break;
    case 4: st = launch_xor<4>(a, s); break;
    case 5: st = launch_xor<5>(a, s); break;
    case 6: st = launch_xor<6>(a, s); break;
    case 7: st = launch_xor<7>(a, s); break;
    default: st = launch_xor<8>(a, s); break;
  }
  if (st) return st;
  hipLaunchKernelGGL(k_xor_finish, dim3(1), dim3(64), 0, s, a.ctrl, round_stats, info, n, summary);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

// peel_kcore: round-synchronous parallel peeling to the k-core.
//
// Paper, Section 1 and Section 3: in round t every vertex whose degree is
// below k at the start of the round is removed at once, together with every
// edge still holding it; the run ends at the first round with nothing to
// remove.  Section 5 ("Implementation Details") notes that a parallel peel
// must never peel one edge twice.
//
// Two engines, both persistent kernels whose team of resident workgroups is
// formed at run time, with no host round trip between rounds:
//
// Owner engine (the default).  Device-scope atomics run at a fixed ~27 G/s on
// this GPU whatever the working set, so the owner engine keeps the per-edge
// work in LDS.  Each of T workgroups (one per CU) owns a range of Vb vertices,
// whose degrees (then removal rounds) it holds as four-bit fields in LDS, and
// a range of Eb edges, whose "alive" bits and removal rounds it holds in LDS.
// A round is two message exchanges through per-destination queues in HBM (a
// workgroup counts its messages per destination in LDS, reserves space with
// one atomic per destination, then writes them):
//   claims      each owner sends, for every vertex of its frontier F_t, one
//               claim per incident edge to that edge's owner;
//   decrements  each edge owner clears the alive bit of every claimed edge
//               (an LDS atomic, so an edge claimed by several peeled vertices
//               dies once), stamps its round, and sends one decrement per slot
//               to the slot vertex's owner, which lowers the LDS degree; a
//               decrement that takes a degree from k to k-1 puts the vertex
//               into the owner's F_{t+1}.
// A hierarchical barrier after each exchange also sums |F_t| and the edges
// removed.  A degree >= 15 lives in the global degree array instead (marked
// 15 in LDS) and is updated with device atomics; a round >= 15 is written to
// vertex_round or edge_round at once (also marked 15).  The other rounds and
// degrees are written in order at the end.
//
// Global engine (used when a workgroup's vertex or edge range does not fit in
// LDS, or the team is too small).  Every round, the threads walk F_t and claim
// each still-alive incident edge by compare-and-swap on its round word
// (0 -> t); the winner lowers the degree of each of its r slots with a device
// atomic and pushes a vertex whose degree crossed k -> k-1 onto F_{t+1}.
//
// Both are exact: a vertex alive at the start of round t with degree >= k
// crosses k -> k-1 at most once, so F_{t+1} is exactly the set of alive
// vertices whose degree dropped below k during round t; vertices of F_t start
// below k and never trigger a push.  Every slot of a removed edge is
// decremented, so removed vertices end at degree 0 and core vertices at their
// core degree, whatever the order of the atomics.
#include "common.hpp"
#include "host.hpp"

#include <cstring>

namespace peel {
namespace {

#ifndef PEEL_LDS_QUEUE
#define PEEL_LDS_QUEUE 4096
#endif
constexpr int kQueue = PEEL_LDS_QUEUE;  // LDS push-queue entries per workgroup (global engine)
constexpr int kDenseItems = 8;          // vertices per thread in the dense pass
constexpr int kDenseTile = kBlock * kDenseItems;

constexpr int kOT = 1024;             // threads per owner workgroup
constexpr uint32_t kOwnMaxV = 98304;  // owned vertices (LDS degree nibbles)
constexpr uint32_t kOwnMaxVX = 65536; // owned vertices when their dead-edge nibbles fit in LDS too
constexpr uint32_t kOwnMaxE = 65536;  // owned edges (LDS alive and claimed bits)
constexpr uint32_t kOwnMaxT = 256;    // owner workgroups (LDS per-destination counters)
constexpr uint64_t kDenseRatio = 3;   // dense round when |F_{t-1}| * 3 >= alive edges
constexpr uint32_t kNoVertex = 0xffffffffu;
constexpr uint32_t kNib = 15;         // escape value of the owner engine's 4-bit fields
constexpr int kSendU = 4;             // messages per thread in one sorted send chunk
constexpr uint32_t kSendChunk = kSendU * kOT;  // messages sorted in LDS at a time
constexpr int kLU = 4;                // queue entries per thread whose loads are in flight
constexpr int kCV = 2;                // frontier vertices per lane in one pass of the claim walk
constexpr int kCE = 8;                // incidences per frontier vertex loaded at once
constexpr uint32_t kIdMask = 0x0fffffffu;  // a decrement's vertex; its top four bits carry
constexpr int kNibShift = 28;              // the low four bits of the dying edge's id
// Compact list bounds (owner engine): a 64-byte block per kCoffV of a
// workgroup's vertices holds the first one's CSR offset (bit 31 set: the
// block holds more than 255 incidences, read the offsets array instead) and
// kCoffV + 1 one-byte offsets from it, the last being the end of the block's
// last list.  Neighbouring frontier vertices then share far more lines than
// in the 4-byte offsets array.  The blocks are built at the start from the
// degrees (a workgroup scan), so building them reads nothing more.
constexpr uint32_t kCoffV = 56;  // seven words of eight degree nibbles
constexpr uint32_t kCoffW = kCoffV / 8;
constexpr uint32_t kCoffIt = (kOT / kCoffW) * kCoffW;  // degree words per pass of the build
constexpr uint32_t kCoffEsc = 0x80000000u;

// kModeRetry: the claim-filter kernel declined (the team that formed was too
// small for its LDS), the owner kernel without the filter takes the run
enum : uint32_t { kModeUndecided = 0, kModeOwnerDone = 1, kModeGlobal = 2, kModeRetry = 3 };
enum : uint32_t { kRoundsAuto = 0, kRoundsDense = 1, kRoundsSparse = 2 };

struct PeelCtrl {
  SumBar bar;          // owner engine barrier
  GridSync sync;       // global engine barrier
  Team team_own;
  Team team_own2;  // the owner kernel without the claim filter, after kModeRetry
  Team team_glob;
  uint32_t mode;
  uint32_t fcount[3];  // global engine: |F_t| lives in fcount[t % 3]
  uint32_t flags;
  uint32_t rounds;
  uint32_t team;
  uint32_t pad;
  uint64_t removed;
  uint32_t qh_claim[kOwnMaxT];  // owner engine queue heads
  uint32_t qh_dec[kOwnMaxT];
  uint64_t stamp[256];          // wall clock at each barrier generation (diagnostic)
};

struct PeelArgs {
  const uint32_t *edges;
  const uint32_t *offsets;
  const uint32_t *inc;
  uint32_t *deg;
  uint32_t *vr;
  uint32_t *er;
  uint64_t *stats;
  uint32_t *fa;      // frontiers (n each)
  uint32_t *fb;
  uint32_t *qclaim;  // owner engine: R * (m + grid) claim slots
  uint32_t *qdec;    // owner engine: R * m decrement slots, laid out by the CSR offsets
  uint32_t *stage;   // owner engine: R * (m + grid) rows of the edges won this round
  uint32_t *fbits;   // owner engine: F_t as a bitmap over the vertices (dense rounds)
  uint32_t *coff;    // owner engine: compact list bounds, 16 words per block of kCoffV vertices
  uint64_t coff_blocks;  // blocks that coff holds
  PeelCtrl *ctrl;
  uint64_t m;
  uint64_t limit;
  uint64_t quiet;
  uint64_t team_limit;
  uint32_t n;
  uint32_t k;
  uint32_t max_rounds;
  uint32_t force_global;  // PEEL_ENGINE=global: skip the owner engine (testing)
  uint32_t round_policy;  // PEEL_ROUNDS=sparse (default) | dense | auto (chosen per round)
  uint32_t subtables;     // 1: peeling with subtables, rounds are subrounds
  uint32_t claims_all;    // PEEL_CLAIMS=all: owner engine without the claim filter;
                          // =retry: the claim-filter kernel declines as if its team
                          // were too small (testing)
  uint32_t retry;         // this launch runs only after the claim-filter kernel declined
  uint32_t sub_lo[9];     // subtable j holds the vertices sub_lo[j] .. sub_lo[j+1]-1
};

// The subtable of vertex v (subtables mode).
__device__ inline uint32_t subtable_of_vertex(const PeelArgs &a, uint32_t r, uint32_t v) {
  uint32_t j = 0;
  for (uint32_t i = 1; i < r; ++i)
    if (v >= a.sub_lo[i]) j = i;
  return j;
}

__global__ void k_peel_init(PeelCtrl *ctrl, uint32_t slot_groups) {
  uint32_t *w = reinterpret_cast<uint32_t *>(ctrl);
  for (uint32_t i = threadIdx.x; i < sizeof(PeelCtrl) / 4; i += blockDim.x) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) bar_force_slot_groups(&ctrl->bar, slot_groups != 0);
}

// ===========================================================================
// Owner engine.

// Position of the r-th set bit (from 0) of x; x has more than r set bits.
__device__ inline uint32_t nth_set_bit(uint32_t x, uint32_t r) {
  uint32_t pos = 0, c;
  c = __popc(x & 0xffffu);
  if (r >= c) { r -= c; x >>= 16; pos += 16; }
  c = __popc(x & 0xffu);
  if (r >= c) { r -= c; x >>= 8; pos += 8; }
  c = __popc(x & 0xfu);
  if (r >= c) { r -= c; x >>= 4; pos += 4; }
  c = __popc(x & 0x3u);
  if (r >= c) { r -= c; x >>= 2; pos += 2; }
  return pos + (r >= (x & 1u) ? 1u : 0u);
}

// XF (the claim filter; for up to kOwnMaxVX vertices per workgroup): each
// owned vertex also keeps, in four bits of LDS, the XOR of the low four bits
// of the ids of its dead incident edges (every decrement carries them).  A
// frontier vertex that holds exactly one alive edge XORs the low four bits of
// its whole list with these, which gives the low four bits of that edge, and
// claims only the list entries that match: the alive edge, and on average one
// dead entry in sixteen.  Without it such a vertex claims its whole list, most
// of which names edges that died in earlier rounds (claims of dead edges are
// ignored by their owners, so both are exact).
template <int R, bool XF>
__global__ void __launch_bounds__(kOT) k_peel_owner(PeelArgs a) {
  constexpr uint32_t kV = XF ? kOwnMaxVX : kOwnMaxV;
  // Four bits per owned vertex: its degree while alive (kNib = held in the
  // global degree array instead), its removal round once removed (kNib = t >=
  // kNib, written to vertex_round directly).  `gone` marks the removed vertices.
  __shared__ uint32_t deg4[kV / 8];
  __shared__ uint32_t gone[kV / 32];
  __shared__ uint32_t dx4[XF ? kV / 8 : 1];  // XF: dead-edge id nibbles, XORed
  __shared__ uint32_t alive[kOwnMaxE / 32];
  __shared__ uint32_t claimed[kOwnMaxE / 32];  // edges claimed this round
  // Four bits per owned edge: its removal round (0 = alive; kNib = t >= kNib,
  // written to edge_round directly).  edge_round is written in order at the end.
  __shared__ uint32_t er4[kOwnMaxE / 8];
  __shared__ uint32_t cnt[kOwnMaxT];
  __shared__ uint32_t cur[kOwnMaxT];
  __shared__ uint32_t s_start[kOT];
  __shared__ uint32_t s_pre[kOT];
  __shared__ uint32_t scan_lds[kOT / kWave + 1];
  __shared__ uint32_t fbl[kV / 32];        // the next frontier, as bits over my vertices
  __shared__ uint32_t sbuf[kSendChunk];    // messages sorted by destination before a send
  __shared__ uint32_t sst[kOwnMaxT];       // their starts per destination
  __shared__ uint32_t s_n, s_w, s_p, s_c;

  PeelCtrl *ctrl = a.ctrl;
  if (a.retry &&
      __hip_atomic_load(&ctrl->mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kModeRetry)
    return;
  uint32_t slot, T;
  if (!team_join(a.retry ? &ctrl->team_own2 : &ctrl->team_own, a.quiet, a.team_limit, &slot, &T))
    return;
  const uint32_t n = a.n;
  // vertex ranges start on 32-vertex boundaries, so bitmap slices do not share words
  const uint32_t Vb = ((n + T - 1) / T + 31u) & ~31u;
  const uint64_t m = a.m;
  const uint32_t Eb = m ? (uint32_t)((m + T - 1) / T) : 1u;
  if (a.force_global || T > kOwnMaxT || Vb > kV || Eb > kOwnMaxE || (XF && a.claims_all == 2)) {
    // a team too small for the claim filter's LDS may still fit the wider kernel
    const bool wider = XF && !a.force_global && T <= kOwnMaxT && Vb <= kOwnMaxV && Eb <= kOwnMaxE;
    if (slot == 0 && threadIdx.x == 0) ctrl->mode = wider ? kModeRetry : kModeGlobal;
    return;
  }
  const uint32_t tid = threadIdx.x;
  const uint32_t v0 = slot * Vb < n ? slot * Vb : n;
  const uint32_t v1 = v0 + Vb < n ? v0 + Vb : n;
  const uint64_t e0 = (uint64_t)slot * Eb < m ? (uint64_t)slot * Eb : m;
  const uint64_t e1 = e0 + Eb < m ? e0 + Eb : m;
  const uint32_t k = a.k;
  uint32_t *myF = a.fa + v0;
  uint32_t *myStage = a.stage + (uint64_t)slot * Eb * R;
  const uint32_t *myClaims = a.qclaim + (uint64_t)slot * Eb * R;
  uint32_t *myDecs = a.qdec + a.offsets[v0];

  // ---- init: LDS degrees, alive bits, outputs, F_1 --------------------------
  if (tid == 0) s_p = 0;
  for (uint32_t w = tid; w < Vb / 32; w += kOT) {
    gone[w] = 0;
    fbl[w] = 0;
  }
  if (XF)
    for (uint32_t w = tid; w < Vb / 8; w += kOT) dx4[w] = 0;
  for (uint32_t w = tid; w < (Eb + 31) / 32; w += kOT) {
    const uint64_t lo = e0 + 32ull * w;
    uint32_t bits = 0;
    if (lo < e1) bits = (e1 - lo >= 32) ? 0xffffffffu : ((1u << (uint32_t)(e1 - lo)) - 1u);
    alive[w] = bits;
    claimed[w] = 0;
  }
  for (uint32_t w = tid; w < (Eb + 7) / 8; w += kOT) er4[w] = 0;
  __syncthreads();
  // Degrees into LDS nibbles and F_1 into the bitmap, kCoffIt words of eight
  // vertices a pass; the same pass writes the compact list bounds: a scan of
  // the words' degree sums gives every vertex its offset, a block's first word
  // writes the block's base, each word its eight bytes, a block's last word
  // the closing byte.  They are used only if they end at offsets[v1].
  const uint32_t nbk = (Vb + kCoffV - 1) / kCoffV;  // blocks per workgroup
  uint32_t *myCoff = a.coff + (uint64_t)slot * nbk * 16;
  const bool coff_fits = (uint64_t)T * nbk <= a.coff_blocks;
  const uint32_t off0 = a.offsets[v0];
  uint32_t run = 0;   // degree sum of my vertices before this pass
  uint32_t nlow = 0;  // my vertices below k
  // the degrees of my word of the pass at w0 (0 past my range); the next
  // pass's load while this pass scans
  auto load_deg = [&](uint32_t w0, uint32_t *dg) {
    const uint32_t w = w0 + tid;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t v = v0 + 8 * w + i;
      dg[i] = tid < kCoffIt && w < Vb / 8 && v < v1 ? a.deg[v] : 0u;
    }
  };
  uint32_t dnext[8];
  load_deg(0, dnext);
  for (uint32_t w0 = 0; w0 < Vb / 8; w0 += kCoffIt) {
    const uint32_t w = w0 + tid;
    const bool mine = tid < kCoffIt && w < Vb / 8;
    uint32_t dg[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) dg[i] = dnext[i];
    load_deg(w0 + kCoffIt, dnext);
    uint32_t word = 0, low = 0, sum = 0;
    uint32_t loc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t v = v0 + 8 * w + i;
      loc[i] = sum;
      if (mine && v < v1) {
        const uint32_t d = dg[i];
        word |= (d >= kNib ? kNib : d) << (4 * i);
        if (d < k) low |= 1u << i;
        sum += d;
      }
    }
    if (mine) {
      deg4[w] = word;
      if (low) atomicOr(&fbl[w >> 2], low << (8 * (w & 3)));
      nlow += __popc(low);
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kOT>(sum, &tot, scan_lds);
    s_pre[tid] = ex;  // s_pre[kCoffIt] is the pass's end (kCoffIt < kOT)
    __syncthreads();
    if (coff_fits && mine) {
      const uint32_t kb = tid % kCoffW, b = w / kCoffW;
      const uint32_t bstart = s_pre[tid - kb];  // the block's first offset in this pass
      const uint32_t bend = s_pre[tid - kb + kCoffW];
      uint32_t *blk = myCoff + b * 16;
      if (kb == 0) blk[0] = (off0 + run + bstart) | (bend - bstart > 255u ? kCoffEsc : 0u);
      const uint32_t rel = ex - bstart;
      blk[1 + 2 * kb] = ((rel + loc[0]) & 255u) | ((rel + loc[1]) & 255u) << 8 |
                        ((rel + loc[2]) & 255u) << 16 | (rel + loc[3]) << 24;
      blk[2 + 2 * kb] = ((rel + loc[4]) & 255u) | ((rel + loc[5]) & 255u) << 8 |
                        ((rel + loc[6]) & 255u) << 16 | (rel + loc[7]) << 24;
      if (kb == kCoffW - 1)
        blk[15] = (bend - bstart) & 255u;
      else if (w == Vb / 8 - 1)  // my last block ends early: its closing byte
        blk[3 + 2 * kb] = (rel + sum) & 255u;
    }
    run += tot;
    __syncthreads();
  }
  nlow = block_sum<kOT>(nlow, scan_lds);
  if (tid == 0) {
    s_w = (off0 + run == a.offsets[v1]) ? 1u : 0u;
    s_p = nlow;
  }
  __syncthreads();
  const bool coff = coff_fits && s_w != 0;
  if (slot == 0)
    for (uint64_t i = tid; i < 2ull * a.max_rounds; i += kOT) a.stats[i] = 0;
  if (tid == 0) s_n = ~0u;  // F_1 is taken from the bitmap
  __syncthreads();
  uint32_t fcnt = 0;
  // Subtables mode: subround t takes only the frontier bits of subtable
  // (t-1) mod R; the bits of the other subtables wait in the bitmap.  `pend`
  // counts my waiting bits, so that the run ends when no workgroup has any.
  const bool sub = a.subtables != 0;
  uint32_t pend = s_p;

  // v leaves in round t with every edge it still holds, so its final degree
  // is 0; its nibble now keeps the round (vertex_round is written at the end)
  auto mark_removed = [&](uint32_t v, uint32_t lv, uint32_t t) {
    const uint32_t sh = 4 * (lv & 7);
    atomicOr(&gone[lv >> 5], 1u << (lv & 31));
    atomicAnd(&deg4[lv >> 3], ~(kNib << sh));
    if (t < kNib)
      atomicOr(&deg4[lv >> 3], t << sh);
    else {
      atomicOr(&deg4[lv >> 3], kNib << sh);
      a.vr[v] = t;
    }
  };
  // Sends the messages src[0, total) whose bits under `mask` are below `lim`
  // to the queues q, at cur[d] onwards for destination d = (x & mask) / per
  // (cur[] already reserved; it advances).
  // kSendChunk messages at a time are ranked per destination, sorted in LDS
  // and stored in sorted order, so neighbouring lanes store to neighbouring
  // places of one destination's run instead of one store per destination.
  // Uses cnt[] (free once cur[] is set).  Every thread calls it; `total` is
  // the same in every thread.
  auto sorted_send = [&](const uint32_t *src, uint32_t total, uint32_t lim, uint32_t per,
                         uint32_t T_, uint32_t *q, uint32_t mask) {
    if (total <= (uint32_t)kOT) {
      // a few messages (the many small rounds near and above the threshold):
      // sorting would cost more than the stores it merges
      const uint32_t x = tid < total ? src[tid] : lim;
      if ((x & mask) < lim) q[atomicAdd(&cur[(x & mask) / per], 1u)] = x;
      return;
    }
    for (uint32_t c0 = 0; c0 < total; c0 += kSendChunk) {
      const uint32_t cn = total - c0 < kSendChunk ? total - c0 : kSendChunk;
      for (uint32_t d = tid; d < T_; d += kOT) cnt[d] = 0;
      __syncthreads();
      uint32_t x[kSendU], rk[kSendU];
#pragma unroll
      for (int u = 0; u < kSendU; ++u) {
        const uint32_t i = (uint32_t)u * kOT + tid;
        x[u] = i < cn ? src[c0 + i] : lim;
      }
#pragma unroll
      for (int u = 0; u < kSendU; ++u)
        if ((x[u] & mask) < lim) rk[u] = atomicAdd(&cnt[(x[u] & mask) / per], 1u);
      __syncthreads();
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan<kOT>(tid < T_ ? cnt[tid] : 0u, &tot, scan_lds);
      if (tid < T_) sst[tid] = ex;
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kSendU; ++u)
        if ((x[u] & mask) < lim) sbuf[sst[(x[u] & mask) / per] + rk[u]] = x[u];
      __syncthreads();
      for (uint32_t i = tid; i < tot; i += kOT) {
        const uint32_t v = sbuf[i];
        const uint32_t d = (v & mask) / per;
        q[cur[d] + (i - sst[d])] = v;
      }
      __syncthreads();
      for (uint32_t d = tid; d < T_; d += kOT) cur[d] += cnt[d];
    }
  };
  // The decrement for slot vertex id of dying edge e (XF: with e's low four
  // bits on top; an id >= n is dropped)
  auto dmsg = [&](uint32_t id, uint64_t e) -> uint32_t {
    if (!XF) return id;
    return id < n ? id | (static_cast<uint32_t>(e) & 15u) << kNibShift : kNoVertex;
  };
  // my edge le dies in round t; its nibble held cn until now (the claim
  // marking's note, else 0)
  auto mark_edge = [&](uint32_t le, uint32_t t, uint32_t cn) {
    const uint32_t sh = 4 * (le & 7);
    atomicXor(&er4[le >> 3], ((t < kNib ? t : kNib) ^ cn) << sh);
    if (t >= kNib) a.er[e0 + le] = t;
  };
  // Stages the decrements of dying edge e (row ids) at stage slot w; the slot
  // whose vertex's low four bits are cn (the one claimer's) is skipped when it
  // is the only such slot: that vertex leaves this round and would ignore it.
  auto stage_row = [&](uint32_t w, uint64_t e, const uint32_t *ids, uint32_t cn) {
    uint32_t skip = R;
    if (cn < kNib) {
      uint32_t hits = 0;
#pragma unroll
      for (int q = 0; q < R; ++q)
        if ((ids[q] & 15u) == cn) {
          skip = q;
          ++hits;
        }
      if (hits != 1) skip = R;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const bool send = (uint32_t)q != skip && ids[q] < n;
      myStage[(uint64_t)w * R + q] = send ? dmsg(ids[q], e) : kNoVertex;
      if (send) atomicAdd(&cnt[ids[q] / Vb], 1u);
    }
  };

  uint32_t epoch = 0;
  uint64_t removed = 0;
  uint64_t alive_m = m;  // edges alive at the start of the round
  uint64_t prev_v = 0;   // |F_{t-1}|
  uint32_t last = 0;     // the last round that removed a vertex
  uint32_t t = 1;
  for (;; ++t) {
    const bool over = t > a.max_rounds;
    // Two ways to find the edges that die in round t.  Sparse (the default):
    // every vertex of F_t that still holds an edge sends a claim for each
    // incident edge to the edge's owner.  Dense: every edge owner streams the
    // rows of its alive edges and tests their slots against F_t, published as
    // a bitmap (n bits, which stays in L2).  Both are bound by random reads: a
    // few CSR lines per frontier vertex against R bitmap tests per alive edge.
    // Measured on the n = 2^24 workloads, sparse rounds are never slower by
    // much and the scan loses badly above the threshold, so dense rounds run
    // only when asked for (every round, or chosen per round by the size of the
    // last frontier against the alive edges).  Every workgroup takes the same
    // decision from the same global counts.
    const bool dense = sub ? false
                     : a.round_policy == kRoundsAuto ? (t == 1 || prev_v * kDenseRatio >= alive_m)
                                                      : a.round_policy == kRoundsDense;
    // ---- F_t in vertex order: the bitmap is compacted into myF (and cleared for
    // F_{t+1}); a dense round also publishes it.  Walking F_t in vertex order
    // makes neighbouring frontier vertices share the lines of the CSR.
    // A frontier of at most kOT vertices was also listed in s_start by the
    // decrement phase: it is taken from there (its bits cleared one by one)
    // instead of scanning the whole bitmap.
    const bool publish = dense && !over;
    if (!sub && s_n <= (uint32_t)kOT && !publish) {
      fcnt = s_n;
      for (uint32_t i = tid; i < fcnt; i += kOT) {
        const uint32_t v = s_start[i];
        myF[i] = v;
        atomicAnd(&fbl[(v - v0) >> 5], ~(1u << ((v - v0) & 31)));
      }
      __syncthreads();
    } else {
      // the vertices [x0, x1) whose bits are taken: all of mine, or in
      // subtables mode those of this subround's subtable
      uint32_t x0 = v0, x1 = v1;
      if (sub) {
        const uint32_t j = (t - 1) % R;
        x0 = a.sub_lo[j] > v0 ? a.sub_lo[j] : v0;
        x1 = a.sub_lo[j + 1] < v1 ? a.sub_lo[j + 1] : v1;
        if (x1 < x0) x1 = x0;
      }
      const uint32_t wlo = (x0 - v0) >> 5, whi = (x1 - v0 + 31) >> 5;
      fcnt = 0;
      for (uint32_t w0 = wlo; w0 < whi; w0 += kOT) {
        const uint32_t w = w0 + tid;
        uint32_t bits = 0;
        if (w < whi) {
          const uint32_t base = v0 + 32 * w;
          const uint32_t b0 = x0 > base ? x0 - base : 0u;
          const uint32_t b1 = x1 - base < 32u ? x1 - base : 32u;
          const uint32_t mask = (b1 == 32u ? ~0u : (1u << b1) - 1u) & ~((1u << b0) - 1u);
          bits = fbl[w] & mask;
          fbl[w] &= ~mask;
          if (publish) a.fbits[v0 / 32 + w] = bits;
        }
        uint32_t tot;
        uint32_t pos = fcnt + block_exclusive_scan<kOT>(__popc(bits), &tot, scan_lds);
        while (bits) {
          myF[pos++] = v0 + 32 * w + (__ffs(bits) - 1);
          bits &= bits - 1;
        }
        fcnt += tot;
      }
      __syncthreads();
    }
    if (!over && dense) {
      // ---- dense: F_t's vertices leave with every edge they hold, so their
      // degrees go to 0 now and the edge scan sends them no decrement
      for (uint32_t i = tid; i < fcnt; i += kOT) {
        const uint32_t v = myF[i];
        mark_removed(v, v - v0, t);
      }
    }
    // ---- sparse: claims for the incidences of every vertex of F_t that still
    // holds an edge (XF: only the matching ones of a vertex holding one).  Each
    // wave walks its own frontier vertices, kCV per lane at a time, with no
    // workgroup-wide step: a lane loads the list bounds of its vertices, then
    // up to kCE incidences of each at once (the rest of a longer list is read
    // one incidence at a time), and the wave reserves its claims' places with
    // one LDS atomic.  The claims are counted per destination and kept in this
    // workgroup's decrement queue, which is idle until the edge owners write it
    // after the next barrier and is as long as my vertices' lists; then they
    // are copied to their destinations.
    if (!over && !dense) {
      uint32_t *claims = myDecs;
      for (uint32_t d = tid; d < T; d += kOT) cnt[d] = 0;
      if (tid == 0) s_c = 0;
      __syncthreads();
      const uint32_t lane = tid & (kWave - 1);
      // lane's vertices of the pass at b: bounds of their lists, and the low
      // bits to match (16 = claim every entry)
      auto head = [&](uint32_t b, uint32_t *st, uint32_t *len, uint32_t *want) {
#pragma unroll
        for (int u = 0; u < kCV; ++u) {
          const uint32_t i = b + (uint32_t)u * kWave + lane;
          st[u] = 0;
          len[u] = 0;
          want[u] = 16;
          if (i < fcnt) {
            const uint32_t v = myF[i];
            const uint32_t lv = v - v0;
            const uint32_t d4 = (deg4[lv >> 3] >> (4 * (lv & 7))) & kNib;
            if (XF && d4 == 1) want[u] = (dx4[lv >> 3] >> (4 * (lv & 7))) & 15u;
            want[u] |= (v & 15u) << 5;  // the claimer's low bits ride on its claims
            mark_removed(v, lv, t);
            if (d4 != 0) {  // a vertex of degree 0 holds no alive edge
              if (coff) {
                const uint32_t b = lv / kCoffV, q = 4 + lv - b * kCoffV;
                const uint32_t *blk = myCoff + b * 16;
                const uint32_t w0 = blk[0], wa = blk[q >> 2], wb = blk[(q + 1) >> 2];
                const uint32_t la = (wa >> (8 * (q & 3))) & 255u;
                const uint32_t lb = (wb >> (8 * ((q + 1) & 3))) & 255u;
                st[u] = (w0 & ~kCoffEsc) + la;
                len[u] = lb - la;
                if (w0 & kCoffEsc) {
                  st[u] = a.offsets[v];
                  len[u] = a.offsets[v + 1] - st[u];
                }
              } else {
                st[u] = a.offsets[v];
                len[u] = a.offsets[v + 1] - st[u];
              }
            }
          }
        }
      };
      constexpr uint32_t kStride = kOT * kCV;
      uint32_t st[kCV], len[kCV], want[kCV];
      head((tid - lane) * kCV, st, len, want);
      for (uint32_t b = (tid - lane) * kCV; b < fcnt; b += kStride) {
        uint32_t e[kCV][kCE];
#pragma unroll
        for (int u = 0; u < kCV; ++u)
#pragma unroll
          for (int j = 0; j < kCE; ++j) e[u][j] = (uint32_t)j < len[u] ? a.inc[st[u] + j] : 0u;
        // the next pass's list bounds load while this pass's lists do
        uint32_t st2[kCV], len2[kCV], want2[kCV];
        head(b + kStride, st2, len2, want2);
        // want[u]: bits 0-4 the low bits to match (16 = all), bits 5-8 the
        // claimer's low bits
        uint32_t mine = 0;  // my claims in this pass
#pragma unroll
        for (int u = 0; u < kCV; ++u) {
          if (!XF || (want[u] & 31u) == 16) {
            mine += len[u];
            continue;
          }
          // the whole list's low bits, XORed with the dead ones': the alive edge's
          uint32_t x = want[u] & 15u;
#pragma unroll
          for (int j = 0; j < kCE; ++j)
            if ((uint32_t)j < len[u]) x ^= e[u][j] & 15u;
          for (uint32_t j = kCE; j < len[u]; ++j) x ^= a.inc[st[u] + j] & 15u;
          want[u] = (want[u] & ~31u) | x;
#pragma unroll
          for (int j = 0; j < kCE; ++j)
            if ((uint32_t)j < len[u] && (e[u][j] & 15u) == x) ++mine;
          for (uint32_t j = kCE; j < len[u]; ++j)
            if ((a.inc[st[u] + j] & 15u) == x) ++mine;
        }
        const uint32_t incl = wave_inclusive_scan(mine);
        uint32_t base = 0;
        if (lane == kWave - 1 && incl) base = atomicAdd(&s_c, incl);
        uint32_t pos = __shfl(base, kWave - 1, kWave) + incl - mine;
        auto claim = [&](uint32_t x, uint32_t wnt) {
          claims[pos++] = x | (wnt >> 5) << kNibShift;
          atomicAdd(&cnt[x / Eb], 1u);
        };
#pragma unroll
        for (int u = 0; u < kCV; ++u) {
          const uint32_t wl = want[u] & 31u;
#pragma unroll
          for (int j = 0; j < kCE; ++j)
            if ((uint32_t)j < len[u] && (wl == 16 || (e[u][j] & 15u) == wl))
              claim(e[u][j], want[u]);
          for (uint32_t j = kCE; j < len[u]; ++j) {
            const uint32_t x = a.inc[st[u] + j];
            if (wl == 16 || (x & 15u) == wl) claim(x, want[u]);
          }
        }
#pragma unroll
        for (int u = 0; u < kCV; ++u) {
          st[u] = st2[u];
          len[u] = len2[u];
          want[u] = want2[u];
        }
      }
      __syncthreads();
      const uint32_t nc = s_c;
      for (uint32_t d = tid; d < T; d += kOT) {
        const uint32_t c = cnt[d];
        cur[d] = c ? d * Eb * R + atomicAdd(&ctrl->qh_claim[d], c) : 0u;
      }
      __syncthreads();
      sorted_send(claims, nc, (uint32_t)m, Eb, T, a.qclaim, kIdMask);
    }
    // The barrier sums |F_t| and, in subtables mode, the number of workgroups
    // that still hold waiting bits (high word).  The barrier carries 48 bits:
    // |F_t| <= n < 2^32 and at most kOwnMaxT workgroups keep the sum below 2^43.
    pend -= sub ? fcnt : 0u;
    uint64_t tot;
    const uint64_t mine = sub ? ((uint64_t)(pend != 0u) << 32 | fcnt) : (uint64_t)fcnt;
    if (!sum_barrier(&ctrl->bar, T, slot, mine, &epoch, a.limit, &tot, ctrl->stamp)) return;
    const uint64_t vt = sub ? (tot & 0xffffffffull) : tot;
    const uint64_t waiting = sub ? (tot >> 32) : 0u;
    if (vt == 0 && waiting == 0) break;
    if (over) {
      // F_t (or a later subround's frontier) stays in the graph: the outputs
      // hold the state after max_rounds rounds.
      if (slot == 0 && tid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_EROUNDS);
      break;
    }
    if (vt == 0) continue;  // subtables mode: an empty subround
    last = t;
    removed += vt;
    if (slot == 0 && tid == 0) a.stats[2ull * (t - 1)] = vt;

    // ---- edge owners: the edges of F_t die once; decrements to their slots ---
    if (tid == 0) {
      s_n = dense ? 0u : ctrl->qh_claim[slot];
      if (!dense) ctrl->qh_claim[slot] = 0;
      s_w = 0;
    }
    for (uint32_t d = tid; d < T; d += kOT) cnt[d] = 0;
    __syncthreads();
    if (dense) {
      constexpr int kOU = R <= 4 ? 2 : 1;  // edges per thread whose loads are in flight
      // Scan my alive edges in order (coalesced rows), kOU per thread at a time
      // so that their loads overlap.  A dying edge's slots in F_t are replaced
      // by kNoVertex in the staged row: those vertices are already at degree 0.
      const uint32_t nE = (uint32_t)(e1 - e0);
      for (uint32_t b0 = 0; b0 < nE; b0 += kOU * kOT) {
        uint32_t ids[kOU][R];
        bool live[kOU];
#pragma unroll
        for (int u = 0; u < kOU; ++u) {
          const uint32_t le = b0 + u * kOT + tid;
          live[u] = le < nE && ((alive[le >> 5] >> (le & 31)) & 1u);
          if (live[u]) {
            const uint32_t *row = a.edges + (e0 + le) * R;
#pragma unroll
            for (int j = 0; j < R; ++j) ids[u][j] = row[j];
          }
        }
#pragma unroll
        for (int u = 0; u < kOU; ++u) {
          const uint32_t le = b0 + u * kOT + tid;
          bool die = false;
          if (live[u]) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
              const uint32_t x = ids[u][j];
              if (x < n && ((a.fbits[x >> 5] >> (x & 31)) & 1u)) {
                die = true;
                ids[u][j] = kNoVertex;
              }
            }
          }
          const uint32_t w = wave_append(die, &s_w);
          if (die) {
            atomicAnd(&alive[le >> 5], ~(1u << (le & 31)));
            mark_edge(le, t, 0u);
#pragma unroll
            for (int j = 0; j < R; ++j) {
              myStage[(uint64_t)w * R + j] = dmsg(ids[u][j], e0 + le);
              if (ids[u][j] < n) atomicAdd(&cnt[ids[u][j] / Vb], 1u);
            }
          }
        }
      }
    }
    uint32_t won = 0;
    if (!dense) {
      // Sparse: mark the claimed edges, then take the claimed edges that are
      // still alive in edge order (so rows are read and rounds written in
      // order), one per thread, each placed at its rank in the stage.
      const uint32_t nclaims = s_n;
      if (nclaims <= (uint32_t)kOT) {
        // few claims: one per thread, in arrival order
        uint32_t e = 0, cn = kNib;
        bool win = false;
        if (tid < nclaims) {
          const uint32_t c = myClaims[tid];
          e = c & kIdMask;
          cn = c >> kNibShift;
          const uint32_t le = e - (uint32_t)e0;
          const uint32_t bit = 1u << (le & 31);
          win = (atomicAnd(&alive[le >> 5], ~bit) & bit) != 0;
        }
        const uint32_t w = wave_append(win, &s_w);
        if (win) {
          mark_edge(e - (uint32_t)e0, t, 0u);
          const uint32_t *row = a.edges + (uint64_t)e * R;
          uint32_t ids[R];
#pragma unroll
          for (int q = 0; q < R; ++q) ids[q] = row[q];
          stage_row(w, e, ids, cn);  // cn: this claim's claimer, which leaves now
        }
        __syncthreads();
        won = s_w;
      }
      for (uint32_t i0 = tid; nclaims > (uint32_t)kOT && i0 < nclaims; i0 += kLU * kOT) {
        uint32_t e[kLU];
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
          const uint32_t i = i0 + u * kOT;
          e[u] = i < nclaims ? myClaims[i] : kNoVertex;
        }
        // a claim of an alive edge sets its claimed bit and notes the
        // claimer's low bits in the edge's round nibble (0 while alive); a
        // second claim makes the note kNib (no slot skipped)
#pragma unroll
        for (int u = 0; u < kLU; ++u) {
          if (e[u] == kNoVertex) continue;
          const uint32_t le = (e[u] & kIdMask) - (uint32_t)e0;
          const uint32_t bit = 1u << (le & 31);
          if (!(alive[le >> 5] & bit)) continue;
          const uint32_t first = !(atomicOr(&claimed[le >> 5], bit) & bit);
          atomicOr(&er4[le >> 3], (first ? e[u] >> kNibShift : kNib) << (4 * (le & 7)));
        }
      }
      __syncthreads();
      const uint32_t nw = nclaims > (uint32_t)kOT ? (uint32_t)((e1 - e0 + 31) / 32) : 0u;
      for (uint32_t w0 = 0; w0 < nw; w0 += kOT) {
        const uint32_t w = w0 + tid;
        uint32_t dying = 0;
        if (w < nw) {
          dying = claimed[w] & alive[w];
          claimed[w] = 0;
          alive[w] &= ~dying;
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan<kOT>(__popc(dying), &tot, scan_lds);
        s_start[tid] = dying;
        s_pre[tid] = ex;
        __syncthreads();
        constexpr int kEU = R <= 4 ? 2 : 1;  // dying edges per thread whose rows are in flight
        for (uint32_t j0 = tid; j0 < tot; j0 += kEU * kOT) {
          uint64_t e[kEU];
          uint32_t ids[kEU][R];
#pragma unroll
          for (int u = 0; u < kEU; ++u) {
            const uint32_t j = j0 + u * kOT;
            if (j < tot) {
              uint32_t lo = 0, hi = kOT;
              while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (s_pre[mid] <= j) lo = mid; else hi = mid;
              }
              e[u] = e0 + 32ull * (w0 + lo) + nth_set_bit(s_start[lo], j - s_pre[lo]);
              const uint32_t *row = a.edges + e[u] * R;
#pragma unroll
              for (int q = 0; q < R; ++q) ids[u][q] = row[q];
            }
          }
#pragma unroll
          for (int u = 0; u < kEU; ++u) {
            const uint32_t j = j0 + u * kOT;
            if (j >= tot) continue;
            const uint32_t le = (uint32_t)(e[u] - e0);
            const uint32_t cn = (er4[le >> 3] >> (4 * (le & 7))) & kNib;
            mark_edge(le, t, cn);
            stage_row(won + j, e[u], ids[u], cn);
          }
        }
        won += tot;
        __syncthreads();
      }
    } else {
      __syncthreads();
      won = s_w;
    }
    for (uint32_t d = tid; d < T; d += kOT) {
      const uint32_t c = cnt[d];
      const uint32_t dv = d * Vb < n ? d * Vb : n;
      cur[d] = c ? a.offsets[dv] + atomicAdd(&ctrl->qh_dec[d], c) : 0u;
    }
    __syncthreads();
    sorted_send(myStage, won * R, n, Vb, T, a.qdec, XF ? kIdMask : ~0u);
    uint64_t et;
    if (!sum_barrier(&ctrl->bar, T, slot, won, &epoch, a.limit, &et, ctrl->stamp)) return;
    if (slot == 0 && tid == 0) a.stats[2ull * (t - 1) + 1] = et;
    alive_m -= et;
    prev_v = vt;

    // ---- vertex owners: apply decrements, collect F_{t+1} --------------------
    if (tid == 0) {
      s_w = ctrl->qh_dec[slot];
      ctrl->qh_dec[slot] = 0;
      s_n = 0;
    }
    __syncthreads();
    const uint32_t ndec = s_w;
    for (uint32_t i0 = tid; i0 < ndec; i0 += kLU * kOT) {
      uint32_t us[kLU];
#pragma unroll
      for (int q = 0; q < kLU; ++q) {
        const uint32_t i = i0 + q * kOT;
        us[q] = i < ndec ? myDecs[i] : kNoVertex;
      }
#pragma unroll
      for (int q = 0; q < kLU; ++q) {
        if (us[q] == kNoVertex) continue;
        const uint32_t u = XF ? us[q] & kIdMask : us[q];
        const uint32_t lv = u - v0;
        // a vertex removed this round (its edges die with it) keeps its round
        if ((gone[lv >> 5] >> (lv & 31)) & 1u) continue;
        const uint32_t sh = 4 * (lv & 7);
        if (XF) atomicXor(&dx4[lv >> 3], (us[q] >> kNibShift) << sh);
        uint32_t old;
        if (((deg4[lv >> 3] >> sh) & kNib) == kNib)
          old = atomicSub(&a.deg[u], 1u);
        else
          old = (atomicSub(&deg4[lv >> 3], 1u << sh) >> sh) & kNib;
        if (old == k) {
          atomicOr(&fbl[lv >> 5], 1u << (lv & 31));
          const uint32_t p = wave_append(true, &s_n);  // the lanes here
          if (p < (uint32_t)kOT) s_start[p] = u;
        }
      }
    }
    __syncthreads();
    if (sub) pend += s_n;
  }

  // ---- epilogue: removal rounds and final degrees, written in order ----------
  for (uint32_t v = v0 + tid; v < v1; v += kOT) {
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
  for (uint64_t e = e0 + tid; e < e1; e += kOT) {
    const uint32_t le = (uint32_t)(e - e0);
    const uint32_t x = (er4[le >> 3] >> (4 * (le & 7))) & kNib;
    if (x != kNib) a.er[e] = x;
  }
  if (slot == 0 && tid == 0) {
    ctrl->rounds = last;
    ctrl->removed = removed;
    ctrl->team = T;
    ctrl->mode = kModeOwnerDone;
  }
}

// ===========================================================================
// Global engine.

template <int R>
__global__ void __launch_bounds__(kBlock) k_peel_persistent(PeelArgs a) {
  __shared__ uint32_t q[kQueue];
  __shared__ uint32_t qn;
  __shared__ uint32_t s_base;
  __shared__ uint32_t lds[kBlock / kWave + 1];

  PeelCtrl *ctrl = a.ctrl;
  // Runs only when the owner engine declined this input.
  if (__hip_atomic_load(&ctrl->mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kModeGlobal)
    return;
  uint32_t slot, nblocks;
  if (!team_join(&ctrl->team_glob, a.quiet, a.team_limit, &slot, &nblocks)) return;
  const uint64_t gtid = (uint64_t)slot * kBlock + threadIdx.x;
  const uint64_t gsize = (uint64_t)nblocks * kBlock;
  // Subtables mode: the list of round t holds every waiting vertex; those whose
  // subround (vertex_round, set when they fell below k) is not t move on to the
  // next list unchanged.
  const bool sub = a.subtables != 0;

  // ---- phase 0 ------------------------------------------------------------
  for (uint64_t e = gtid; e < a.m; e += gsize) a.er[e] = 0;
  for (uint64_t i = gtid; i < 2ull * a.max_rounds; i += gsize) a.stats[i] = 0;
  for (uint64_t t0 = (uint64_t)slot * kDenseTile; t0 < a.n; t0 += (uint64_t)nblocks * kDenseTile) {
    const uint64_t base = t0 + (uint64_t)threadIdx.x * kDenseItems;
    uint32_t low = 0, cnt = 0;
#pragma unroll
    for (int i = 0; i < kDenseItems; ++i) {
      const uint64_t v = base + i;
      if (v < a.n) {
        const uint32_t is_low = a.deg[v] < a.k ? 1u : 0u;
        // the (sub)round in which v leaves: 1, or its subtable's first subround
        a.vr[v] = is_low ? (sub ? subtable_of_vertex(a, R, (uint32_t)v) + 1u : 1u) : 0u;
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
  uint32_t last = 0;
  uint64_t removed = 0;
  for (;; ++t) {
    const uint32_t size = atomic_load_u32(&ctrl->fcount[t % 3]);
    const uint32_t *cur = (t & 1u) ? a.fa : a.fb;
    if (size == 0) break;
    if (t > a.max_rounds) {
      // Leave the state after max_rounds rounds: F_t (and, with subtables, every
      // waiting vertex) stays in the graph.
      for (uint64_t i = gtid; i < size; i += gsize) a.vr[cur[i]] = 0;
      if (gtid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_EROUNDS);
      break;
    }
    uint32_t *nxt = (t & 1u) ? a.fb : a.fa;
    uint32_t *ncount = &ctrl->fcount[(t + 1) % 3];
    if (gtid == 0) ctrl->fcount[(t + 2) % 3] = 0;
    if (threadIdx.x == 0) qn = 0;
    __syncthreads();

    auto push = [&](uint32_t u) {
      const uint32_t slotq = atomicAdd(&qn, 1u);
      if (slotq < kQueue)
        q[slotq] = u;
      else
        nxt[atomicAdd(ncount, 1u)] = u;
    };
    const uint32_t jt = (t - 1) % R;
    uint32_t wins = 0, taken = 0;
    for (uint64_t i = gtid; i < size; i += gsize) {
      const uint32_t v = cur[i];
      if (sub && a.vr[v] != t) {  // waits for its subtable's subround
        push(v);
        continue;
      }
      ++taken;
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
            // next round, or the next subround of u's subtable (a full round
            // later when that is the subtable of this subround)
            a.vr[u] = sub ? t + (subtable_of_vertex(a, R, u) + R - jt - 1) % R + 1u : t + 1u;
            push(u);
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
    const uint32_t bt = block_sum(taken, lds);
    if (threadIdx.x == 0 && bw) atomicAdd(&a.stats[2ull * (t - 1) + 1], (uint64_t)bw);
    if (threadIdx.x == 0 && bt) atomicAdd(&a.stats[2ull * (t - 1)], (uint64_t)bt);
    if (!grid_barrier(&ctrl->sync, nblocks, a.limit, ctrl->stamp)) return;
    const uint64_t vt = __hip_atomic_load(&a.stats[2ull * (t - 1)], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    if (vt) {
      last = t;
      removed += vt;
    }
  }
  if (gtid == 0) {
    ctrl->rounds = last;
    ctrl->removed = removed;
    ctrl->team = nblocks;
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
  if (ctrl->sync.abort || ctrl->bar.abort || ctrl->mode == kModeUndecided ||
      ctrl->mode == kModeRetry)
    flags |= PEEL_FLAG_TIMEOUT;
  summary[0] = rounds;
  summary[1] = last_e;
  summary[2] = flags;
  summary[3] = static_cast<uint32_t>(n - ctrl->removed);
  summary[4] = ctrl->team;
  summary[5] = summary[6] = summary[7] = 0;
}

struct Layout {
  size_t ctrl, fa, fb, qclaim, qdec, stage, fbits, coff, total;
  uint64_t coff_blocks;
};

Layout layout(uint32_t n, uint64_t m, uint32_t r) {
  const uint64_t g = (uint64_t)device_info().cus + 64;  // owner grid upper bound
  Layout L{};
  L.ctrl = align_up(sizeof(PeelCtrl));
  L.fa = align_up((size_t)n * 4);
  L.fb = align_up((size_t)n * 4);
  L.qclaim = align_up((size_t)r * (m + g) * 4);
  L.qdec = align_up((size_t)r * m * 4 + 4);
  L.stage = align_up((size_t)r * (m + g) * 4);
  L.fbits = align_up(((size_t)n + 31) / 32 * 4 + 4);
  // T workgroups of ceil(Vb / kCoffV) blocks, Vb <= n / T + 32: at most n / kCoffV + 2T
  L.coff_blocks = (uint64_t)n / kCoffV + 2 * g + 2;
  L.coff = align_up((size_t)L.coff_blocks * 64);
  L.total = L.ctrl + L.fa + L.fb + L.qclaim + L.qdec + L.stage + L.fbits + L.coff;
  return L;
}

template <int R>
peel_status launch(PeelArgs &a, hipStream_t s) {
  const DeviceInfo &dev = device_info();
  // owner engine: one workgroup per CU (its LDS use allows no more)
  const unsigned og = static_cast<unsigned>(dev.cus < (int)kOwnMaxT ? dev.cus : (int)kOwnMaxT);
  // the claim filter's LDS fits when each workgroup owns at most kOwnMaxVX vertices
  const uint64_t vb = (((uint64_t)a.n + og - 1) / og + 31) & ~31ull;
  const bool xf = vb <= kOwnMaxVX && a.claims_all != 1;
  if (dev.debug) std::fprintf(stderr, "[peel] owner grid %u, claim filter %d\n", og, (int)xf);
  if (xf) {
    hipLaunchKernelGGL((k_peel_owner<R, true>), dim3(og), dim3(kOT), 0, s, a);
    PEEL_HIP_TRY(hipGetLastError());
    // runs only if the team that formed was too small for the claim filter
    PeelArgs b = a;
    b.retry = 1;
    hipLaunchKernelGGL((k_peel_owner<R, false>), dim3(og), dim3(kOT), 0, s, b);
  } else {
    hipLaunchKernelGGL((k_peel_owner<R, false>), dim3(og), dim3(kOT), 0, s, a);
  }
  PEEL_HIP_TRY(hipGetLastError());
  // global engine: runs only if the owner engine declined
  const void *fn = reinterpret_cast<const void *>(&k_peel_persistent<R>);
  const int cap = coresident_blocks(fn, kBlock, 0);
  uint64_t want = ((uint64_t)a.n + kDenseTile - 1) / kDenseTile;
  const uint64_t want_m = (a.m + 4ull * kBlock - 1) / (4ull * kBlock);
  if (want_m > want) want = want_m;
  if (want < 1) want = 1;
  const unsigned grid = static_cast<unsigned>(want < (uint64_t)cap ? want : (uint64_t)cap);
  if (dev.debug) std::fprintf(stderr, "[peel] global grid %u (cap %d)\n", grid, cap);
  hipLaunchKernelGGL(k_peel_persistent<R>, dim3(grid), dim3(kBlock), 0, s, a);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

}  // namespace
}  // namespace peel

using namespace peel;

extern "C" size_t peel_kcore_workspace(uint32_t n, uint64_t m, uint32_t r) {
  return layout(n, m, r).total;
}

namespace peel {
namespace {

peel_status peel_run(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n, uint32_t k,
                     const uint32_t *offsets, const uint32_t *inc, uint32_t *deg,
                     uint32_t *vertex_round, uint32_t *edge_round, uint64_t *round_stats,
                     uint32_t max_rounds, uint32_t *summary, void *ws, size_t ws_bytes,
                     void *stream, bool subtables) {
  if (r < 2 || r > 8 || n == 0 || k == 0 || max_rounds == 0) return PEEL_EINVAL;
  if (m * (uint64_t)r >= (1ull << 32)) return PEEL_EINVAL;
  if ((m && (!edges || !inc || !edge_round)) || !offsets || !deg || !vertex_round ||
      !round_stats || !summary || !ws)
    return PEEL_EINVAL;
  const Layout L = layout(n, m, r);
  if (ws_bytes < L.total) return PEEL_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ws);
  PeelArgs a;
  a.ctrl = reinterpret_cast<PeelCtrl *>(base);
  base += L.ctrl;
  a.fa = reinterpret_cast<uint32_t *>(base);
  base += L.fa;
  a.fb = reinterpret_cast<uint32_t *>(base);
  base += L.fb;
  a.qclaim = reinterpret_cast<uint32_t *>(base);
  base += L.qclaim;
  a.qdec = reinterpret_cast<uint32_t *>(base);
  base += L.qdec;
  a.stage = reinterpret_cast<uint32_t *>(base);
  base += L.stage;
  a.fbits = reinterpret_cast<uint32_t *>(base);
  base += L.fbits;
  a.coff = reinterpret_cast<uint32_t *>(base);
  a.coff_blocks = L.coff_blocks;
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
  a.limit = barrier_limit_ticks();
  a.team_limit = device_info().team_limit_ticks;
  a.quiet = device_info().team_quiet_ticks;
  const char *engine = std::getenv("PEEL_ENGINE");
  a.force_global = (engine && std::strcmp(engine, "global") == 0) ? 1u : 0u;
  const char *rounds = std::getenv("PEEL_ROUNDS");
  a.round_policy = !rounds ? kRoundsSparse
                   : std::strcmp(rounds, "dense") == 0 ? kRoundsDense
                   : std::strcmp(rounds, "auto") == 0  ? kRoundsAuto
                                                        : kRoundsSparse;
  a.subtables = subtables ? 1u : 0u;
  const char *claims = std::getenv("PEEL_CLAIMS");
  a.claims_all = !claims ? 0u
                 : std::strcmp(claims, "all") == 0   ? 1u
                 : std::strcmp(claims, "retry") == 0 ? 2u
                                                     : 0u;
  a.retry = 0;
  a.sub_lo[0] = 0;
  for (uint32_t j = 0; j < 8; ++j)
    a.sub_lo[j + 1] = a.sub_lo[j] + (j < r ? n / r + (j < n % r ? 1u : 0u) : 0u);

  hipLaunchKernelGGL(k_peel_init, dim3(1), dim3(256), 0, s, a.ctrl,
                     barrier_slots() ? 1u : 0u);
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

}  // namespace
}  // namespace peel

extern "C" peel_status peel_kcore(const uint32_t *edges, uint64_t m, uint32_t r, uint32_t n,
                                  uint32_t k, const uint32_t *offsets, const uint32_t *inc,
                                  uint32_t *deg, uint32_t *vertex_round, uint32_t *edge_round,
                                  uint64_t *round_stats, uint32_t max_rounds, uint32_t *summary,
                                  void *ws, size_t ws_bytes, void *stream) {
  return peel_run(edges, m, r, n, k, offsets, inc, deg, vertex_round, edge_round, round_stats,
                  max_rounds, summary, ws, ws_bytes, stream, false);
}

extern "C" peel_status peel_kcore_subtables(const uint32_t *edges, uint64_t m, uint32_t r,
                                            uint32_t n, uint32_t k, const uint32_t *offsets,
                                            const uint32_t *inc, uint32_t *deg,
                                            uint32_t *vertex_round, uint32_t *edge_round,
                                            uint64_t *round_stats, uint32_t max_rounds,
                                            uint32_t *summary, void *ws, size_t ws_bytes,
                                            void *stream) {
  return peel_run(edges, m, r, n, k, offsets, inc, deg, vertex_round, edge_round, round_stats,
                  max_rounds, summary, ws, ws_bytes, stream, true);
}

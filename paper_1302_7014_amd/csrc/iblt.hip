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
#include <cstring>
#include <type_traits>

#include "common.hpp"
#include "scan.hpp"
#include "host.hpp"

namespace peel {
namespace {

struct Hash {
  uint64_t base[8];
  uint64_t size[8];
  uint64_t salt[8];
  uint64_t salt_c;
  uint32_t r;
};

__host__ __device__ inline Hash make_hash(const iblt_desc &d) {
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

// make_hash for a table whose r is the compile-time R.  Every index is then a
// constant, so a kernel that builds the hash itself keeps it in registers; with
// a run-time r the arrays are indexed dynamically and land in scratch memory,
// which every cell_of then reads.
template <int R>
__device__ inline Hash make_hash_fixed(const iblt_desc &d) {
  Hash h{};
  uint64_t acc = 0;
  h.r = R;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    h.size[j] = d.ncells / R + ((uint64_t)j < d.ncells % R ? 1 : 0);
    h.base[j] = acc;
    acc += h.size[j];
    h.salt[j] = splitmix64(d.seed, (uint64_t)j);
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
    k_insert(Hash h, iblt_cell *cells, const uint64_t *__restrict__ keys, uint64_t nkeys,
             int32_t sign) {
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < nkeys;
       i += (uint64_t)gridDim.x * kBlock) {
    const uint64_t x = keys[i];
    const uint64_t c = check_of(h, x);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      iblt_cell *cell = cells + cell_of(h, j, x);
      atomicAdd(&cell->count, sign);
      atomicXor(reinterpret_cast<unsigned long long *>(&cell->key_sum), (unsigned long long)x);
      atomicXor(reinterpret_cast<unsigned long long *>(&cell->hash_sum), (unsigned long long)c);
    }
  }
}

// ---------------------------------------------------------------------------
// Plain 32-byte store of an empty cell (the cell a key was listed from holds
// that key alone, so no other key touches it in the same round).
__device__ inline void clear_cell(iblt_cell *cell) {
  uint4 *p = reinterpret_cast<uint4 *>(cell);
  p[0] = make_uint4(0u, 0u, 0u, 0u);
  p[1] = make_uint4(0u, 0u, 0u, 0u);
}

__device__ inline void load_cell(const iblt_cell *cell, int32_t *cnt, uint64_t *ks, uint64_t *hs) {
  const uint4 *p = reinterpret_cast<const uint4 *>(cell);
  const uint4 a = p[0];
  const uint4 b = p[1];
  *cnt = static_cast<int32_t>(a.x);
  *ks = (uint64_t)a.z | ((uint64_t)a.w << 32);
  *hs = (uint64_t)b.x | ((uint64_t)b.y << 32);
}

// ---------------------------------------------------------------------------
// Binned update (iblt_update).  Every key makes r cell updates.  They are
// counting-sorted by super-bucket of kUSuper cells: one entry per (key, cell),
// the key in ekey and the cell's place in its super-bucket in eloc.  Then each
// block of kUBlk cells is loaded into LDS, takes the entries of its
// super-bucket whose place falls in the block with LDS atomics, and is written
// back in order.  No device atomic per update: the table is read and written
// once, and each super-bucket's entries, read by its kUPer blocks on one XCD,
// come from L2 after the first.  Each cell hash is computed once per entry in
// the count and the scatter, and the checksum once per entry in the apply.
constexpr int kUSuperShift = 14;                  // 16384 cells per super-bucket
constexpr int kUBlkShift = 12;                    // 4096 cells per apply block
constexpr uint32_t kUBlk = 1u << kUBlkShift;
constexpr uint32_t kUPer = 1u << (kUSuperShift - kUBlkShift);  // apply blocks per super-bucket
constexpr uint32_t kUMaxSuper = 1024;             // up to 2^24 cells
constexpr uint64_t kUTile = 8192;                 // keys per count/scatter tile
constexpr uint32_t kUChunk = 8192;                // entries sorted in LDS per scatter chunk
constexpr int kUT = 1024;                         // threads per workgroup

// hist[s * ntiles + tile] = entries of the tile's keys in super-bucket s.
template <int R>
__global__ void __launch_bounds__(kUT)
    k_upd_count(Hash h, const uint64_t *__restrict__ keys, uint64_t nkeys, uint32_t nsb,
                uint32_t ntiles, uint32_t *hist, const unsigned long long *nkeys_dev) {
  __shared__ uint32_t cnt[kUMaxSuper];
  if (nkeys_dev) nkeys = *nkeys_dev;  // the grid is sized for the most keys there can be
  for (uint32_t b = threadIdx.x; b < nsb; b += kUT) cnt[b] = 0;
  __syncthreads();
  const uint32_t tile = xcd_item(blockIdx.x, ntiles);
  const uint64_t k0 = (uint64_t)tile * kUTile;
  const uint64_t k1 = k0 + kUTile < nkeys ? k0 + kUTile : nkeys;
  constexpr int kU = 4;
  for (uint64_t i0 = k0 + threadIdx.x; i0 < k1; i0 += kU * kUT) {
    uint64_t x[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint64_t i = i0 + (uint64_t)u * kUT;
      x[u] = i < k1 ? keys[i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (i0 + (uint64_t)u * kUT >= k1) continue;
#pragma unroll
      for (int j = 0; j < R; ++j) atomicAdd(&cnt[cell_of(h, j, x[u]) >> kUSuperShift], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nsb; b += kUT) hist[(uint64_t)b * ntiles + tile] = cnt[b];
}

// Each tile writes its entries into its run of every super-bucket, whose
// starts are the scanned hist.  kUChunk entries at a time are ranked per
// super-bucket, sorted in LDS and stored in sorted order.
template <int R>
__global__ void __launch_bounds__(kUT)
    k_upd_scatter(Hash h, const uint64_t *__restrict__ keys, uint64_t nkeys, uint32_t nsb,
                  uint32_t ntiles, const uint32_t *__restrict__ hist, uint64_t *ekey,
                  uint16_t *eloc, const unsigned long long *nkeys_dev) {
  if (nkeys_dev) nkeys = *nkeys_dev;
  constexpr int kKPT = (int)(kUChunk / kUT) / R;      // keys per thread per chunk
  constexpr uint32_t kCK = (uint32_t)kKPT * kUT;      // keys per chunk
  static_assert(kKPT >= 1 && kCK * R <= kUChunk, "a chunk's entries fit in LDS");
  __shared__ uint64_t sk[kUChunk];
  __shared__ uint16_t sl[kUChunk];
  __shared__ uint16_t ss[kUChunk];
  __shared__ uint32_t cur[kUMaxSuper];
  __shared__ uint32_t cnt[kUMaxSuper];
  __shared__ uint32_t st[kUMaxSuper];
  __shared__ uint32_t lds[kUT / kWave + 1];
  const uint32_t tid = threadIdx.x;
  const uint32_t tile = xcd_item(blockIdx.x, ntiles);
  for (uint32_t b = tid; b < nsb; b += kUT) cur[b] = hist[(uint64_t)b * ntiles + tile];
  const uint64_t k0 = (uint64_t)tile * kUTile;
  const uint64_t k1 = k0 + kUTile < nkeys ? k0 + kUTile : nkeys;
  for (uint64_t c0 = k0; c0 < k1; c0 += kCK) {
    for (uint32_t b = tid; b < nsb; b += kUT) cnt[b] = 0;
    __syncthreads();
    uint64_t x[kKPT];
    uint32_t cl[kKPT][R], rk[kKPT][R];
#pragma unroll
    for (int u = 0; u < kKPT; ++u) {
      const uint64_t i = c0 + (uint64_t)u * kUT + tid;
      x[u] = i < k1 ? keys[i] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kKPT; ++u) {
      if (c0 + (uint64_t)u * kUT + tid >= k1) continue;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        cl[u][j] = cell_of(h, j, x[u]);
        rk[u][j] = atomicAdd(&cnt[cl[u][j] >> kUSuperShift], 1u);
      }
    }
    __syncthreads();
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kUT>(tid < nsb ? cnt[tid] : 0u, &tot, lds);
    if (tid < nsb) st[tid] = ex;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kKPT; ++u) {
      if (c0 + (uint64_t)u * kUT + tid >= k1) continue;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t sb = cl[u][j] >> kUSuperShift;
        const uint32_t i = st[sb] + rk[u][j];
        sk[i] = x[u];
        sl[i] = static_cast<uint16_t>(cl[u][j] & ((1u << kUSuperShift) - 1));
        ss[i] = static_cast<uint16_t>(sb);
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < tot; i += kUT) {
      const uint32_t b = ss[i];
      const uint32_t o = cur[b] + (i - st[b]);
      ekey[o] = sk[i];
      eloc[o] = sl[i];
    }
    __syncthreads();
    for (uint32_t b = tid; b < nsb; b += kUT) cur[b] += cnt[b];
  }
}

// One workgroup per block of kUBlk cells (the kUPer blocks of a super-bucket
// on one XCD): the cells in LDS, the super-bucket's entries whose place falls
// in the block applied with LDS atomics, the cells written back.  The
// reserved words are kept as they were.
template <int R>
__global__ void __launch_bounds__(kUT)
    k_upd_apply(Hash h, iblt_cell *cells, uint64_t ncells, const uint64_t *__restrict__ ekey,
                const uint16_t *__restrict__ eloc, const uint32_t *__restrict__ hist,
                uint32_t nsb, uint32_t ntiles, const uint32_t *total, int32_t sign) {
  __shared__ int32_t ccount[kUBlk];
  __shared__ unsigned long long cks[kUBlk];
  __shared__ unsigned long long chs[kUBlk];
  const uint32_t item = xcd_item(blockIdx.x, nsb * kUPer);
  const uint32_t sbi = item / kUPer, q = item % kUPer;
  const uint64_t c_lo = ((uint64_t)sbi << kUSuperShift) + (uint64_t)q * kUBlk;
  if (c_lo >= ncells) return;  // every thread of the block leaves
  const uint32_t nc = ncells - c_lo < kUBlk ? static_cast<uint32_t>(ncells - c_lo) : kUBlk;
  for (uint32_t i = threadIdx.x; i < nc; i += kUT) {
    int32_t cn;
    uint64_t ks, hs;
    load_cell(cells + c_lo + i, &cn, &ks, &hs);
    ccount[i] = cn;
    cks[i] = ks;
    chs[i] = hs;
  }
  __syncthreads();
  const uint32_t lo = hist[(uint64_t)sbi * ntiles];
  const uint32_t hi = sbi + 1 < nsb ? hist[(uint64_t)(sbi + 1) * ntiles] : *total;
  constexpr int kU = 8;
  for (uint32_t i0 = lo + threadIdx.x; i0 < hi; i0 += kU * kUT) {
    uint32_t l[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t i = i0 + u * kUT;
      l[u] = i < hi ? eloc[i] : 0xffffu;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if ((l[u] >> kUBlkShift) != q) continue;  // another block's cell, or past the end
      const uint64_t x = ekey[i0 + u * kUT];
      const uint32_t c = l[u] & (kUBlk - 1);
      atomicAdd(&ccount[c], sign);
      atomicXor(&cks[c], (unsigned long long)x);
      atomicXor(&chs[c], (unsigned long long)check_of(h, x));
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nc; i += kUT) {
    uint4 *p = reinterpret_cast<uint4 *>(cells + c_lo + i);
    const uint4 a = p[0];
    const uint4 b = p[1];
    const uint64_t ks = cks[i], hs = chs[i];
    p[0] = make_uint4(static_cast<uint32_t>(ccount[i]), a.y, static_cast<uint32_t>(ks),
                      static_cast<uint32_t>(ks >> 32));
    p[1] = make_uint4(static_cast<uint32_t>(hs), static_cast<uint32_t>(hs >> 32), b.z, b.w);
  }
}


// True when cell c (already read as cnt/ks/hs) is pure and it is the owner of
// its key: no cell of the key in a lower subtable is a pure cell of that key.
// Sets *bad for a count-1 cell whose checksum does not match.
// SIGNED (tables holding deletions too): a count of -1 is pure as well, and a
// count of +-1 with a wrong checksum is an ordinary cell holding several keys.
// may(l) == false promises that cell l is not pure, so its read is skipped.
struct AnyCell {
  __device__ bool operator()(uint32_t) const { return true; }
};

template <int R, bool SIGNED = false, typename May = AnyCell>
__device__ inline bool owns(const Hash &h, const iblt_cell *cells, uint32_t c, int32_t cnt,
                            uint64_t ks, uint64_t hs, uint32_t *bad, May may = May()) {
  if (cnt != 1 && !(SIGNED && cnt == -1)) return false;
  const uint64_t hx = check_of(h, ks);
  if (hs != hx) {
    if (!SIGNED) *bad = 1;
    return false;
  }
  const uint32_t j = subtable_of(h, c);
#pragma unroll
  for (int i = 0; i < R - 1; ++i) {
    if (i >= (int)j) break;
    const uint32_t l = cell_of(h, i, ks);
    if (!may(l)) continue;
    int32_t oc;
    uint64_t ok, oh;
    load_cell(cells + l, &oc, &ok, &oh);
    if ((oc == 1 || (SIGNED && oc == -1)) && ok == ks && oh == hx) return false;
  }
  return true;
}

// Runs the owner test on cells cell_at(i) for i = i0 + tid, i0 + tid + nt, ...
// below i1.  kDetU cells per lane are loaded before any is tested, so a lane has
// kDetU loads in flight: with one, a scan of a table in HBM is bound by load
// latency rather than bandwidth.  take(key, cell) gets every owned key; *sum
// gets the counts of the cells read.  may: as for owns.
constexpr int kDetU = 4;
template <int R, bool SIGNED, typename At, typename Take, typename May = AnyCell>
__device__ inline void detect_cells(const Hash &h, const iblt_cell *cells, uint64_t i0, uint64_t i1,
                                    uint32_t tid, uint32_t nt, At cell_at, Take take,
                                    uint32_t *bad, long long *sum, May may = May()) {
  for (uint64_t ib = i0 + tid; ib < i1; ib += (uint64_t)kDetU * nt) {
    uint32_t c[kDetU];
    int32_t cnt[kDetU];
    uint64_t ks[kDetU], hs[kDetU];
#pragma unroll
    for (int u = 0; u < kDetU; ++u) {
      const uint64_t i = ib + (uint64_t)u * nt;
      c[u] = 0;
      cnt[u] = 0;
      ks[u] = hs[u] = 0;
      if (i < i1) {
        c[u] = cell_at(i);
        load_cell(cells + c[u], &cnt[u], &ks[u], &hs[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < kDetU; ++u) {
      *sum += cnt[u];  // 0 for the places past i1
      if (ib + (uint64_t)u * nt < i1 && owns<R, SIGNED>(h, cells, c[u], cnt[u], ks[u], hs[u], bad, may))
        take(ks[u], c[u]);
    }
  }
}

// Deletes key x from its R cells; the cell it was listed from (c_own) is simply
// cleared.  Calls push(c) for every cell whose count goes 2 -> 1.
// SIGNED: x leaves with its sign (count -= sign) and a cell whose count lands on
// +-1 is pushed (signed counts need not fall monotonically).
template <int R, bool SIGNED = false, typename Push>
__device__ inline void delete_key(const Hash &h, iblt_cell *cells, uint64_t x, uint32_t c_own,
                                  Push push, int32_t sign = 1) {
  const uint64_t hx = check_of(h, x);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const uint32_t c = cell_of(h, j, x);
    iblt_cell *cell = cells + c;
    if (c == c_own) {
      clear_cell(cell);
      continue;
    }
    const int32_t old = atomicSub(&cell->count, sign);
    atomicXor(reinterpret_cast<unsigned long long *>(&cell->key_sum), (unsigned long long)x);
    atomicXor(reinterpret_cast<unsigned long long *>(&cell->hash_sum), (unsigned long long)hx);
    if (SIGNED ? (old - sign == 1 || old - sign == -1) : old == 2) push(c);
  }
}

// ===========================================================================
// Multi-workgroup listing of one table (persistent kernel, run-time team).
//
// Each workgroup keeps the keys it found in this round's detect phase in its
// own staging slice (with a shared overflow region), applies exactly those
// keys, and keeps the cells it pushed as its own candidates for the next
// detect phase.  The hierarchical barrier after detect sums the staged counts
// and gives each workgroup its exclusive prefix, which places its keys in
// out_keys without any contended atomic.

constexpr int kLT = 1024;  // threads per listing workgroup

struct ListCtrl {
  SumBar bar;
  Team team;
  uint32_t flags;
  uint32_t rounds;
  uint32_t team_size;
  uint32_t pad;
  uint64_t listed;
  unsigned long long count_sum;  // sum of all counts at the start (two's complement)
  uint32_t ovf_own[2];           // overflow keys found by detect for round u: [u & 1]
  uint32_t ovf_cand[2];          // overflow candidates pushed by apply of round u: [u & 1]
  uint32_t qn[3];                // subtables mode: candidate queue of subround s has qn[s % 3]
  uint32_t pad2;
  unsigned long long nonempty;   // signed listing: cells left non-zero
  unsigned long long first_keys; // binned first round: the keys it listed
  uint64_t stamp[256];           // wall clock at each barrier generation (diagnostic)
};

struct ListArgs {
  Hash h;
  iblt_cell *cells;
  uint64_t *out;
  uint64_t out_cap;
  uint64_t *stats;
  uint64_t *skeys;   // G * cb staged keys
  uint32_t *scells;  // G * cb cells they were found in
  uint32_t *cand;    // G * cb candidate cells
  uint64_t *okeys;   // ncells overflow keys
  uint32_t *ocells;  // ncells
  uint32_t *ocand;   // 2 * ncells overflow candidates
  int8_t *signs;     // signed listing: the sign of each listed key
  uint32_t signed_list;
  ListCtrl *ctrl;
  uint64_t limit;
  uint64_t quiet;
  uint64_t team_limit;
  uint32_t ncells;
  uint32_t max_rounds;
  uint32_t cb;
  uint32_t grid;
  uint32_t first_binned;  // round 1 ran before the launch: outputs and rounds follow it
};

__global__ void k_list_init(ListCtrl *ctrl, uint32_t slot_groups) {
  uint32_t *w = reinterpret_cast<uint32_t *>(ctrl);
  for (uint32_t i = threadIdx.x; i < sizeof(ListCtrl) / 4; i += blockDim.x) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) bar_force_slot_groups(&ctrl->bar, slot_groups != 0);
}

// Claims cell c for this round's listing (signed tables: a cell can be queued
// twice in a round, since its count can pass +-1 twice); the listing clears it.
__device__ inline bool claim_cell(iblt_cell *cells, uint32_t c) {
  return atomicCAS(&cells[c].reserved0, 0u, 1u) == 0u;
}

// Round 1 of a plain listing whose removals go through the binned update:
// every pure cell that owns its key (the test of the persistent kernel's first
// detect) gives its key to out.  Each workgroup scans a contiguous range of
// cells and stages its keys in LDS; a full stage takes its place in out with
// one device atomic on ctrl->first_keys.  The table is only read.
constexpr uint32_t kD1Cap = 4096;  // keys staged per workgroup before they are written
template <int R>
__global__ void __launch_bounds__(kBlock)
    k_list_detect1(Hash h, const iblt_cell *cells, uint32_t N, uint64_t *out, ListCtrl *ctrl) {
  __shared__ uint64_t sk[kD1Cap];
  __shared__ uint32_t s_n;
  __shared__ unsigned long long s_base;
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (N + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = (uint64_t)blockIdx.x * per;
  const uint32_t c0 = lo < N ? static_cast<uint32_t>(lo) : N;
  const uint32_t c1 = N - c0 < per ? N : c0 + per;
  if (tid == 0) s_n = 0;
  __syncthreads();
  auto flush = [&]() {  // every thread; s_n is final
    const uint32_t n = s_n;
    if (tid == 0) s_base = n ? atomicAdd(&ctrl->first_keys, (unsigned long long)n) : 0ull;
    __syncthreads();
    const unsigned long long base = s_base;
    for (uint32_t i = tid; i < n; i += kBlock) out[base + i] = sk[i];
    __syncthreads();
    if (tid == 0) s_n = 0;
    __syncthreads();
  };
  uint32_t bad = 0;
  long long unused = 0;
  constexpr uint32_t kStep = kDetU * kBlock;  // cells per step, kDetU per lane
  for (uint64_t cb = c0; cb < c1; cb += kStep) {
    const uint64_t ce = c1 - cb < kStep ? c1 : cb + kStep;
    detect_cells<R, false>(
        h, cells, cb, ce, tid, kBlock, [](uint64_t i) { return static_cast<uint32_t>(i); },
        [&](uint64_t ks, uint32_t) { sk[wave_append(true, &s_n)] = ks; }, &bad, &unused);
    __syncthreads();
    if (s_n + kStep > kD1Cap) flush();  // the next step could overflow the stage
  }
  flush();
  if (bad) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
}

template <int R, bool SIGNED = false>
__global__ void __launch_bounds__(kLT) k_list_persistent(ListArgs a) {
  __shared__ uint32_t s_own, s_cand, s_bad;
  __shared__ unsigned long long s_sum;

  ListCtrl *ctrl = a.ctrl;
  uint32_t slot, T;
  if (!team_join(&ctrl->team, a.quiet, a.team_limit, &slot, &T)) return;
  const uint32_t tid = threadIdx.x;
  const uint64_t gtid = (uint64_t)slot * kLT + tid;
  const uint64_t gsize = (uint64_t)T * kLT;
  const uint32_t cb = a.cb;
  const uint32_t N = a.ncells;
  uint64_t *myKeys = a.skeys + (uint64_t)slot * cb;
  uint32_t *myOwn = a.scells + (uint64_t)slot * cb;
  uint32_t *myCand = a.cand + (uint64_t)slot * cb;
  // after a binned first round (launched before this kernel), this kernel's
  // rounds are the run's rounds 2, 3, ... and their keys follow round 1's
  uint64_t *out = a.out;
  uint64_t out_cap = a.out_cap;
  if (a.first_binned) {
    const uint64_t f = ctrl->first_keys;
    out += f;
    out_cap = out_cap > f ? out_cap - f : 0;
  }

  auto stage = [&](uint64_t x, uint32_t c, uint32_t parity) {
    const uint32_t pos = wave_append(true, &s_own);
    if (pos < cb) {
      myKeys[pos] = x;
      myOwn[pos] = c;
    } else {
      const uint32_t j = atomicAdd(&ctrl->ovf_own[parity], 1u);
      a.okeys[j] = x;
      a.ocells[j] = c;
    }
  };

  // ---- round-1 detect over my range of cells ------------------------------
  if (tid == 0) {
    s_own = 0;
    s_bad = 0;
    s_sum = 0;
  }
  if (slot == 0)
    for (uint32_t i = tid; i < a.max_rounds; i += kLT) a.stats[i] = 0;
  __syncthreads();
  {
    const uint32_t cr = (N + T - 1) / T;
    const uint32_t c0 = slot * cr < N ? slot * cr : N;
    const uint32_t c1 = c0 + cr < N ? c0 + cr : N;
    long long local = 0;
    uint32_t bad = 0;
    detect_cells<R, SIGNED>(
        a.h, a.cells, c0, c1, tid, kLT, [](uint64_t i) { return static_cast<uint32_t>(i); },
        [&](uint64_t ks, uint32_t c) {
          if (!SIGNED || claim_cell(a.cells, c)) stage(ks, c, 1u);
        },
        &bad, &local);
    if (bad) s_bad = 1;
    atomicAdd(&s_sum, (unsigned long long)local);
  }
  __syncthreads();
  if (tid == 0) {
    if (s_sum) atomicAdd(&ctrl->count_sum, s_sum);
    if (s_bad) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
  }
  uint32_t staged = s_own < cb ? s_own : cb;
  uint32_t epoch = 0;
  uint64_t total, prefix;
  if (!sum_barrier(&ctrl->bar, T, slot, staged, &epoch, a.limit, &total, ctrl->stamp, &prefix))
    return;
  uint32_t ovf = __hip_atomic_load(&ctrl->ovf_own[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  uint64_t listed = 0;
  uint32_t t = 1;
  for (;; ++t) {
    const uint64_t K = total + ovf;
    if (K == 0) break;
    if (t > a.max_rounds || listed + K > out_cap) {
      if (slot == 0 && tid == 0)
        atomicOr(&ctrl->flags, t > a.max_rounds ? PEEL_FLAG_EROUNDS : PEEL_FLAG_ENOSPC);
      if (SIGNED) {  // give back the claims of the round that does not run
        for (uint32_t i = tid; i < staged; i += kLT) a.cells[myOwn[i]].reserved0 = 0;
        for (uint64_t j = gtid; j < ovf; j += gsize) a.cells[a.ocells[j]].reserved0 = 0;
      }
      break;
    }
    // outputs of round t, grouped after the previous rounds
    for (uint32_t i = tid; i < staged; i += kLT) {
      out[listed + prefix + i] = myKeys[i];
      if (SIGNED) a.signs[listed + prefix + i] = static_cast<int8_t>(a.cells[myOwn[i]].count);
    }
    for (uint64_t j = gtid; j < ovf; j += gsize) {
      out[listed + total + j] = a.okeys[j];
      if (SIGNED) a.signs[listed + total + j] = static_cast<int8_t>(a.cells[a.ocells[j]].count);
    }
    if (slot == 0 && tid == 0) {
      a.stats[t - 1] = K;
      ctrl->ovf_cand[(t + 1) & 1] = 0;  // consumed by the detect phase of round t
    }
    // apply: delete this round's keys; cells going 2 -> 1 are next round's candidates
    if (tid == 0) s_cand = 0;
    __syncthreads();
    const uint32_t par = t & 1;
    // A plain listing pushes a cell at most once a round (its count passes
    // 2 -> 1 once), so the N overflow places always suffice.  A signed listing
    // can push a cell again each time its count lands on +-1: past N places
    // the cell is dropped and the call reports PEEL_FLAG_ENOSPC.
    auto push = [&](uint32_t c) {
      const uint32_t pos = wave_append(true, &s_cand);
      if (pos < cb) {
        myCand[pos] = c;
      } else {
        const uint32_t j = atomicAdd(&ctrl->ovf_cand[par], 1u);
        if (j < N)
          a.ocand[(uint64_t)par * N + j] = c;
        else
          atomicOr(&ctrl->flags, PEEL_FLAG_ENOSPC);
      }
    };
    for (uint32_t i = tid; i < staged; i += kLT)
      delete_key<R, SIGNED>(a.h, a.cells, myKeys[i], myOwn[i], push,
                            SIGNED ? a.cells[myOwn[i]].count : 1);
    for (uint64_t j = gtid; j < ovf; j += gsize)
      delete_key<R, SIGNED>(a.h, a.cells, a.okeys[j], a.ocells[j], push,
                            SIGNED ? a.cells[a.ocells[j]].count : 1);
    __syncthreads();
    const uint32_t ncand = s_cand < cb ? s_cand : cb;
    uint64_t dummy;
    if (!sum_barrier(&ctrl->bar, T, slot, 0, &epoch, a.limit, &dummy, ctrl->stamp)) return;
    listed += K;
    // detect for round t+1 over my candidates and a share of the overflow
    const uint32_t npar = (t + 1) & 1;
    if (tid == 0) {
      s_own = 0;
      s_bad = 0;
      if (slot == 0) ctrl->ovf_own[par] = 0;  // consumed by round t
    }
    __syncthreads();
    {
      uint32_t bad = 0;
      long long unused = 0;
      auto take = [&](uint64_t ks, uint32_t c) {
        if (!SIGNED || claim_cell(a.cells, c)) stage(ks, c, npar);
      };
      detect_cells<R, SIGNED>(
          a.h, a.cells, 0, ncand, tid, kLT, [&](uint64_t i) { return myCand[i]; }, take, &bad,
          &unused);
      uint32_t ovc =
          __hip_atomic_load(&ctrl->ovf_cand[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ovc = ovc < N ? ovc : N;  // the places written (see push)
      const uint32_t *oc = a.ocand + (uint64_t)par * N;
      detect_cells<R, SIGNED>(
          a.h, a.cells, (uint64_t)slot * kLT, ovc, tid, (uint32_t)gsize,
          [&](uint64_t i) { return oc[i]; }, take, &bad, &unused);
      if (bad) s_bad = 1;
    }
    __syncthreads();
    if (tid == 0 && s_bad) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
    staged = s_own < cb ? s_own : cb;
    if (!sum_barrier(&ctrl->bar, T, slot, staged, &epoch, a.limit, &total, ctrl->stamp, &prefix))
      return;
    ovf = __hip_atomic_load(&ctrl->ovf_own[npar], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (slot == 0 && tid == 0) {
    ctrl->rounds = t - 1 < a.max_rounds ? t - 1 : a.max_rounds;
    ctrl->listed = listed;
    ctrl->team_size = T;
  }
}

// ===========================================================================
// Owner engine for the plain listing (the default).  Device-scope atomics run
// at a fixed ~27 G/s on this GPU, and the persistent kernel above spends three
// per cell a listed key leaves.  Here each of T workgroups owns a range of
// cr = ceil(N / T) cells and is their only writer:
//   detect  each owner examines its candidates (round 1: all its cells; then
//           the cells whose count fell to 1), with the read-only ownership
//           test of the kernel above, and keeps the keys its cells list; for
//           each it makes one message (cell, key) per other cell of the key,
//           to that cell's owner.  The messages are written into the sender's
//           own region, sorted by destination (kMC at a time ranked and sorted
//           in LDS, so neighbouring lanes store neighbouring words), and the
//           per-destination counts and starts are published.
//   apply   after the barrier, each owner reads the runs addressed to it from
//           every sender, combines the updates of each cell in an LDS hash
//           table (kAC at a time: count, key XOR, checksum XOR), and applies
//           each with one plain 32-byte read-modify-write; a cell whose count
//           becomes 1 is its own next candidate.  It clears the cells its keys
//           were listed from and writes its keys to out.
// Two barriers a round, as above; no device atomic per key or per cell.  Every
// list has a fixed bound: an owner lists at most one key per cell it owns and
// pushes each of its cells at most once a round, and sends at most r - 1
// messages per key it lists.
constexpr uint32_t kLMaxT = 1024;   // owners (LDS per-destination counters)
constexpr uint32_t kMC = 2048;      // messages sorted in LDS at a time
constexpr uint32_t kOAC = 2048;     // messages combined in LDS at a time
constexpr uint32_t kOHBits = 12;
constexpr uint32_t kOHS = 1u << kOHBits;  // hash slots for one apply chunk
constexpr uint32_t kSeenMax = 98304;      // owned cells the LDS bitmaps of the listing cover
static_assert(2 * kOAC <= kOHS, "the apply's hash table stays at most half full");

struct OwnArgs {
  Hash h;
  iblt_cell *cells;
  uint64_t *out;
  uint64_t out_cap;
  uint64_t *stats;
  uint64_t *keys;   // N: the keys each owner lists this round (at its first cell)
  uint32_t *ownc;   // N: the cells they were listed from
  uint32_t *cand;   // N: each owner's candidates for the next round
  uint64_t *candk;  // N: their keys (a candidate is pushed pure: count 1, checksum good)
  uint4 *msg;       // (r-1) N: each owner's outgoing messages {cell, 0, key lo, key hi}
  uint32_t *mcnt;   // grid x grid: messages from owner s to owner d at [s * grid + d]
  uint32_t *moff;   // grid x grid: where in s's region they start
  ListCtrl *ctrl;
  uint64_t limit;
  uint64_t quiet;
  uint64_t team_limit;
  uint32_t ncells;
  uint32_t max_rounds;
  uint32_t grid;
};

struct OwnSlot {  // LDS: one cell's combined updates in an apply chunk
  unsigned long long ks;
  unsigned long long hs;
  uint32_t cell;
  int32_t n;
};

template <int R>
__global__ void __launch_bounds__(kLT) k_list_owner(OwnArgs a) {
  // keys whose messages are sorted at a time: one per thread, at most kMC messages
  constexpr uint32_t kKC = kMC / (R - 1) < (uint32_t)kLT ? kMC / (R - 1) : (uint32_t)kLT;
  // the send's sort buffer and the apply's hash table share one LDS area
  constexpr size_t kPool = kOHS * sizeof(OwnSlot) > kMC * sizeof(uint4) + kMC * 2
                               ? kOHS * sizeof(OwnSlot) : kMC * sizeof(uint4) + kMC * 2;
  __shared__ __align__(16) unsigned char pool[kPool];
  __shared__ uint32_t cnt[kLMaxT];
  __shared__ uint32_t cur[kLMaxT];
  __shared__ uint32_t sst[kLMaxT];
  __shared__ uint32_t inpre[kLMaxT + 1];
  __shared__ uint32_t scan_lds[kLT / kWave + 1];
  __shared__ uint32_t s_own, s_cand, s_bad;
  __shared__ unsigned long long s_sum;
  // apply: my cells updated in this round's apply (seen) and those updated in
  // two of its chunks (multi), whose pushed value may be stale
  __shared__ uint32_t seen[kSeenMax / 32];
  __shared__ uint32_t multi[kSeenMax / 32];
  // my cells whose key has been listed: cleared once, in cell order, at the end
  // (no later round reads such a cell: it held that key alone)
  __shared__ uint32_t listed_at[kSeenMax / 32];

  ListCtrl *ctrl = a.ctrl;
  uint32_t slot, T;
  if (!team_join(&ctrl->team, a.quiet, a.team_limit, &slot, &T)) return;
  const uint32_t tid = threadIdx.x;
  if (T > kLMaxT) {  // cannot happen: the grid is at most the CU count
    if (slot == 0 && tid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_TIMEOUT);
    return;
  }
  // My cells: the slot-th piece of every subtable (pieces of pw[j] cells).
  // An owner of only low-subtable cells would have no ownership tests to make
  // and most of the round-1 keys to list, and one of only high-subtable cells
  // the opposite; a piece of each balances every phase across the team.
  uint32_t pw[R], plo[R], pn[R];
  uint32_t cw = 0, nmine = 0;  // cells per workgroup at most, and mine
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const uint32_t sz = static_cast<uint32_t>(a.h.size[j]);
    pw[j] = (sz + T - 1) / T;
    const uint32_t lo = slot * pw[j] < sz ? slot * pw[j] : sz;
    const uint32_t hi = lo + pw[j] < sz ? lo + pw[j] : sz;
    plo[j] = static_cast<uint32_t>(a.h.base[j]) + lo;
    pn[j] = hi - lo;
    cw += pw[j];
    nmine += pn[j];
  }
  // the owner of cell c of subtable j
  auto owner = [&](int j, uint32_t c) {
    return (c - static_cast<uint32_t>(a.h.base[j])) / pw[j];
  };
  // my i-th cell, i < nmine
  auto my_cell = [&](uint64_t i) {
    uint32_t k = static_cast<uint32_t>(i), c = 0;
    bool found = false;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (!found && k < pn[j]) {
        c = plo[j] + k;
        found = true;
      }
      if (!found) k -= pn[j];
    }
    return c;
  };
  // the place of my cell c among my cells
  auto my_index = [&](uint32_t c) {
    uint32_t k = 0, r = 0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (c >= plo[j] && c < plo[j] + pn[j]) r = k + (c - plo[j]);
      k += pn[j];
    }
    return r;
  };
  const bool track = nmine <= kSeenMax;  // else every candidate is read back, and
                                         // a listed key's cell is cleared at once
  uint64_t *myKeys = a.keys + (uint64_t)slot * cw;
  uint32_t *myOwn = a.ownc + (uint64_t)slot * cw;
  uint32_t *myCand = a.cand + (uint64_t)slot * cw;
  uint64_t *myCandK = a.candk + (uint64_t)slot * cw;
  uint4 *myMsg = a.msg + (uint64_t)(R - 1) * slot * cw;
  uint4 *sbuf = reinterpret_cast<uint4 *>(pool);
  uint16_t *sdst = reinterpret_cast<uint16_t *>(pool + kMC * sizeof(uint4));
  OwnSlot *hslot = reinterpret_cast<OwnSlot *>(pool);
  const Hash &h = a.h;

  if (tid == 0) {
    s_own = 0;
    s_bad = 0;
    s_sum = 0;
  }
  if (slot == 0)
    for (uint32_t i = tid; i < a.max_rounds; i += kLT) a.stats[i] = 0;
  if (track)
    for (uint32_t w = tid; w < (nmine + 31) / 32; w += kLT) listed_at[w] = 0;
  __syncthreads();
  auto take = [&](uint64_t ks, uint32_t c) {
    const uint32_t pos = wave_append(true, &s_own);
    myKeys[pos] = ks;
    myOwn[pos] = c;
  };
  // ---- round-1 detect over my cells ------------------------------------------
  {
    long long local = 0;
    uint32_t bad = 0;
    detect_cells<R, false>(h, a.cells, 0, nmine, tid, kLT, my_cell, take, &bad, &local);
    if (bad) s_bad = 1;
    atomicAdd(&s_sum, (unsigned long long)local);
  }
  __syncthreads();
  if (tid == 0) {
    if (s_sum) atomicAdd(&ctrl->count_sum, s_sum);
    if (s_bad) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
  }

  // the keys of round t leave their other cells: messages to those cells' owners
  auto send = [&](uint32_t nk) {
    for (uint32_t d = tid; d < T; d += kLT) cnt[d] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < nk; i += kLT) {
      const uint64_t x = myKeys[i];
      const uint32_t jo = subtable_of(h, myOwn[i]);
#pragma unroll
      for (int j = 0; j < R; ++j)
        if ((uint32_t)j != jo) atomicAdd(&cnt[owner(j, cell_of(h, j, x))], 1u);
    }
    __syncthreads();
    uint32_t base = 0;
    for (uint32_t d0 = 0; d0 < T; d0 += kLT) {
      const uint32_t d = d0 + tid;
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan<kLT>(d < T ? cnt[d] : 0u, &tot, scan_lds);
      if (d < T) {
        cur[d] = base + ex;
        a.mcnt[(uint64_t)slot * a.grid + d] = cnt[d];
        a.moff[(uint64_t)slot * a.grid + d] = base + ex;
      }
      base += tot;
    }
    __syncthreads();
    for (uint32_t k0 = 0; k0 < nk; k0 += kKC) {
      for (uint32_t d = tid; d < T; d += kLT) cnt[d] = 0;
      __syncthreads();
      const uint32_t i = k0 + tid;
      uint64_t x = 0;
      uint32_t cl[R], rk[R];
      bool live = tid < kKC && i < nk;
      uint32_t jo = R;
      if (live) {
        x = myKeys[i];
        jo = subtable_of(h, myOwn[i]);
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
        cl[j] = cell_of(h, j, x);
        if (live && (uint32_t)j != jo) rk[j] = atomicAdd(&cnt[owner(j, cl[j])], 1u);
      }
      __syncthreads();
      uint32_t tot = 0, run = 0;
      for (uint32_t d0 = 0; d0 < T; d0 += kLT) {
        const uint32_t d = d0 + tid;
        uint32_t t0;
        const uint32_t ex = block_exclusive_scan<kLT>(d < T ? cnt[d] : 0u, &t0, scan_lds);
        if (d < T) sst[d] = run + ex;
        run += t0;
      }
      tot = run;
      __syncthreads();
      if (live) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
          if ((uint32_t)j == jo) continue;
          const uint32_t d = owner(j, cl[j]);
          const uint32_t p = sst[d] + rk[j];
          sbuf[p] = make_uint4(cl[j], 0u, static_cast<uint32_t>(x), static_cast<uint32_t>(x >> 32));
          sdst[p] = static_cast<uint16_t>(d);
        }
      }
      __syncthreads();
      for (uint32_t q = tid; q < tot; q += kLT) {
        const uint32_t d = sdst[q];
        myMsg[cur[d] + (q - sst[d])] = sbuf[q];
      }
      __syncthreads();
      for (uint32_t d = tid; d < T; d += kLT) cur[d] += cnt[d];
    }
  };

  uint32_t nk = s_own;
  send(nk);
  uint32_t epoch = 0;
  uint64_t total, prefix;
  if (!sum_barrier(&ctrl->bar, T, slot, nk, &epoch, a.limit, &total, ctrl->stamp, &prefix)) return;

  uint64_t listed = 0;
  uint32_t t = 1;
  for (;; ++t) {
    const uint64_t K = total;
    if (K == 0) break;
    if (t > a.max_rounds || listed + K > a.out_cap) {
      if (slot == 0 && tid == 0)
        atomicOr(&ctrl->flags, t > a.max_rounds ? PEEL_FLAG_EROUNDS : PEEL_FLAG_ENOSPC);
      break;
    }
    if (slot == 0 && tid == 0) a.stats[t - 1] = K;
    // ---- apply ---------------------------------------------------------------
    for (uint32_t i = tid; i < nk; i += kLT) {
      a.out[listed + prefix + i] = myKeys[i];
      if (track) {
        const uint32_t lc = my_index(myOwn[i]);
        atomicOr(&listed_at[lc >> 5], 1u << (lc & 31));
      } else {
        clear_cell(a.cells + myOwn[i]);
      }
    }
    // the runs addressed to me, one per sender, laid end to end
    uint32_t nin = 0;
    for (uint32_t s0 = 0; s0 < T; s0 += kLT) {
      const uint32_t sd = s0 + tid;
      uint32_t tot;
      const uint32_t x = sd < T ? a.mcnt[(uint64_t)sd * a.grid + slot] : 0u;
      const uint32_t ex = block_exclusive_scan<kLT>(x, &tot, scan_lds);
      if (sd < T) {
        inpre[sd] = nin + ex;
        sst[sd] = a.moff[(uint64_t)sd * a.grid + slot];
      }
      nin += tot;
    }
    if (tid == 0) {
      inpre[T] = nin;
      s_cand = 0;
    }
    if (track)
      for (uint32_t w = tid; w < (nmine + 31) / 32; w += kLT) seen[w] = multi[w] = 0;
    __syncthreads();
    // kOAC messages a chunk, kOU per thread.  A chunk's messages were loaded
    // during the previous chunk, and each thread loads the cells of its
    // messages before the hashing, so that one global latency per chunk is
    // exposed; the cell a leader loaded is current, since only the leader of a
    // cell writes it in a chunk and the chunk before has finished.
    constexpr int kOU = (int)(kOAC / kLT);
    auto fetch = [&](uint32_t m0, uint4 *mm) {
#pragma unroll
      for (int u = 0; u < kOU; ++u) {
        const uint32_t i = m0 + (uint32_t)u * kLT + tid;
        mm[u] = make_uint4(0xffffffffu, 0u, 0u, 0u);
        if (i >= nin) continue;
        // the sender whose run holds incoming message i
        uint32_t lo = 0, hi = T;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (inpre[mid] <= i) lo = mid; else hi = mid;
        }
        mm[u] = a.msg[(uint64_t)(R - 1) * lo * cw + sst[lo] + (i - inpre[lo])];
      }
    };
    uint4 mnext[kOU];
    fetch(0, mnext);
    for (uint32_t m0 = 0; m0 < nin; m0 += kOAC) {
      uint4 mm[kOU], x0[kOU];
      uint2 x1[kOU];  // the hash sum; the cell's last 8 bytes are not touched
#pragma unroll
      for (int u = 0; u < kOU; ++u) {
        mm[u] = mnext[u];
        if (mm[u].x != 0xffffffffu) {
          const uint4 *p = reinterpret_cast<const uint4 *>(a.cells + mm[u].x);
          x0[u] = p[0];
          x1[u] = *reinterpret_cast<const uint2 *>(p + 1);
        }
      }
      for (uint32_t q = tid; q < kOHS; q += kLT) {
        hslot[q].cell = 0xffffffffu;
        hslot[q].n = 0;
        hslot[q].ks = 0ull;
        hslot[q].hs = 0ull;
      }
      __syncthreads();
      uint32_t lead[kOU];
#pragma unroll
      for (int u = 0; u < kOU; ++u) {
        lead[u] = 0xffffffffu;
        const uint32_t c = mm[u].x;
        if (c == 0xffffffffu) continue;
        const uint64_t x = (uint64_t)mm[u].z | ((uint64_t)mm[u].w << 32);
        uint32_t q = (c * 0x9e3779b1u) >> (32 - kOHBits);
        for (;;) {
          const uint32_t old = atomicCAS(&hslot[q].cell, 0xffffffffu, c);
          if (old == 0xffffffffu) {
            lead[u] = q;
            break;
          }
          if (old == c) break;
          q = (q + 1) & (kOHS - 1);
        }
        atomicAdd(&hslot[q].n, 1);
        atomicXor(&hslot[q].ks, (unsigned long long)x);
        atomicXor(&hslot[q].hs, (unsigned long long)check_of(h, x));
      }
      fetch(m0 + kOAC, mnext);  // in flight while the chunk is applied
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kOU; ++u) {
        if (lead[u] == 0xffffffffu) continue;
        const OwnSlot &sl = hslot[lead[u]];
        const int32_t now = static_cast<int32_t>(x0[u].x) - sl.n;
        x0[u].x = static_cast<uint32_t>(now);
        x0[u].z ^= static_cast<uint32_t>(sl.ks);
        x0[u].w ^= static_cast<uint32_t>(sl.ks >> 32);
        x1[u].x ^= static_cast<uint32_t>(sl.hs);
        x1[u].y ^= static_cast<uint32_t>(sl.hs >> 32);
        uint4 *p = reinterpret_cast<uint4 *>(a.cells + sl.cell);
        p[0] = x0[u];
        *reinterpret_cast<uint2 *>(p + 1) = x1[u];
        // A cell that went to count 1 is pushed with its key.  The detect
        // trusts that value unless the cell is marked multi: updated by two
        // chunks of this apply (the value may be stale), or pushed with a
        // checksum that does not match (the detect reads it back and judges).
        const uint32_t lc = track ? my_index(sl.cell) : 0u, bit = 1u << (lc & 31);
        if (track && (atomicOr(&seen[lc >> 5], bit) & bit)) atomicOr(&multi[lc >> 5], bit);
        if (now == 1) {
          const uint64_t ks = (uint64_t)x0[u].z | ((uint64_t)x0[u].w << 32);
          const uint64_t hs = (uint64_t)x1[u].x | ((uint64_t)x1[u].y << 32);
          if (track && hs != check_of(h, ks)) atomicOr(&multi[lc >> 5], bit);
          const uint32_t pos = wave_append(true, &s_cand);
          myCand[pos] = sl.cell;
          myCandK[pos] = ks;
        }
      }
      __syncthreads();
    }
    listed += K;
    uint64_t dummy;
    if (!sum_barrier(&ctrl->bar, T, slot, 0, &epoch, a.limit, &dummy, ctrl->stamp)) return;
    // ---- detect for round t+1 over my candidates ------------------------------
    const uint32_t ncand = s_cand;
    if (tid == 0) {
      s_own = 0;
      s_bad = 0;
    }
    __syncthreads();
    {
      // a candidate not marked multi is pure with the pushed key: only the
      // ownership test reads the table; a marked one is read back
      uint32_t bad = 0;
      for (uint32_t ib = tid; ib < ncand; ib += kDetU * kLT) {
        uint32_t c[kDetU];
        int32_t cn[kDetU];
        uint64_t ks[kDetU], hs[kDetU];
#pragma unroll
        for (int u = 0; u < kDetU; ++u) {
          const uint32_t i = ib + (uint32_t)u * kLT;
          c[u] = 0;
          cn[u] = 0;
          ks[u] = hs[u] = 0;
          if (i < ncand) {
            c[u] = myCand[i];
            ks[u] = myCandK[i];
            const uint32_t lc = track ? my_index(c[u]) : 0u;
            if (!track || ((multi[lc >> 5] >> (lc & 31)) & 1u)) {
              load_cell(a.cells + c[u], &cn[u], &ks[u], &hs[u]);
            } else {
              cn[u] = 1;
              hs[u] = check_of(h, ks[u]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kDetU; ++u)
          if (ib + (uint32_t)u * kLT < ncand && owns<R, false>(h, a.cells, c[u], cn[u], ks[u], hs[u], &bad))
            take(ks[u], c[u]);
      }
      if (bad) s_bad = 1;
    }
    __syncthreads();
    if (tid == 0 && s_bad) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
    nk = s_own;
    send(nk);
    if (!sum_barrier(&ctrl->bar, T, slot, nk, &epoch, a.limit, &total, ctrl->stamp, &prefix))
      return;
  }
  // the cells my listed keys came from, cleared in cell order
  if (track) {
    __syncthreads();
    for (uint32_t lc = tid; lc < nmine; lc += kLT)
      if ((listed_at[lc >> 5] >> (lc & 31)) & 1u) clear_cell(a.cells + my_cell(lc));
  }
  if (slot == 0 && tid == 0) {
    ctrl->rounds = t - 1 < a.max_rounds ? t - 1 : a.max_rounds;
    ctrl->listed = listed;
    ctrl->team_size = T;
  }
}

// ===========================================================================
// Listing with subtables (Section 5, "Implementation Details"; Appendix B):
// the paper's GPU process.  Each round is r subrounds; subround s = (i-1) r + j
// + 1 lists the key of every cell of subtable j that is pure at its start and
// deletes those keys from their r cells.  A key has one cell per subtable, so
// it is listed once without any ownership test.
//
// Candidates: in round 1 every cell of subtable j is examined (a dense pass);
// afterwards only cells that went 2 -> 1 are.  They wait in a queue shared by
// the team (two buffers of ncells entries; each cell enters it at most once,
// since counts only fall) until their subtable's subround; a push into a
// subtable whose round-1 pass is still to come is dropped, that pass covers it.
// The run ends once round 1 is over and the queue is empty.

constexpr int kLQ = 4096;  // workgroup-local push buffer (flushed to the queue)

template <int R>
__global__ void __launch_bounds__(kLT) k_list_sub(ListArgs a) {
  __shared__ uint32_t s_own, s_bad, s_lq, s_qbase;
  __shared__ unsigned long long s_sum;
  __shared__ uint32_t lq[kLQ];

  ListCtrl *ctrl = a.ctrl;
  uint32_t slot, T;
  if (!team_join(&ctrl->team, a.quiet, a.team_limit, &slot, &T)) return;
  const uint32_t tid = threadIdx.x;
  const uint64_t gtid = (uint64_t)slot * kLT + tid;
  const uint64_t gsize = (uint64_t)T * kLT;
  const uint32_t cb = a.cb;
  const uint32_t N = a.ncells;
  uint64_t *myKeys = a.skeys + (uint64_t)slot * cb;
  uint32_t *myOwn = a.scells + (uint64_t)slot * cb;
  uint32_t *queue[2] = {a.ocand, a.ocand + N};

  auto stage = [&](uint64_t x, uint32_t c, uint32_t parity) {
    const uint32_t pos = wave_append(true, &s_own);
    if (pos < cb) {
      myKeys[pos] = x;
      myOwn[pos] = c;
    } else {
      const uint32_t q = atomicAdd(&ctrl->ovf_own[parity], 1u);
      a.okeys[q] = x;
      a.ocells[q] = c;
    }
  };
  auto flush = [&](uint32_t *nxt, uint32_t *ncount) {
    __syncthreads();
    const uint32_t nq = s_lq < (uint32_t)kLQ ? s_lq : (uint32_t)kLQ;
    if (tid == 0) s_qbase = nq ? atomicAdd(ncount, nq) : 0u;
    __syncthreads();
    for (uint32_t i = tid; i < nq; i += kLT) nxt[s_qbase + i] = lq[i];
  };

  if (slot == 0)
    for (uint32_t i = tid; i < a.max_rounds; i += kLT) a.stats[i] = 0;
  uint32_t epoch = 0;
  uint64_t listed = 0;
  uint32_t last = 0;
  uint32_t s = 1;
  bool early = false;  // stopped before round 1 ended
  for (;; ++s) {
    const uint32_t j = (s - 1) % R;
    const bool first = s <= R;
    const uint32_t par = s & 1u;
    const uint32_t *cur = queue[s & 1u];
    uint32_t *nxt = queue[(s + 1) & 1u];
    uint32_t *ncount = &ctrl->qn[(s + 1) % 3];
    const uint32_t size = __hip_atomic_load(&ctrl->qn[s % 3], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) {
      s_own = 0;
      s_bad = 0;
      s_sum = 0;
      s_lq = 0;
      if (slot == 0) ctrl->qn[(s + 2) % 3] = 0;  // the next subround's push counter
    }
    __syncthreads();
    auto lpush = [&](uint32_t c) {
      const uint32_t p = wave_append(true, &s_lq);
      if (p < (uint32_t)kLQ)
        lq[p] = c;
      else
        nxt[atomicAdd(ncount, 1u)] = c;
    };
    // ---- detect ------------------------------------------------------------
    {
      uint32_t bad = 0;
      if (first) {
        // every cell of subtable j (its counts also feed the table's key count)
        const uint32_t lo = (uint32_t)a.h.base[j], sz = (uint32_t)a.h.size[j];
        const uint32_t cr = (sz + T - 1) / T;
        const uint32_t c0 = lo + (slot * cr < sz ? slot * cr : sz);
        const uint32_t c1 = lo + ((slot + 1) * cr < sz ? (slot + 1) * cr : sz);
        long long local = 0;
        for (uint32_t c = c0 + tid; c < c1; c += kLT) {
          int32_t cnt;
          uint64_t ks, hs;
          load_cell(a.cells + c, &cnt, &ks, &hs);
          local += cnt;
          if (cnt == 1) {
            if (hs == check_of(a.h, ks))
              stage(ks, c, par);
            else
              bad = 1;
          }
        }
        atomicAdd(&s_sum, (unsigned long long)local);
      }
      for (uint64_t i = gtid; i < size; i += gsize) {
        const uint32_t c = cur[i];
        if (subtable_of(a.h, c) != j) {  // waits for its subtable's subround
          lpush(c);
          continue;
        }
        int32_t cnt;
        uint64_t ks, hs;
        load_cell(a.cells + c, &cnt, &ks, &hs);
        if (cnt == 1) {
          if (hs == check_of(a.h, ks))
            stage(ks, c, par);
          else
            bad = 1;
        }
      }
      if (bad) s_bad = 1;
    }
    flush(nxt, ncount);
    __syncthreads();
    if (tid == 0) {
      // Each key listed so far left one cell of subtable j, so the counts of
      // subtable j now plus those keys are its counts at the start.
      if (first) {
        const unsigned long long add = s_sum + (slot == 0 ? listed : 0ull);
        if (add) atomicAdd(&ctrl->count_sum, add);
      }
      if (s_bad) atomicOr(&ctrl->flags, PEEL_FLAG_ECORRUPT);
    }
    const uint32_t staged = s_own < cb ? s_own : cb;
    uint64_t total, prefix;
    if (!sum_barrier(&ctrl->bar, T, slot, staged, &epoch, a.limit, &total, ctrl->stamp, &prefix))
      return;
    const uint32_t ovf =
        __hip_atomic_load(&ctrl->ovf_own[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t K = total + ovf;
    if (K == 0) {
      // nothing listed: the queue holds only waiting cells
      if (s >= R && __hip_atomic_load(ncount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        break;
      continue;
    }
    if (s > a.max_rounds) {
      if (slot == 0 && tid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_EROUNDS);
      early = s < R;
      break;
    }
    if (listed + K > a.out_cap) {
      if (slot == 0 && tid == 0) atomicOr(&ctrl->flags, PEEL_FLAG_ENOSPC);
      early = s < R;
      break;
    }
    // ---- outputs of subround s, then apply -----------------------------------
    for (uint32_t i = tid; i < staged; i += kLT) a.out[listed + prefix + i] = myKeys[i];
    for (uint64_t q = gtid; q < ovf; q += gsize) a.out[listed + total + q] = a.okeys[q];
    if (slot == 0 && tid == 0) a.stats[s - 1] = K;
    if (tid == 0) s_lq = 0;
    __syncthreads();
    auto push = [&](uint32_t c) {
      // a subtable whose round-1 pass is still to come will see c anyway
      if (first && subtable_of(a.h, c) > j) return;
      lpush(c);
    };
    for (uint32_t i = tid; i < staged; i += kLT) delete_key<R>(a.h, a.cells, myKeys[i], myOwn[i], push);
    for (uint64_t q = gtid; q < ovf; q += gsize) delete_key<R>(a.h, a.cells, a.okeys[q], a.ocells[q], push);
    flush(nxt, ncount);
    uint64_t dummy;
    if (!sum_barrier(&ctrl->bar, T, slot, 0, &epoch, a.limit, &dummy, ctrl->stamp)) return;
    listed += K;
    last = s;
    if (slot == 0 && tid == 0) ctrl->ovf_own[par] = 0;  // consumed
    if (s >= R && __hip_atomic_load(ncount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
      break;
  }
  if (early) {
    // stopped inside round 1: the subtables not yet passed over are summed now,
    // each of their counts plus one per key listed so far
    for (uint32_t jj = (s - 1) % R + 1; jj < R; ++jj) {
      const uint32_t lo = (uint32_t)a.h.base[jj], sz = (uint32_t)a.h.size[jj];
      long long local = 0;
      for (uint64_t c = gtid; c < sz; c += gsize) {
        int32_t cnt;
        uint64_t ks, hs;
        load_cell(a.cells + lo + c, &cnt, &ks, &hs);
        local += cnt;
      }
      if (tid == 0) s_sum = 0;
      __syncthreads();
      atomicAdd(&s_sum, (unsigned long long)local);
      __syncthreads();
      if (tid == 0) {
        const unsigned long long add = s_sum + (slot == 0 ? listed : 0ull);
        if (add) atomicAdd(&ctrl->count_sum, add);
      }
    }
  }
  if (slot == 0 && tid == 0) {
    ctrl->rounds = last;
    ctrl->listed = listed;
    ctrl->team_size = T;
  }
}

// summary = [listed, rounds, keys left, flags, workgroups in the persistent team, 0, 0, 0].
// Signed listing: the cells left non-zero (summary[2]).
__global__ void __launch_bounds__(kBlock) k_count_nonempty(const iblt_cell *cells, uint64_t n,
                                                         ListCtrl *ctrl) {
  __shared__ uint32_t lds[kBlock / kWave + 1];
  uint32_t c = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock) {
    int32_t cnt;
    uint64_t ks, hs;
    load_cell(cells + i, &cnt, &ks, &hs);
    c += (cnt != 0 || ks != 0 || hs != 0) ? 1u : 0u;
  }
  const uint32_t tot = block_sum(c, lds);
  if (threadIdx.x == 0 && tot) atomicAdd(&ctrl->nonempty, (unsigned long long)tot);
}

// first_binned: round 1 ran before the persistent kernel, which counted the
// keys it left (count_sum) and its own rounds and keys; stats[0] gets round 1.
__global__ void k_list_finish(const ListCtrl *ctrl, uint32_t r, uint64_t *summary,
                              uint32_t signed_list, uint64_t *stats, uint32_t first_binned) {
  if (threadIdx.x != 0) return;
  const long long total = (long long)ctrl->count_sum;
  const long long keys = total / (long long)r;
  uint32_t flags = ctrl->flags;
  if (ctrl->bar.abort) flags |= PEEL_FLAG_TIMEOUT;
  uint64_t listed = ctrl->listed;
  uint32_t rounds = ctrl->rounds;
  if (first_binned) {
    const uint64_t f = ctrl->first_keys;
    stats[0] = f;
    if (f) {
      listed += f;
      rounds += 1;
    }
  }
  summary[0] = listed;
  summary[1] = rounds;
  summary[2] = signed_list ? (uint64_t)ctrl->nonempty : (uint64_t)(keys - (long long)ctrl->listed);
  summary[3] = flags;
  summary[4] = ctrl->team_size;
  summary[5] = summary[6] = summary[7] = 0;
}

// ===========================================================================
// Batched listing: many independent tables in one launch, one workgroup per
// table at a time (tables taken in the given order from a shared ticket), the
// round barrier being the workgroup barrier.

// Deletes keys[0, K) -- key i listed from its cell own[i] -- from a table that
// this workgroup alone writes, with no device atomic: the other r - 1 cells of
// a key take one plain 32-byte read-modify-write each.  kXU keys per thread at
// a time, one subtable after another (a key has one cell per subtable, and the
// subtables are disjoint).  In each pass, an LDS hash set of cell indices lets
// the first update of a cell apply and defers the others to the next pass, so
// the updates of one cell apply one after another and each sees the count the
// one before left: a cell is pushed when its count goes from 2 to 1, exactly
// as with atomics.  The cell a key was listed from held that key alone, so it
// is cleared with a plain store and no other update reaches it.
constexpr int kXU = 2;  // keys per thread per apply chunk
constexpr uint32_t kNoCell = 0xffffffffu;

template <int NT>
constexpr uint32_t kApplySet = 2u * kXU * NT;  // hash slots: at most half of them are used

// hset: LDS of kApplySet<NT> words.
template <int R, int NT, typename Push>
__device__ void apply_exclusive(const Hash &h, iblt_cell *cells, const uint64_t *keys,
                                const uint32_t *own, uint32_t K, uint32_t *hset, Push push) {
  constexpr uint32_t kSet = kApplySet<NT>;
  constexpr uint32_t kBits = kSet == 1024 ? 10 : kSet == 2048 ? 11 : 12;
  static_assert((1u << kBits) == kSet, "NT is 256, 512 or 1024");
  const uint32_t tid = threadIdx.x;
  for (uint32_t k0 = 0; k0 < K; k0 += kXU * NT) {
    uint64_t x[kXU], hx[kXU];
    uint32_t co[kXU];
    bool live[kXU];
#pragma unroll
    for (int u = 0; u < kXU; ++u) {
      const uint32_t i = k0 + (uint32_t)u * NT + tid;
      live[u] = i < K;
      x[u] = live[u] ? keys[i] : 0ull;
      co[u] = live[u] ? own[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kXU; ++u) {
      hx[u] = check_of(h, x[u]);
      if (live[u]) clear_cell(cells + co[u]);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      uint32_t c[kXU];
      bool pend[kXU];
#pragma unroll
      for (int u = 0; u < kXU; ++u) {
        c[u] = cell_of(h, j, x[u]);
        pend[u] = live[u] && c[u] != co[u];
      }
      for (;;) {
        for (uint32_t q = tid; q < kSet; q += NT) hset[q] = kNoCell;
        __syncthreads();
        bool any = false;
#pragma unroll
        for (int u = 0; u < kXU; ++u) {
          if (!pend[u]) continue;
          uint32_t q = (c[u] * 0x9e3779b1u) >> (32 - kBits);
          bool lead = false;
          for (;;) {
            const uint32_t old = atomicCAS(&hset[q], kNoCell, c[u]);
            if (old == kNoCell) {
              lead = true;
              break;
            }
            if (old == c[u]) break;
            q = (q + 1) & (kSet - 1);
          }
          if (!lead) {
            any = true;  // this cell already has an update in this pass
            continue;
          }
          uint4 *p = reinterpret_cast<uint4 *>(cells + c[u]);
          uint4 a = p[0], b = p[1];
          const int32_t old = static_cast<int32_t>(a.x);
          a.x = static_cast<uint32_t>(old - 1);
          a.z ^= static_cast<uint32_t>(x[u]);
          a.w ^= static_cast<uint32_t>(x[u] >> 32);
          b.x ^= static_cast<uint32_t>(hx[u]);
          b.y ^= static_cast<uint32_t>(hx[u] >> 32);
          p[0] = a;
          p[1] = b;
          if (old == 2) push(c[u]);
          pend[u] = false;
        }
        if (!__syncthreads_or(any)) break;
      }
    }
  }
}

// The in-place schedule's ownership filter: one LDS bit per cell of the lower
// subtables (the cells below base[R-1], the only ones an owner test reads),
// folded modulo the bits there are when the table has more such cells.  A
// clear bit promises that the cell is not pure at the start of the round, so
// the owner test skips its HBM read; a set bit only says it may be.
//   - Round 1 scans the subtables in order and marks the cells that own their
//     key: when subtable j is tested, every lower pure cell that can decide a
//     test (the key's lowest pure cell) is marked.
//   - Round t > 1: a cell pure at the start of the round went 2 -> 1 in round
//     t - 1's apply (every cell pure at the start of t - 1 lost its key in
//     t - 1, and counts only fall), and the apply marks every such push.
// The bits are cleared before each apply.  Skipped reads change no result: the
// test only ever returns false on a cell of count 1 whose checksum matches.
struct OwnFilter {
  uint32_t *w;
  uint32_t nbits;  // min(lower, bits in w)
  uint32_t lower;  // cells of the lower subtables
  __device__ uint32_t slot(uint32_t c) const { return c < nbits ? c : c % nbits; }
  __device__ bool operator()(uint32_t c) const {
    const uint32_t q = slot(c);
    return (w[q >> 5] >> (q & 31)) & 1u;
  }
  __device__ void mark(uint32_t c) const {
    if (c >= lower) return;
    const uint32_t q = slot(c);
    atomicOr(&w[q >> 5], 1u << (q & 31));
  }
  __device__ void clear(uint32_t tid, uint32_t nt) const {
    for (uint32_t q = tid; q < (nbits + 31) / 32; q += nt) w[q] = 0;
  }
};

// Lists one table with one NT-thread workgroup.  cand and own are scratch of
// ncells entries each; filt is LDS of filt_words words.  Writes the table's
// outputs like iblt_list.
template <int R, int NT>
__device__ __forceinline__ void list_table_block(const iblt_desc desc, iblt_cell *cells, uint32_t N, uint64_t *out,
                                 uint64_t out_cap, uint64_t *stats, uint32_t max_rounds,
                                 uint64_t *summary, uint32_t *cand, uint32_t *own,
                                 uint32_t *hset, uint32_t *filt, uint32_t filt_words) {
  const Hash h = make_hash_fixed<R>(desc);
  __shared__ uint32_t s_k, s_c, s_bad, s_flags;
  __shared__ unsigned long long s_sum;
  const uint32_t tid = threadIdx.x;
  const uint32_t lower = static_cast<uint32_t>(h.base[R - 1]);
  const OwnFilter f{filt, lower < 32u * filt_words ? lower : 32u * filt_words, lower};
  for (uint32_t i = tid; i < max_rounds; i += NT) stats[i] = 0;
  f.clear(tid, NT);
  if (tid == 0) {
    s_k = 0;
    s_bad = 0;
    s_flags = 0;
    s_sum = 0;
  }
  __syncthreads();
  uint64_t listed = 0;
  // round-1 detect over every cell, one subtable after another: owned keys go
  // straight to out[listed + pos], and their cells are marked
  {
    long long local = 0;
    uint32_t bad = 0;
    // subtable j is [j q + min(j, m), (j + 1) q + min(j + 1, m)), as make_hash
    // lays them out (q = N / R, m = N % R)
    const uint32_t q = N / R, m = N % R;
    for (uint32_t j = 0; j < (uint32_t)R; ++j) {
      const uint32_t lo = j * q + (j < m ? j : m);
      const uint32_t hi = lo + q + (j < m ? 1u : 0u);
      // kDetU cells per lane in flight (detect_cells)
      detect_cells<R, false>(
          h, cells, lo, hi, tid, NT,
          [](uint64_t i) { return static_cast<uint32_t>(i); },
          [&](uint64_t ks, uint32_t c) {
            const uint32_t pos = wave_append(true, &s_k);
            if (pos < N) own[pos] = c;
            if (listed + pos < out_cap) out[listed + pos] = ks;
            f.mark(c);
          },
          &bad, &local, f);
      if (j + 1 < (uint32_t)R) __syncthreads();
    }
    if (bad) s_bad = 1;
    atomicAdd(&s_sum, (unsigned long long)local);
  }
  __syncthreads();
  uint32_t t = 1;
  for (;; ++t) {
    const uint32_t K = s_k;
    if (K == 0) break;
    if (t > max_rounds) {
      if (tid == 0) s_flags |= PEEL_FLAG_EROUNDS;
      break;
    }
    if (listed + K > out_cap) {
      if (tid == 0) s_flags |= PEEL_FLAG_ENOSPC;
      break;
    }
    if (tid == 0) {
      stats[t - 1] = K;
      s_c = 0;
    }
    f.clear(tid, NT);
    __syncthreads();
    apply_exclusive<R, NT>(h, cells, out + listed, own, K, hset, [&](uint32_t c) {
      cand[wave_append(true, &s_c)] = c;
      f.mark(c);
    });
    __syncthreads();
    listed += K;
    const uint32_t nc = s_c;
    if (tid == 0) s_k = 0;
    __syncthreads();
    uint32_t bad = 0;
    long long unused = 0;
    detect_cells<R, false>(
        h, cells, 0, nc, tid, NT, [&](uint64_t i) { return cand[i]; },
        [&](uint64_t ks, uint32_t c) {
          const uint32_t pos = wave_append(true, &s_k);
          own[pos] = c;
          if (listed + pos < out_cap) out[listed + pos] = ks;
        },
        &bad, &unused, f);
    if (bad) s_bad = 1;
    __syncthreads();
  }
  if (tid == 0) {
    const long long keys = (long long)s_sum / (long long)R;
    summary[0] = listed;
    summary[1] = t - 1 < max_rounds ? t - 1 : max_rounds;
    summary[2] = (uint64_t)(keys - (long long)listed);
    summary[3] = s_flags | (s_bad ? PEEL_FLAG_ECORRUPT : 0u);
    summary[4] = 1;
    summary[5] = summary[6] = summary[7] = 0;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Team ("tile") schedule for large tables: Gt workgroups of the one launch list
// one table together.  Member g takes cells [g N / Gt, (g+1) N / Gt) in round
// 1, then the keys it found and the cells it pushed; the cells are shared, so
// keys leave them with device atomics, and a barrier among the members (one
// per table) ends each detect and each apply.  Same rounds, key sets and
// summary as the single-workgroup schedules.
struct TeamCtrl {
  GridSync bar;
  uint32_t kpos[2];            // keys found this round, by round parity
  uint32_t flags;
  uint32_t bad;
  unsigned long long sum;      // counts of every cell at the start
  uint32_t pad[6];
};
static_assert(sizeof(TeamCtrl) == 64, "one line per table");

template <int R, int NT>
__device__ void list_table_team(const iblt_desc desc, iblt_cell *cells, uint32_t N, uint64_t *out,
                                uint64_t out_cap, uint64_t *stats, uint32_t max_rounds,
                                uint64_t *summary, uint32_t *cand, uint32_t *own, uint32_t g,
                                uint32_t Gt, TeamCtrl *tc, uint64_t limit) {
  const Hash h = make_hash_fixed<R>(desc);
  __shared__ uint32_t s_k, s_c, s_bad, s_pos;
  __shared__ unsigned long long s_sum;
  const uint32_t tid = threadIdx.x;
  if (g == 0)
    for (uint32_t i = tid; i < max_rounds; i += NT) stats[i] = 0;
  if (tid == 0) {
    s_k = 0;
    s_bad = 0;
    s_sum = 0;
  }
  __syncthreads();
  // round-1 detect over my slice of the cells
  {
    const uint32_t c0 = (uint32_t)((uint64_t)N * g / Gt), c1 = (uint32_t)((uint64_t)N * (g + 1) / Gt);
    long long local = 0;
    uint32_t bad = 0;
    for (uint32_t c = c0 + tid; c < c1; c += NT) {
      int32_t cnt;
      uint64_t ks, hs;
      load_cell(cells + c, &cnt, &ks, &hs);
      local += cnt;
      if (owns<R>(h, cells, c, cnt, ks, hs, &bad)) own[wave_append(true, &s_k)] = c;
    }
    if (bad) s_bad = 1;
    atomicAdd(&s_sum, (unsigned long long)local);
  }
  uint64_t listed = 0;
  uint32_t t = 1;
  bool ok = true;
  for (;; ++t) {
    __syncthreads();
    const uint32_t mine = s_k;
    if (tid == 0) {
      s_pos = atomicAdd(&tc->kpos[t & 1], mine);
      if (t == 1) atomicAdd(&tc->sum, s_sum);
      if (s_bad) atomicOr(&tc->bad, 1u);
    }
    // the keys go to out only once the round is known to fit; the cells
    // still hold them until the apply, which starts after the barrier
    if (!grid_barrier(&tc->bar, Gt, limit)) {
      ok = false;
      break;
    }
    const uint32_t K = atomic_load_u32(&tc->kpos[t & 1]);
    if (K == 0) break;
    if (t > max_rounds) {
      if (g == 0 && tid == 0) atomicOr(&tc->flags, PEEL_FLAG_EROUNDS);
      break;
    }
    if (listed + K > out_cap) {
      if (g == 0 && tid == 0) atomicOr(&tc->flags, PEEL_FLAG_ENOSPC);
      break;
    }
    if (g == 0 && tid == 0) {
      stats[t - 1] = K;
      // every member read last round's total before this barrier
      __hip_atomic_store(&tc->kpos[(t + 1) & 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t base = (uint32_t)listed + s_pos;
    for (uint32_t i = tid; i < mine; i += NT) {
      int32_t cnt;
      uint64_t ks, hs;
      load_cell(cells + own[i], &cnt, &ks, &hs);
      out[base + i] = ks;
    }
    if (tid == 0) s_c = 0;
    __syncthreads();
    for (uint32_t i = tid; i < mine; i += NT)
      delete_key<R>(h, cells, out[base + i], own[i], [&](uint32_t c) { cand[wave_append(true, &s_c)] = c; });
    listed += K;
    if (!grid_barrier(&tc->bar, Gt, limit)) {
      ok = false;
      break;
    }
    const uint32_t nc = s_c;
    if (tid == 0) s_k = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (uint32_t i = tid; i < nc; i += NT) {
      const uint32_t c = cand[i];
      int32_t cnt;
      uint64_t ks, hs;
      load_cell(cells + c, &cnt, &ks, &hs);
      if (owns<R>(h, cells, c, cnt, ks, hs, &bad)) own[wave_append(true, &s_k)] = c;
    }
    if (bad) s_bad = 1;
  }
  // Every member stops at the same round (the totals are the team's), so
  // member 0 writes the summary with no further barrier: the flags and counts
  // it reads were all in before the barrier that ended the detect.
  if (g == 0) {
    if (tid == 0) {
      const long long keys = (long long)atomic_load_u64(reinterpret_cast<uint64_t *>(&tc->sum)) / (long long)R;
      summary[0] = listed;
      summary[1] = t - 1 < max_rounds ? t - 1 : max_rounds;
      summary[2] = (uint64_t)(keys - (long long)listed);
      summary[3] = atomic_load_u32(&tc->flags) | (atomic_load_u32(&tc->bad) ? PEEL_FLAG_ECORRUPT : 0u) |
                   (ok ? 0u : PEEL_FLAG_TIMEOUT);
      summary[4] = Gt;
      summary[5] = summary[6] = summary[7] = 0;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// LDS-resident schedule for small tables: the table is read once into the
// workgroup's local memory (structure of arrays), every round's detect and
// apply run on it with LDS atomics, and the final cells are written back.
// Same rounds and key sets as the in-place schedule.

// The most cells an NT-thread workgroup lists from LDS: what its share of the
// CU's LDS holds at 24 bytes a cell (kBatchLdsWords below).
template <int NT>
constexpr uint32_t kLdsCap = NT == 1024 ? 5120u : NT == 512 ? 3072u : 2048u;
constexpr uint32_t kLdsCells = kLdsCap<1024>;
static_assert(kLdsCells == IBLT_LDS_MAX_CELLS, "the header's limit is the largest capacity");

template <uint32_t Cap>
struct LdsTable {
  int32_t cnt[Cap];
  uint64_t ks[Cap];
  uint64_t hs[Cap];
  uint16_t own[Cap];   // cells whose key this round lists (at most one per cell)
  uint16_t cand[Cap];  // cells that went 2 -> 1 this round (at most once each)
};

template <int R, typename Table>
__device__ inline bool owns_lds(const Hash &h, const Table &T, uint32_t c, uint32_t *bad) {
  if (T.cnt[c] != 1) return false;
  const uint64_t ks = T.ks[c];
  const uint64_t hx = check_of(h, ks);
  if (T.hs[c] != hx) {
    *bad = 1;
    return false;
  }
  const uint32_t j = subtable_of(h, c);
#pragma unroll
  for (int i = 0; i < R - 1; ++i) {
    if (i >= (int)j) break;
    const uint32_t o = cell_of(h, i, ks);
    if (T.cnt[o] == 1 && T.ks[o] == ks && T.hs[o] == hx) return false;
  }
  return true;
}

template <int R, int NT>
__device__ void list_table_lds(const iblt_desc desc, iblt_cell *cells, uint32_t N, uint64_t *out,
                               uint64_t out_cap, uint64_t *stats, uint32_t max_rounds,
                               uint64_t *summary, LdsTable<kLdsCap<NT>> &T) {
  const Hash h = make_hash_fixed<R>(desc);
  __shared__ uint32_t s_k, s_c, s_bad, s_flags;
  __shared__ unsigned long long s_sum;
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < max_rounds; i += NT) stats[i] = 0;
  if (tid == 0) {
    s_k = 0;
    s_bad = 0;
    s_flags = 0;
    s_sum = 0;
  }
  {
    long long local = 0;
    for (uint32_t c = tid; c < N; c += NT) {
      int32_t cnt;
      uint64_t ks, hs;
      load_cell(cells + c, &cnt, &ks, &hs);
      T.cnt[c] = cnt;
      T.ks[c] = ks;
      T.hs[c] = hs;
      local += cnt;
    }
    __syncthreads();
    atomicAdd(&s_sum, (unsigned long long)local);
  }
  uint64_t listed = 0;
  {
    uint32_t bad = 0;
    for (uint32_t c = tid; c < N; c += NT) {
      if (owns_lds<R>(h, T, c, &bad)) {
        const uint32_t pos = wave_append(true, &s_k);
        T.own[pos] = static_cast<uint16_t>(c);
        if (pos < out_cap) out[pos] = T.ks[c];
      }
    }
    if (bad) s_bad = 1;
  }
  __syncthreads();
  uint32_t t = 1;
  for (;; ++t) {
    const uint32_t K = s_k;
    if (K == 0) break;
    if (t > max_rounds) {
      if (tid == 0) s_flags |= PEEL_FLAG_EROUNDS;
      break;
    }
    if (listed + K > out_cap) {
      if (tid == 0) s_flags |= PEEL_FLAG_ENOSPC;
      break;
    }
    if (tid == 0) {
      stats[t - 1] = K;
      s_c = 0;
    }
    __syncthreads();
    // apply: the listed key of cell own[i] is still that cell's key_sum
    for (uint32_t i = tid; i < K; i += NT) {
      const uint32_t co = T.own[i];
      const uint64_t x = T.ks[co];
      const uint64_t hx = check_of(h, x);
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint32_t c = cell_of(h, j, x);
        if (c == co) continue;
        const int32_t old = atomicSub(&T.cnt[c], 1);
        atomicXor(reinterpret_cast<unsigned long long *>(&T.ks[c]), (unsigned long long)x);
        atomicXor(reinterpret_cast<unsigned long long *>(&T.hs[c]), (unsigned long long)hx);
        if (old == 2) T.cand[wave_append(true, &s_c)] = static_cast<uint16_t>(c);
      }
    }
    __syncthreads();
    // the owner cells held their key alone: clear them after every key was read
    for (uint32_t i = tid; i < K; i += NT) {
      const uint32_t co = T.own[i];
      T.cnt[co] = 0;
      T.ks[co] = 0;
      T.hs[co] = 0;
    }
    listed += K;
    const uint32_t nc = s_c;
    __syncthreads();
    if (tid == 0) s_k = 0;
    __syncthreads();
    uint32_t bad = 0;
    for (uint32_t i = tid; i < nc; i += NT) {
      const uint32_t c = T.cand[i];
      if (owns_lds<R>(h, T, c, &bad)) {
        const uint32_t pos = wave_append(true, &s_k);
        T.own[pos] = static_cast<uint16_t>(c);
        if (listed + pos < out_cap) out[listed + pos] = T.ks[c];
      }
    }
    if (bad) s_bad = 1;
    __syncthreads();
  }
  for (uint32_t c = tid; c < N; c += NT) {
    uint4 *p = reinterpret_cast<uint4 *>(cells + c);
    const uint64_t ks = T.ks[c], hs = T.hs[c];
    p[0] = make_uint4(static_cast<uint32_t>(T.cnt[c]), 0u, static_cast<uint32_t>(ks),
                      static_cast<uint32_t>(ks >> 32));
    p[1] = make_uint4(static_cast<uint32_t>(hs), static_cast<uint32_t>(hs >> 32), 0u, 0u);
  }
  if (tid == 0) {
    const long long keys = (long long)s_sum / (long long)R;
    summary[0] = listed;
    summary[1] = t - 1 < max_rounds ? t - 1 : max_rounds;
    summary[2] = (uint64_t)(keys - (long long)listed);
    summary[3] = s_flags | (s_bad ? PEEL_FLAG_ECORRUPT : 0u);
    summary[4] = 1;
    summary[5] = summary[6] = summary[7] = 0;
  }
  __syncthreads();
}

struct BatchCtrl {
  uint32_t ticket;
  uint32_t units;  // work units: one per table, tile_workgroups per team table
  uint32_t pad[62];
};

// first/teams: null when the team schedule is off (a work unit is then a table).
// LDS words of one batched-listing workgroup.  A 1024-thread workgroup is
// alone on its CU by its registers (128 VGPRs), so it takes 128 KiB.  A
// 512-thread one takes 78 KiB (two fit in a CU's 160 KiB), a 256-thread one
// 48 KiB with the LDS table (three fit) or 39 KiB without it (four).
template <int NT, bool LDS>
constexpr uint32_t kBatchLdsWords = NT == 1024 ? 32768u : NT == 512 ? 19968u : LDS ? 12288u : 9984u;

template <int NT, bool LDS>
__global__ void __launch_bounds__(NT)
    k_list_batched(const iblt_batch_entry *entries, uint32_t ntables, uint32_t max_rounds,
                   BatchCtrl *ctrl, uint32_t *scratch, uint64_t max_cells, uint32_t lds_max,
                   const uint32_t *first, TeamCtrl *teams, uint64_t limit) {
  __shared__ uint32_t s_t;
  // the LDS-resident table, or the in-place schedule's hash set and filter
  __shared__ __align__(16) uint32_t region[kBatchLdsWords<NT, LDS>];
  using Table = LdsTable<kLdsCap<NT>>;
  static_assert(!LDS || sizeof(Table) <= sizeof(region), "the LDS table fits");
  static_assert(kBatchLdsWords<NT, LDS> >= kApplySet<NT> + 1024, "the filter has room");
  Table &lt = *reinterpret_cast<Table *>(region);
  uint32_t *hset = region;
  uint32_t *filt = region + kApplySet<NT>;
  constexpr uint32_t filt_words = kBatchLdsWords<NT, LDS> - kApplySet<NT>;
  uint32_t *cand = scratch + (uint64_t)blockIdx.x * 2 * max_cells;
  uint32_t *own = cand + max_cells;
  __shared__ uint32_t s_g, s_gt;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint32_t u = atomicAdd(&ctrl->ticket, 1u);
      uint32_t ti = u, g = 0, gt = 1;
      if (first) {
        // the table whose units hold unit u: the last i with first[i] <= u
        uint32_t lo = 0, hi = ntables;
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (first[mid] <= u) lo = mid; else hi = mid;
        }
        ti = u < first[ntables] ? lo : ntables;
        if (ti < ntables) {
          g = u - first[ti];
          gt = first[ti + 1] - first[ti];
        }
      }
      s_t = ti;
      s_g = g;
      s_gt = gt;
    }
    __syncthreads();
    // the same in every lane: read once, so the entry and its hash are scalar
    const uint32_t ti = __builtin_amdgcn_readfirstlane(s_t);
    const uint32_t g = __builtin_amdgcn_readfirstlane(s_g);
    const uint32_t gt = __builtin_amdgcn_readfirstlane(s_gt);
    __syncthreads();
    if (ti >= ntables) return;
    const iblt_batch_entry e = entries[ti];
    if (e.desc.r < 2 || e.desc.r > 8 || e.desc.ncells < e.desc.r || e.desc.ncells > max_cells ||
        !e.cells || (reinterpret_cast<uintptr_t>(e.cells) & 31u)) {
      // a bad entry is skipped: listing it could overrun this workgroup's scratch
      if (e.summary && threadIdx.x < 8) e.summary[threadIdx.x] = threadIdx.x == 3 ? PEEL_FLAG_EINVAL : 0u;
      continue;
    }
    const uint32_t N = static_cast<uint32_t>(e.desc.ncells);
    if (gt > 1) {
#define PEEL_TEAM_CASE(RR)                                                                        \
  case RR:                                                                                        \
    list_table_team<RR, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds,     \
                            e.summary, cand, own, g, gt, teams + ti, limit);                      \
    break;
      switch (e.desc.r) {
        PEEL_TEAM_CASE(2)
        PEEL_TEAM_CASE(3)
        PEEL_TEAM_CASE(4)
        PEEL_TEAM_CASE(5)
        PEEL_TEAM_CASE(6)
        PEEL_TEAM_CASE(7)
        PEEL_TEAM_CASE(8)
      }
#undef PEEL_TEAM_CASE
      continue;
    }
    if constexpr (LDS) {
      if (N <= lds_max && N <= kLdsCap<NT>) {
#define PEEL_LDS_CASE(RR) \
  case RR: list_table_lds<RR, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, lt); break;
        switch (e.desc.r) {
          PEEL_LDS_CASE(2)
          PEEL_LDS_CASE(3)
          PEEL_LDS_CASE(4)
          PEEL_LDS_CASE(5)
          PEEL_LDS_CASE(6)
          PEEL_LDS_CASE(7)
          default: list_table_lds<8, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, lt); break;
        }
#undef PEEL_LDS_CASE
        continue;
      }
    }
    switch (e.desc.r) {
      case 2: list_table_block<2, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, cand, own, hset, filt, filt_words); break;
      case 3: list_table_block<3, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, cand, own, hset, filt, filt_words); break;
      case 4: list_table_block<4, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, cand, own, hset, filt, filt_words); break;
      case 5: list_table_block<5, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, cand, own, hset, filt, filt_words); break;
      case 6: list_table_block<6, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, cand, own, hset, filt, filt_words); break;
      case 7: list_table_block<7, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, cand, own, hset, filt, filt_words); break;
      default: list_table_block<8, NT>(e.desc, e.cells, N, e.out_keys, e.out_cap, e.round_stats, max_rounds, e.summary, cand, own, hset, filt, filt_words); break;
    }
  }
}

// Clears the ticket; with the team schedule on, also gives each table its
// work units (tile_workgroups for a table of at least tile_min cells, else 1),
// their exclusive prefix in `first` (ntables + 1 entries), and a cleared
// TeamCtrl per table.  One workgroup of kInitT threads.
constexpr int kInitT = 1024;
__global__ void __launch_bounds__(kInitT)
    k_batch_init(BatchCtrl *ctrl, const iblt_batch_entry *entries, uint32_t ntables,
                 uint32_t tile_min, uint32_t tile_g, uint32_t *first, TeamCtrl *teams) {
  __shared__ uint32_t lds[kInitT / kWave + 1];
  if (threadIdx.x == 0) {
    ctrl->ticket = 0;
    ctrl->units = ntables;
  }
  if (tile_g < 2) return;
  uint32_t base = 0;
  for (uint32_t i0 = 0; i0 < ntables; i0 += kInitT) {
    const uint32_t i = i0 + threadIdx.x;
    uint32_t u = 0;
    if (i < ntables) {
      u = entries[i].desc.ncells >= tile_min ? tile_g : 1u;
      uint32_t *w = reinterpret_cast<uint32_t *>(teams + i);
      for (int q = 0; q < (int)(sizeof(TeamCtrl) / 4); ++q) w[q] = 0;
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan<kInitT>(u, &tot, lds);
    if (i < ntables) first[i] = base + ex;
    base += tot;
  }
  if (threadIdx.x == 0) {
    first[ntables] = base;
    ctrl->units = base;
  }
}

// ===========================================================================
// Host side.

struct ListLayout {
  size_t ctrl, skeys, scells, cand, okeys, ocells, ocand, total;
  uint32_t grid, cb;
};

// grid: the persistent workgroups asked for (0 = one per CU; at most one per CU).
// Cells per persistent workgroup that a listing's default team aims at: a
// smaller table is listed by fewer workgroups (measured on 2^10 .. 2^24 cells,
// this is within a few percent of the best team size at every size, and the
// whole GPU from 2^20 cells).
constexpr uint64_t kListCellsPerWG = 4096;

ListLayout list_layout(uint64_t ncells, uint32_t want) {
  ListLayout L{};
  const uint32_t cus = static_cast<uint32_t>(device_info().cus);  // 1024-thread workgroups
  const uint64_t by_size = (ncells + kListCellsPerWG - 1) / kListCellsPerWG;
  const uint32_t dflt = by_size < cus ? (by_size ? static_cast<uint32_t>(by_size) : 1u) : cus;
  L.grid = want == 0 ? dflt : (want > cus ? cus : want);
  L.cb = static_cast<uint32_t>((ncells + L.grid - 1) / L.grid + 4096);
  const uint64_t slots = (uint64_t)L.grid * L.cb;
  L.ctrl = align_up(sizeof(ListCtrl));
  L.skeys = align_up(slots * 8);
  L.scells = align_up(slots * 4);
  L.cand = align_up(slots * 4);
  L.okeys = align_up(ncells * 8);
  L.ocells = align_up(ncells * 4);
  L.ocand = align_up(2 * ncells * 4);
  L.total = L.ctrl + L.skeys + L.scells + L.cand + L.okeys + L.ocells + L.ocand;
  return L;
}

bool desc_ok(const iblt_desc *d) {
  return d && d->r >= 2 && d->r <= 8 && d->ncells >= d->r && d->ncells < (1ull << 32);
}

template <int R>
peel_status launch_insert(const Hash &h, iblt_cell *cells, const uint64_t *keys, uint64_t nkeys,
                          hipStream_t s, int32_t sign) {
  const unsigned grid = grid_for(nkeys, kBlock, 1u << 16);
  hipLaunchKernelGGL(k_insert<R>, dim3(grid), dim3(kBlock), 0, s, h, cells, keys, nkeys, sign);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

template <int R>
peel_status launch_list(ListArgs &a, hipStream_t s, bool subtables) {
  if (device_info().debug) std::fprintf(stderr, "[peel] list grid %u\n", a.grid);
  if (subtables)
    hipLaunchKernelGGL(k_list_sub<R>, dim3(a.grid), dim3(kLT), 0, s, a);
  else if (a.signed_list)
    hipLaunchKernelGGL((k_list_persistent<R, true>), dim3(a.grid), dim3(kLT), 0, s, a);
  else
    hipLaunchKernelGGL((k_list_persistent<R, false>), dim3(a.grid), dim3(kLT), 0, s, a);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

// Workspace: the control block, two max_cells lists per workgroup, then (for
// the team schedule) the tables' first work units and their TeamCtrl.
struct BatchLayout {
  size_t ctrl, lists, first, teams, total;
};

BatchLayout batched_layout(uint32_t ntables, uint64_t max_cells, uint32_t grid) {
  BatchLayout L{};
  L.ctrl = align_up(sizeof(BatchCtrl));
  L.lists = align_up((uint64_t)grid * 2 * max_cells * 4);
  L.first = align_up(((uint64_t)ntables + 1) * 4);
  L.teams = align_up((uint64_t)ntables * sizeof(TeamCtrl));
  L.total = L.ctrl + L.lists + L.first + L.teams;
  return L;
}

constexpr uint32_t kTeamMax = 64;  // most workgroups in one team

// Workgroups of a launch: two per CU, fewer for a batch with fewer tables (or,
// with teams, fewer table units).  The workspace is sized for the most any
// schedule launches.
uint32_t batched_grid(uint32_t ntables, uint32_t tile_g = 1) {
  const uint64_t g = 2ull * device_info().cus;
  const uint64_t want = (uint64_t)(ntables ? ntables : 1) * (tile_g ? tile_g : 1);
  return static_cast<uint32_t>(want < g ? want : g);
}

size_t batched_ws_bytes(uint32_t ntables, uint64_t max_cells, uint32_t grid) {
  return batched_layout(ntables, max_cells, grid).total;
}

}  // namespace
}  // namespace peel

using namespace peel;

namespace peel {
namespace {

peel_status update_run(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                       uint64_t nkeys, void *stream, int32_t sign) {
  if (!desc_ok(desc) || !cells || (nkeys && !keys)) return PEEL_EINVAL;
  if (reinterpret_cast<uintptr_t>(cells) % 32) return PEEL_EINVAL;
  if (nkeys == 0) return PEEL_OK;
  const Hash h = make_hash(*desc);
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (desc->r) {
    case 2: return launch_insert<2>(h, cells, keys, nkeys, s, sign);
    case 3: return launch_insert<3>(h, cells, keys, nkeys, s, sign);
    case 4: return launch_insert<4>(h, cells, keys, nkeys, s, sign);
    case 5: return launch_insert<5>(h, cells, keys, nkeys, s, sign);
    case 6: return launch_insert<6>(h, cells, keys, nkeys, s, sign);
    case 7: return launch_insert<7>(h, cells, keys, nkeys, s, sign);
    default: return launch_insert<8>(h, cells, keys, nkeys, s, sign);
  }
}

struct UpdSizes {
  uint32_t nsb, ntiles;
  uint64_t hist, entries;
};

UpdSizes upd_sizes(const iblt_desc *d, uint64_t nkeys) {
  UpdSizes z{};
  z.nsb = static_cast<uint32_t>((d->ncells + (1ull << kUSuperShift) - 1) >> kUSuperShift);
  z.ntiles = static_cast<uint32_t>((nkeys + kUTile - 1) / kUTile);
  z.hist = (uint64_t)z.nsb * (z.ntiles ? z.ntiles : 1);
  z.entries = (uint64_t)d->r * nkeys;
  return z;
}

// The binned update runs up to 2^24 cells and while entry places fit 32 bits.
bool upd_binned(const iblt_desc *d, uint64_t nkeys) {
  const UpdSizes z = upd_sizes(d, nkeys);
  return nkeys > 0 && z.nsb <= kUMaxSuper && z.entries < (1ull << 32) && z.hist < (1ull << 32);
}

size_t upd_ws_bytes(const iblt_desc *d, uint64_t nkeys) {
  if (!upd_binned(d, nkeys)) return 256;
  const UpdSizes z = upd_sizes(d, nkeys);
  return align_up(z.hist * 4) + align_up((scan_tiles(z.hist) + 1) * 4) + align_up(16) +
         align_up(z.entries * 8) + align_up(z.entries * 2);
}

// nkeys_dev (if given): the key count, read on the device; nkeys is then the
// most there can be and sizes the grids and the workspace.
template <int R>
peel_status launch_update_binned(const Hash &h, const iblt_desc *d, iblt_cell *cells,
                                 const uint64_t *keys, uint64_t nkeys, int32_t sign, void *ws,
                                 hipStream_t s, const unsigned long long *nkeys_dev = nullptr) {
  const UpdSizes z = upd_sizes(d, nkeys);
  Carver c(ws);
  uint32_t *hist = c.take<uint32_t>(z.hist);
  uint32_t *part = c.take<uint32_t>(scan_tiles(z.hist) + 1);
  uint32_t *total = c.take<uint32_t>(4);
  uint64_t *ekey = c.take<uint64_t>(z.entries);
  uint16_t *eloc = c.take<uint16_t>(z.entries);
  hipLaunchKernelGGL(k_upd_count<R>, dim3(z.ntiles), dim3(kUT), 0, s, h, keys, nkeys, z.nsb,
                     z.ntiles, hist, nkeys_dev);
  scan_u32(hist, z.hist, hist, nullptr, part, nullptr, total, nullptr, s);
  hipLaunchKernelGGL(k_upd_scatter<R>, dim3(z.ntiles), dim3(kUT), 0, s, h, keys, nkeys, z.nsb,
                     z.ntiles, hist, ekey, eloc, nkeys_dev);
  hipLaunchKernelGGL(k_upd_apply<R>, dim3(z.nsb * kUPer), dim3(kUT), 0, s, h, cells, d->ncells,
                     ekey, eloc, hist, z.nsb, z.ntiles, total, sign);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

peel_status update_binned_run(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                              uint64_t nkeys, int32_t sign, void *ws, size_t ws_bytes,
                              void *stream) {
  if (!desc_ok(desc) || !cells || (nkeys && !keys)) return PEEL_EINVAL;
  if (reinterpret_cast<uintptr_t>(cells) % 32) return PEEL_EINVAL;
  if (sign != 1 && sign != -1) return PEEL_EINVAL;
  if (nkeys == 0) return PEEL_OK;
  if (!upd_binned(desc, nkeys)) return update_run(desc, cells, keys, nkeys, stream, sign);
  if (!ws) return PEEL_EINVAL;
  if (ws_bytes < upd_ws_bytes(desc, nkeys)) return PEEL_ENOSPC;
  const Hash h = make_hash(*desc);
  hipStream_t s = static_cast<hipStream_t>(stream);
  switch (desc->r) {
    case 2: return launch_update_binned<2>(h, desc, cells, keys, nkeys, sign, ws, s);
    case 3: return launch_update_binned<3>(h, desc, cells, keys, nkeys, sign, ws, s);
    case 4: return launch_update_binned<4>(h, desc, cells, keys, nkeys, sign, ws, s);
    case 5: return launch_update_binned<5>(h, desc, cells, keys, nkeys, sign, ws, s);
    case 6: return launch_update_binned<6>(h, desc, cells, keys, nkeys, sign, ws, s);
    case 7: return launch_update_binned<7>(h, desc, cells, keys, nkeys, sign, ws, s);
    default: return launch_update_binned<8>(h, desc, cells, keys, nkeys, sign, ws, s);
  }
}

}  // namespace
}  // namespace peel

extern "C" peel_status iblt_insert(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                                   uint64_t nkeys, void *stream) {
  return update_run(desc, cells, keys, nkeys, stream, 1);
}

extern "C" size_t iblt_update_workspace(const iblt_desc *desc, uint64_t nkeys) {
  if (!desc_ok(desc)) return 0;
  return upd_ws_bytes(desc, nkeys);
}

extern "C" peel_status iblt_update(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                                   uint64_t nkeys, int32_t sign, void *ws, size_t ws_bytes,
                                   void *stream) {
  return update_binned_run(desc, cells, keys, nkeys, sign, ws, ws_bytes, stream);
}

extern "C" peel_status iblt_delete(const iblt_desc *desc, iblt_cell *cells, const uint64_t *keys,
                                   uint64_t nkeys, void *stream) {
  return update_run(desc, cells, keys, nkeys, stream, -1);
}

namespace peel {
namespace {

// A plain listing of a large table on the whole GPU runs its first round's
// removals through the binned update (its keys are the first round's output).
constexpr uint64_t kListBinnedMin = 1ull << 20;

bool list_first_binned_fits(const iblt_desc *d) {
  return d->workgroups == 0 && d->ncells >= kListBinnedMin && upd_binned(d, d->ncells);
}

// The owner engine's arrays: keys, their cells, the candidates and their keys (one
// entry per cell), (r-1) 16-byte messages per cell, and the owners' message tables.
// A team of T workgroups owns pieces of ceil(size_j / T) cells of each
// subtable: T * sum_j ceil(size_j / T) <= N + r * T places in all.
size_t owner_ws_bytes(const iblt_desc *d) {
  const ListLayout L = list_layout(d->ncells, d->workgroups);
  const uint64_t g = L.grid, N = d->ncells + (uint64_t)d->r * g;
  return L.ctrl + 2 * align_up(N * 8) + 2 * align_up(N * 4) +
         align_up((uint64_t)(d->r - 1) * N * 16) + 2 * align_up(g * g * 4);
}

size_t list_ws_bytes(const iblt_desc *d) {
  const ListLayout L = list_layout(d->ncells, d->workgroups);
  size_t need = L.total;
  const size_t o = owner_ws_bytes(d);
  need = o > need ? o : need;
  if (list_first_binned_fits(d)) {
    const size_t b = L.ctrl + upd_ws_bytes(d, d->ncells);
    need = b > need ? b : need;
  }
  return need;
}

template <int R>
peel_status first_round_binned(const iblt_desc *d, const Hash &h, iblt_cell *cells, uint64_t *out,
                                ListCtrl *ctrl, void *ws, hipStream_t s) {
  const uint32_t N = static_cast<uint32_t>(d->ncells);
  const uint32_t grid = static_cast<uint32_t>(4 * device_info().cus);
  hipLaunchKernelGGL(k_list_detect1<R>, dim3(grid), dim3(kBlock), 0, s, h, cells, N, out, ctrl);
  PEEL_HIP_TRY(hipGetLastError());
  // every key of round 1 leaves its r cells; its own cell comes out empty
  return launch_update_binned<R>(h, d, cells, out, d->ncells, -1, ws, s, &ctrl->first_keys);
}

}  // namespace
}  // namespace peel

extern "C" size_t iblt_list_workspace(const iblt_desc *desc) {
  return desc_ok(desc) ? list_ws_bytes(desc) : 0;
}

namespace peel {
namespace {

peel_status list_run(const iblt_desc *desc, iblt_cell *cells, uint64_t *out_keys,
                     uint64_t out_cap, uint64_t *round_stats, uint32_t max_rounds,
                     uint64_t *summary, void *ws, size_t ws_bytes, void *stream, bool subtables,
                     int8_t *out_signs = nullptr, bool signed_list = false) {
  if (!desc_ok(desc) || !cells || (out_cap && !out_keys) || !round_stats || !summary || !ws ||
      max_rounds == 0 || (signed_list && out_cap && !out_signs))
    return PEEL_EINVAL;
  if (reinterpret_cast<uintptr_t>(cells) % 32) return PEEL_EINVAL;
  const ListLayout L = list_layout(desc->ncells, desc->workgroups);
  if (ws_bytes < L.total) return PEEL_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ws);
  ListArgs a{};
  a.h = make_hash(*desc);
  a.ctrl = reinterpret_cast<ListCtrl *>(base);
  base += L.ctrl;
  a.skeys = reinterpret_cast<uint64_t *>(base);
  base += L.skeys;
  a.scells = reinterpret_cast<uint32_t *>(base);
  base += L.scells;
  a.cand = reinterpret_cast<uint32_t *>(base);
  base += L.cand;
  a.okeys = reinterpret_cast<uint64_t *>(base);
  base += L.okeys;
  a.ocells = reinterpret_cast<uint32_t *>(base);
  base += L.ocells;
  a.ocand = reinterpret_cast<uint32_t *>(base);
  a.cells = cells;
  a.out = out_keys;
  a.out_cap = out_cap;
  a.stats = round_stats;
  a.signs = out_signs;
  a.signed_list = signed_list ? 1u : 0u;
  a.limit = barrier_limit_ticks();
  a.team_limit = device_info().team_limit_ticks;
  a.quiet = device_info().team_quiet_ticks;
  a.ncells = static_cast<uint32_t>(desc->ncells);
  a.max_rounds = max_rounds;
  a.cb = L.cb;
  // PEEL_LIST_SLOT_CAP: a smaller staging slot per workgroup, so that the
  // overflow queues take the keys and candidates past it (for testing them)
  const long slot_cap = env_long("PEEL_LIST_SLOT_CAP", 0);
  if (slot_cap > 0 && (uint64_t)slot_cap < a.cb) a.cb = static_cast<uint32_t>(slot_cap);
  a.grid = L.grid;
  a.first_binned = 0;
  hipLaunchKernelGGL(k_list_init, dim3(1), dim3(256), 0, s, a.ctrl,
                     barrier_slots() ? 1u : 0u);
  PEEL_HIP_TRY(hipGetLastError());
  peel_status st;
  // The plain listing runs on the owner engine; PEEL_LIST_ENGINE=atomic (or a
  // PEEL_LIST_SLOT_CAP, which exercises the atomic kernel's overflow queues)
  // selects the persistent kernel with device-atomic deletes instead.
  const char *eng = std::getenv("PEEL_LIST_ENGINE");
  const bool atomic_engine = (eng && std::strcmp(eng, "atomic") == 0) || slot_cap > 0;
  if (!subtables && !signed_list && !atomic_engine) {
    if (ws_bytes < owner_ws_bytes(desc)) return PEEL_ENOSPC;
    OwnArgs o{};
    o.h = a.h;
    o.cells = cells;
    o.out = out_keys;
    o.out_cap = out_cap;
    o.stats = round_stats;
    o.ctrl = a.ctrl;
    o.limit = a.limit;
    o.quiet = a.quiet;
    o.team_limit = a.team_limit;
    o.ncells = a.ncells;
    o.max_rounds = max_rounds;
    o.grid = L.grid;
    const uint64_t g = L.grid, N = desc->ncells + (uint64_t)desc->r * g;
    char *ob = static_cast<char *>(ws) + L.ctrl;
    o.keys = reinterpret_cast<uint64_t *>(ob);
    ob += align_up(N * 8);
    o.ownc = reinterpret_cast<uint32_t *>(ob);
    ob += align_up(N * 4);
    o.cand = reinterpret_cast<uint32_t *>(ob);
    ob += align_up(N * 4);
    o.candk = reinterpret_cast<uint64_t *>(ob);
    ob += align_up(N * 8);
    o.msg = reinterpret_cast<uint4 *>(ob);
    ob += align_up((uint64_t)(desc->r - 1) * N * 16);
    o.mcnt = reinterpret_cast<uint32_t *>(ob);
    ob += align_up(g * g * 4);
    o.moff = reinterpret_cast<uint32_t *>(ob);
    if (device_info().debug) std::fprintf(stderr, "[peel] list owner grid %u\n", o.grid);
    switch (desc->r) {
      case 2: hipLaunchKernelGGL(k_list_owner<2>, dim3(o.grid), dim3(kLT), 0, s, o); break;
      case 3: hipLaunchKernelGGL(k_list_owner<3>, dim3(o.grid), dim3(kLT), 0, s, o); break;
      case 4: hipLaunchKernelGGL(k_list_owner<4>, dim3(o.grid), dim3(kLT), 0, s, o); break;
      case 5: hipLaunchKernelGGL(k_list_owner<5>, dim3(o.grid), dim3(kLT), 0, s, o); break;
      case 6: hipLaunchKernelGGL(k_list_owner<6>, dim3(o.grid), dim3(kLT), 0, s, o); break;
      case 7: hipLaunchKernelGGL(k_list_owner<7>, dim3(o.grid), dim3(kLT), 0, s, o); break;
      default: hipLaunchKernelGGL(k_list_owner<8>, dim3(o.grid), dim3(kLT), 0, s, o); break;
    }
    PEEL_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_list_finish, dim3(1), dim3(64), 0, s, a.ctrl, desc->r, summary, 0u,
                       round_stats, 0u);
    PEEL_HIP_TRY(hipGetLastError());
    return PEEL_OK;
  }
  // Round 1 binned: a plain listing with room for every key (so round 1 always
  // runs, as in the persistent kernel) and at least two rounds allowed; the
  // persistent kernel then runs rounds 2, 3, ... with one round fewer allowed.
  if (!subtables && !signed_list && out_cap >= desc->ncells && max_rounds >= 2 &&
      list_first_binned_fits(desc) && ws_bytes >= list_ws_bytes(desc)) {
    void *bws = static_cast<char *>(ws) + L.ctrl;
    switch (desc->r) {
      case 2: st = first_round_binned<2>(desc, a.h, cells, out_keys, a.ctrl, bws, s); break;
      case 3: st = first_round_binned<3>(desc, a.h, cells, out_keys, a.ctrl, bws, s); break;
      case 4: st = first_round_binned<4>(desc, a.h, cells, out_keys, a.ctrl, bws, s); break;
      case 5: st = first_round_binned<5>(desc, a.h, cells, out_keys, a.ctrl, bws, s); break;
      case 6: st = first_round_binned<6>(desc, a.h, cells, out_keys, a.ctrl, bws, s); break;
      case 7: st = first_round_binned<7>(desc, a.h, cells, out_keys, a.ctrl, bws, s); break;
      default: st = first_round_binned<8>(desc, a.h, cells, out_keys, a.ctrl, bws, s); break;
    }
    if (st) return st;
    a.first_binned = 1;
    a.stats = round_stats + 1;
    a.max_rounds = max_rounds - 1;
  }
  switch (desc->r) {
    case 2: st = launch_list<2>(a, s, subtables); break;
    case 3: st = launch_list<3>(a, s, subtables); break;
    case 4: st = launch_list<4>(a, s, subtables); break;
    case 5: st = launch_list<5>(a, s, subtables); break;
    case 6: st = launch_list<6>(a, s, subtables); break;
    case 7: st = launch_list<7>(a, s, subtables); break;
    default: st = launch_list<8>(a, s, subtables); break;
  }
  if (st) return st;
  if (signed_list)
    hipLaunchKernelGGL(k_count_nonempty, dim3(grid_for(desc->ncells, kBlock * 8, 4096)),
                       dim3(kBlock), 0, s, cells, desc->ncells, a.ctrl);
  hipLaunchKernelGGL(k_list_finish, dim3(1), dim3(64), 0, s, a.ctrl, desc->r, summary,
                     signed_list ? 1u : 0u, round_stats, a.first_binned);
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

}  // namespace
}  // namespace peel

extern "C" peel_status iblt_list(const iblt_desc *desc, iblt_cell *cells, uint64_t *out_keys,
                                 uint64_t out_cap, uint64_t *round_stats, uint32_t max_rounds,
                                 uint64_t *summary, void *ws, size_t ws_bytes, void *stream) {
  return list_run(desc, cells, out_keys, out_cap, round_stats, max_rounds, summary, ws, ws_bytes,
                  stream, false);
}

extern "C" peel_status iblt_list_signed(const iblt_desc *desc, iblt_cell *cells,
                                        uint64_t *out_keys, int8_t *out_signs, uint64_t out_cap,
                                        uint64_t *round_stats, uint32_t max_rounds,
                                        uint64_t *summary, void *ws, size_t ws_bytes,
                                        void *stream) {
  return list_run(desc, cells, out_keys, out_cap, round_stats, max_rounds, summary, ws, ws_bytes,
                  stream, false, out_signs, true);
}

extern "C" peel_status iblt_list_subtables(const iblt_desc *desc, iblt_cell *cells,
                                           uint64_t *out_keys, uint64_t out_cap,
                                           uint64_t *round_stats, uint32_t max_rounds,
                                           uint64_t *summary, void *ws, size_t ws_bytes,
                                           void *stream) {
  return list_run(desc, cells, out_keys, out_cap, round_stats, max_rounds, summary, ws, ws_bytes,
                  stream, true);
}

extern "C" size_t iblt_list_batched_workspace(uint32_t ntables, uint64_t max_cells) {
  return batched_ws_bytes(ntables, max_cells, batched_grid(ntables, kTeamMax));
}

namespace peel {

// Scratch of iblt_list_batched_noalloc: the batch's control block and the
// per-workgroup candidate lists, in place of a caller workspace.  One copy per
// device, held until the process ends; every call on a device shares it.
// It holds IBLT_NOALLOC_MAX_CELLS-cell lists for kNoAllocGrid workgroups and
// 1 MiB for the team schedule's per-table arrays.
constexpr uint32_t kNoAllocGrid = 512;
constexpr size_t kNoAllocBytes =
    4096 + (size_t)kNoAllocGrid * 2 * IBLT_NOALLOC_MAX_CELLS * sizeof(uint32_t) + (1u << 20);
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// grid_cap: at most this many workgroups (0 = no cap).  Each workgroup lists
// whole tables, so the grid changes the schedule, never the results.
peel_status batched_run(const iblt_batch_entry *entries, uint32_t ntables, uint64_t max_cells,
                        uint32_t max_rounds, const iblt_batch_schedule *sched, void *ws,
                        size_t ws_bytes, void *stream, uint32_t grid_cap = 0) {
  if ((ntables && !entries) || max_rounds == 0 || max_cells >= (1ull << 32) || !ws)
    return PEEL_EINVAL;
  iblt_batch_schedule sc{512u, kLdsCells, 0u, 0u};
  if (sched) sc = *sched;
  if (sc.block_threads == 0) sc.block_threads = 512;
  if (sc.block_threads != 256 && sc.block_threads != 512 && sc.block_threads != 1024)
    return PEEL_EINVAL;
  if (sc.lds_max_cells > kLdsCells || sc.tile_workgroups > kTeamMax) return PEEL_EINVAL;
  const bool teams = sc.tile_workgroups >= 2 && sc.tile_min_cells >= 1;
  const uint32_t tg = teams ? sc.tile_workgroups : 1u;
  uint32_t grid = batched_grid(ntables, tg);
  if (grid_cap && grid > grid_cap) grid = grid_cap;
  const BatchLayout L = batched_layout(ntables, max_cells, grid);
  // the per-table arrays are needed only with teams
  if (ws_bytes < (teams ? L.total : L.ctrl + L.lists)) return PEEL_ENOSPC;
  if (ntables == 0) return PEEL_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = static_cast<char *>(ws);
  BatchCtrl *ctrl = reinterpret_cast<BatchCtrl *>(base);
  uint32_t *lists = reinterpret_cast<uint32_t *>(base + L.ctrl);
  uint32_t *first = teams ? reinterpret_cast<uint32_t *>(base + L.ctrl + L.lists) : nullptr;
  TeamCtrl *tctrl = teams ? reinterpret_cast<TeamCtrl *>(base + L.ctrl + L.lists + L.first) : nullptr;
  // the ticket counter (and the team arrays) start cleared by a kernel, not a
  // memset, so that the call can be captured in a graph
  hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(kInitT), 0, s, ctrl, entries, ntables,
                     sc.tile_min_cells, tg, first, tctrl);
  const uint32_t lm = sc.lds_max_cells;
  const uint64_t limit = barrier_limit_ticks();
#define PEEL_BATCH_LAUNCH(NT, L) \
  hipLaunchKernelGGL((k_list_batched<NT, L>), dim3(grid), dim3(NT), 0, s, entries, ntables, \
                     max_rounds, ctrl, lists, max_cells, lm, first, tctrl, limit)
  switch (sc.block_threads) {
    case 256:
      if (lm) PEEL_BATCH_LAUNCH(256, true); else PEEL_BATCH_LAUNCH(256, false);
      break;
    case 512:
      if (lm) PEEL_BATCH_LAUNCH(512, true); else PEEL_BATCH_LAUNCH(512, false);
      break;
    default:
      if (lm) PEEL_BATCH_LAUNCH(1024, true); else PEEL_BATCH_LAUNCH(1024, false);
      break;
  }
#undef PEEL_BATCH_LAUNCH
  PEEL_HIP_TRY(hipGetLastError());
  return PEEL_OK;
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current (each device holds its own copy at its own
// address; the host-side name is only a stand-in).  Null if the lookup fails.
void *noalloc_scratch() {
  static std::mutex mu;
  static void *addr[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    addr[dev] = p;
  }
  return addr[dev];
}

}  // namespace
}  // namespace peel

extern "C" peel_status iblt_list_batched(const iblt_batch_entry *entries, uint32_t ntables,
                                         uint64_t max_cells, uint32_t max_rounds,
                                         const iblt_batch_schedule *sched, void *ws,
                                         size_t ws_bytes, void *stream) {
  return batched_run(entries, ntables, max_cells, max_rounds, sched, ws, ws_bytes, stream);
}

extern "C" peel_status iblt_list_batched_noalloc(const iblt_batch_entry *entries,
                                                 uint32_t ntables, uint64_t max_cells,
                                                 uint32_t max_rounds,
                                                 const iblt_batch_schedule *sched, void *stream) {
  if (max_cells > IBLT_NOALLOC_MAX_CELLS) return PEEL_ENOSPC;
  void *ws = noalloc_scratch();
  if (!ws) return PEEL_EHIP;
  return batched_run(entries, ntables, max_cells, max_rounds, sched, ws, kNoAllocBytes, stream,
                     kNoAllocGrid);
}

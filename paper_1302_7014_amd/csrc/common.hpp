// Device helpers shared by the libpeel kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "peel.h"

namespace peel {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup for every kernel here

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output finaliser and the
// counter-based draw i of the stream whose state starts at `seed`.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t i) {
  return mix64(seed + (i + 1) * 0x9e3779b97f4a7c15ull);
}

// floor(a * b / 2^64): multiply-shift map of a 64-bit hash onto [0, b).
__device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// ---------------------------------------------------------------------------
// Blocks are dispatched to the GPU's 8 XCDs round robin (block b runs on XCD
// b % 8).  For a grid of `count` blocks, one per item, this maps block b to an
// item so that each XCD takes a contiguous range of items: neighbouring items,
// whose outputs share cache lines, then go through one XCD's L2.  A bijection
// on [0, count) whatever the dispatch order, so only speed depends on it.
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_item(uint32_t b, uint32_t count) {
  const uint32_t x = b % kXcds, i = b / kXcds;
  const uint32_t q = count / kXcds, rem = count % kXcds;
  return x * q + (x < rem ? x : rem) + i;
}

// ---------------------------------------------------------------------------
// Wave / block prefix sums.

__device__ inline uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below this one.
__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// Gives every active lane with `pred` its own slot of a list whose length is
// *counter, with one atomic per wave; the result is meaningful only where pred
// holds.  Every active lane of the wave calls it.
__device__ inline uint32_t wave_append(bool pred, uint32_t *counter) {
  const uint64_t bal = __ballot(pred);
  if (bal == 0) return 0;
  const uint32_t leader = static_cast<uint32_t>(__builtin_ctzll(bal));
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, static_cast<uint32_t>(__popcll(bal)));
  base = __shfl(base, leader, kWave);
  return base + lanes_below(bal);
}

__device__ inline uint32_t wave_inclusive_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t t = __shfl_up(v, d, kWave);
    if (lane >= static_cast<uint32_t>(d)) v += t;
  }
  return v;
}

// Exclusive scan of one value per thread across an NT-thread workgroup.
// `lds` holds NT/kWave + 1 words.  Every thread must call it.
template <int NT = kBlock>
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total, uint32_t *lds) {
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  uint32_t inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) lds[wave] = inc;
  __syncthreads();
  if (threadIdx.x < kWave) {  // the first wave scans the waves' sums
    constexpr uint32_t kW = NT / kWave;
    const uint32_t x = lane < kW ? lds[lane] : 0u;
    const uint32_t y = wave_inclusive_scan(x);
    if (lane < kW) lds[lane] = y - x;
    if (lane == kW - 1) lds[kW] = y;
  }
  __syncthreads();
  uint32_t out = lds[wave] + inc - v;
  *total = lds[NT / kWave];
  __syncthreads();
  return out;
}

template <int NT = kBlock>
__device__ inline uint32_t block_sum(uint32_t v, uint32_t *lds) {
  uint32_t total;
  (void)block_exclusive_scan<NT>(v, &total, lds);
  return total;
}

// Maximum of one value per thread across the workgroup (every thread calls it).
template <int NT = kBlock>
__device__ inline uint32_t block_max(uint32_t v, uint32_t *lds) {
  for (int d = kWave / 2; d > 0; d >>= 1) {
    const uint32_t o = __shfl_xor(v, d, kWave);
    v = o > v ? o : v;
  }
  if (lane_id() == 0) lds[threadIdx.x / kWave] = v;
  __syncthreads();
  uint32_t m = 0;
  for (int w = 0; w < NT / kWave; ++w) m = lds[w] > m ? lds[w] : m;
  __syncthreads();
  return m;
}

// ---------------------------------------------------------------------------
// Device-wide barrier among the `nblocks` members of a team (every member is
// resident).  One thread per workgroup takes part: it makes the workgroup's
// writes visible device-wide (one release fence, which writes back the XCD's
// L2), arrives on `count`, and polls `gen` with relaxed loads (a poll with
// acquire semantics would invalidate the L2 on every iteration and starve the
// workgroups still working), then takes one acquire fence.  The last arriver
// acquires everyone's writes, resets `count` and releases the new `gen`.  A
// wait longer than `limit` wall-clock ticks, or one that sees `abort`, sets
// `abort` and returns false; the caller then leaves the kernel, so every wave
// ends.  `stamp`, when not null, receives the wall clock of each generation.
struct GridSync {
  uint32_t count;
  uint32_t gen;
  uint32_t abort;
  uint32_t pad;
};

__device__ inline bool grid_barrier(GridSync *gs, uint32_t nblocks, uint64_t limit,
                                    uint64_t *stamp = nullptr) {
  __shared__ uint32_t s_ok;
  __syncthreads();  // every wave's stores of this workgroup have completed
  if (threadIdx.x == 0) {
    uint32_t ok = 1;
    if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      ok = 0;
    } else {
      const uint32_t g = __hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const uint32_t arrived =
          __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == nblocks - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (stamp) stamp[g & 255] = wall_clock64();
        __hip_atomic_store(&gs->gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
          if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = 0;
            break;
          }
          if (wall_clock64() - t0 > limit) {
            __hip_atomic_store(&gs->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// ---------------------------------------------------------------------------
// Hierarchical device-wide barrier that also sums one 48-bit value per
// workgroup.  Members are split into up to kBarGroups groups (slot % groups);
// each arrives on its group word (low 16 bits count arrivals, the rest sums the
// values), the last of a group forwards the group's sum to the top word, and
// the last group publishes the total and a new top generation.  A call that
// wants its prefix waits for its group's leader to pass the release down (the
// leader stores the group's base first); any other waits on the top
// generation itself, one hop less.  Every poll is a relaxed load with a short
// sleep.  Timeouts and `abort` behave as in grid_barrier.
//
// Groups.  In the first barrier of a run the groups are slots mod 16, every
// workgroup makes its stores visible device-wide with its own release fence
// (a write-back of its XCD's L2) before arriving, and each counts itself in a
// census of the XCDs.  From the second barrier on, the groups are the XCDs:
// a workgroup only waits until its stores have reached its XCD's L2, and the
// group's last arriver writes that L2 back once for all of them.  Measured
// with 256 workgroups, 32 release fences per XCD, one per workgroup, cost
// 6.5 us; one per XCD 0.8 us.  Every workgroup still takes its own acquire
// fence after the wait.
constexpr int kBarGroups = 16;

// The XCD (accelerator complex die) this wave runs on.
__device__ inline uint32_t xcd_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u;  // HW_REG_XCC_ID, bits 3:0
}

struct alignas(128) BarGroup {
  uint64_t word;
  uint64_t base;  // sum of the values of the groups that reached the top before this one
  uint32_t gen;
  uint32_t pad[27];
};

struct alignas(128) SumBar {
  uint64_t top;
  uint32_t top_gen;
  uint32_t abort;
  uint64_t total[2];
  uint64_t census;      // byte x: the members on XCD x (XCDs 0-7), taken in the first barrier
  uint32_t census_bad;  // a member on an XCD past 7
  uint32_t pad0;
  uint64_t pad[9];
  BarGroup grp[kBarGroups];
};

// Called by a run's init kernel after it zeroes the barrier: with slots set,
// the XCD census is marked unusable, so every barrier keeps the slot groups.
__device__ inline void bar_force_slot_groups(SumBar *sb, bool slots) {
  if (slots) sb->census_bad = 1u;
}

__device__ inline bool bar_wait(const uint32_t *gen, uint32_t e, uint32_t *abort, uint64_t limit) {
  const uint64_t t0 = wall_clock64();
  while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != e) {
    if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (wall_clock64() - t0 > limit) {
      __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Returns false on timeout/abort (the caller leaves the kernel).  `epoch` is the
// workgroup's count of barriers passed (thread 0's copy is the one used).  A
// kernel uses one SumBar for its whole run: the XCD grouping learned in the
// first call is kept in the workgroup's LDS for the later ones.
// `*total` receives the sum of all values; `*prefix` (if given) the sum of the
// values of the workgroups ordered before this one in this barrier (an
// exclusive prefix in arrival order).
__device__ inline bool sum_barrier(SumBar *sb, uint32_t nblocks, uint32_t slot, uint64_t value,
                                   uint32_t *epoch, uint64_t limit, uint64_t *total,
                                   uint64_t *stamp = nullptr, uint64_t *prefix = nullptr) {
  __shared__ uint32_t s_ok;
  __shared__ uint64_t s_total;
  __shared__ uint64_t s_prefix;
  // XCD grouping, set by thread 0 at the end of the first barrier and read
  // only by thread 0 (x_groups 0: the census did not cover the team, keep the
  // slot groups)
  __shared__ uint32_t x_g, x_size, x_groups;
  // every wave waits until its stores are acknowledged, that is, in its XCD's L2
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ok = 1;
    uint64_t tot = 0, pre = 0;
    const bool by_xcd = *epoch >= 1 && x_groups != 0;
    const uint32_t e = ++*epoch;
    uint32_t groups, g, gsize;
    if (by_xcd) {
      groups = x_groups;
      g = x_g;
      gsize = x_size;
    } else {
      groups = nblocks < (uint32_t)kBarGroups ? nblocks : (uint32_t)kBarGroups;
      g = slot % groups;
      gsize = nblocks / groups + (g < nblocks % groups ? 1u : 0u);
    }
    if (e == 1) {
      const uint32_t x = xcd_id();
      if (x < 8)
        __hip_atomic_fetch_add(&sb->census, 1ull << (8 * x), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      else
        __hip_atomic_store(&sb->census_bad, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    BarGroup *gp = &sb->grp[g];
    if (!by_xcd) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint64_t old = __hip_atomic_fetch_add(&gp->word, 1ull | (value << 16), __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if ((old & 0xffffull) + 1 == gsize) {
      const uint64_t gsum = (old >> 16) + value;
      __hip_atomic_store(&gp->word, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // by XCD this is the one write-back of the XCD's L2 for the whole group
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      const uint64_t old2 = __hip_atomic_fetch_add(&sb->top, 1ull | (gsum << 16), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
      pre = (old2 >> 16) + (old >> 16);
      __hip_atomic_store(&gp->base, old2 >> 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((old2 & 0xffffull) + 1 == groups) {
        tot = (old2 >> 16) + gsum;
        __hip_atomic_store(&sb->top, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&sb->total[e & 1], tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (stamp) stamp[e & 255] = wall_clock64();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(&sb->top_gen, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ok = bar_wait(&sb->top_gen, e, &sb->abort, limit);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        tot = __hip_atomic_load(&sb->total[e & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      if (ok) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(&gp->gen, e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
      // no prefix wanted: wait on the top generation itself (one hop)
      ok = bar_wait(prefix ? &gp->gen : &sb->top_gen, e, &sb->abort, limit);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      tot = __hip_atomic_load(&sb->total[e & 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (prefix)
        pre = __hip_atomic_load(&gp->base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + (old >> 16);
    }
    if (e == 1) {
      // every member counted itself before arriving: the census is complete
      const uint64_t c = __hip_atomic_load(&sb->census, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t bad =
          __hip_atomic_load(&sb->census_bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint32_t sum = 0, ng = 0;
      for (int x = 0; x < 8; ++x) {
        const uint32_t n = static_cast<uint32_t>(c >> (8 * x)) & 255u;
        sum += n;
        ng += n ? 1u : 0u;
      }
      const uint32_t x = xcd_id();
      x_g = x;
      x_size = x < 8 ? static_cast<uint32_t>(c >> (8 * x)) & 255u : 0u;
      x_groups = (ok && !bad && sum == nblocks) ? ng : 0u;
    }
    s_ok = ok;
    s_total = tot;
    s_prefix = pre;
  }
  __syncthreads();
  *total = s_total;
  if (prefix) *prefix = s_prefix;
  return s_ok != 0;
}

// ---------------------------------------------------------------------------
// Team of resident workgroups for a persistent kernel.  A device-wide barrier
// is only safe among workgroups that are running at the same time, and the
// number the hardware keeps resident is not reliably the occupancy estimate.
// So the team is formed at run time: every workgroup adds one to `join`; the
// first (slot 0) waits until all gridDim.x workgroups have joined, or until no
// new one has joined for `quiet` ticks, then sets the CLOSED bit and publishes
// the count as `size`.  Workgroups that joined before the close are members
// (they are running, hence resident); later ones see CLOSED and leave at once.
// Members use their slot and the team size in place of blockIdx.x/gridDim.x.
struct Team {
  uint32_t join;
  uint32_t size;
};

constexpr uint32_t kTeamClosed = 0x80000000u;

// True for a member; `slot` and `size` then hold its index and the team size.
__device__ inline bool team_join(Team *tm, uint64_t quiet, uint64_t limit, uint32_t *slot,
                                 uint32_t *size) {
  __shared__ uint32_t s_slot, s_size;
  if (threadIdx.x == 0) {
    uint32_t sl = 0xffffffffu, sz = 0;
    const uint32_t old =
        __hip_atomic_fetch_add(&tm->join, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!(old & kTeamClosed)) {
      sl = old;
      if (old == 0) {
        const uint64_t t0 = wall_clock64();
        uint64_t last = t0;
        uint32_t seen = 1;
        for (;;) {
          const uint32_t c =
              __hip_atomic_load(&tm->join, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
              ~kTeamClosed;
          if (c >= gridDim.x) break;
          const uint64_t now = wall_clock64();
          if (c != seen) {
            seen = c;
            last = now;
          } else if (now - last > quiet) {
            break;
          }
          if (now - t0 > limit) break;
          __builtin_amdgcn_s_sleep(1);
        }
        sz = __hip_atomic_fetch_or(&tm->join, kTeamClosed, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT) &
             ~kTeamClosed;
        __hip_atomic_store(&tm->size, sz, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const uint64_t t0 = wall_clock64();
        while ((sz = __hip_atomic_load(&tm->size, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ==
               0) {
          if (wall_clock64() - t0 > limit) break;
          __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    s_slot = sl;
    s_size = sz;
  }
  __syncthreads();
  *slot = s_slot;
  *size = s_size;
  return s_size != 0 && s_slot < s_size;
}

// ---------------------------------------------------------------------------
// Small device utilities.

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T *p, uint64_t n, T v) {
  for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * kBlock)
    p[i] = v;
}

__device__ inline uint32_t atomic_load_u32(const uint32_t *p) {
  return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t atomic_load_u64(const uint64_t *p) {
  return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace peel

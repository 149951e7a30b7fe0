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
// Wave / block prefix sums.

__device__ inline uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below this one.
__device__ inline uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
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

// Exclusive scan of one value per thread across a kBlock-thread workgroup.
// `lds` holds kBlock/kWave + 1 words.  Every thread must call it.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *total, uint32_t *lds) {
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  uint32_t inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) lds[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      uint32_t t = lds[w];
      lds[w] = acc;
      acc += t;
    }
    lds[kBlock / kWave] = acc;
  }
  __syncthreads();
  uint32_t out = lds[wave] + inc - v;
  *total = lds[kBlock / kWave];
  __syncthreads();
  return out;
}

__device__ inline uint32_t block_sum(uint32_t v, uint32_t *lds) {
  uint32_t total;
  (void)block_exclusive_scan(v, &total, lds);
  return total;
}

// ---------------------------------------------------------------------------
// Device-wide barrier for persistent kernels launched cooperatively (every
// workgroup resident).  Workgroups arrive on `count`; the last one resets it
// and advances `gen`; the others wait for `gen` to move.  A wait that passes
// `limit` wall-clock ticks, or that sees `abort` set, sets `abort` and
// returns false: the caller then leaves the kernel, so every wave ends.
struct GridSync {
  uint32_t count;
  uint32_t gen;
  uint32_t abort;
  uint32_t pad;
};

__device__ inline bool grid_barrier(GridSync *gs, uint32_t nblocks, uint64_t limit) {
  __shared__ uint32_t s_ok;
  __threadfence();  // publish this thread's writes device-wide
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ok = 1;
    if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      ok = 0;
    } else {
      const uint32_t g = __hip_atomic_load(&gs->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t arrived =
          __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == nblocks - 1) {
        __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&gs->gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&gs->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
          if (__hip_atomic_load(&gs->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            ok = 0;
            break;
          }
          if (wall_clock64() - t0 > limit) {
            __hip_atomic_store(&gs->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  __threadfence();  // see every other workgroup's writes from before the barrier
  return s_ok != 0;
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

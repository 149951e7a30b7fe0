// Host-side helpers for libpeel entry points.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "peel.h"

namespace peel {

#define PEEL_HIP_TRY(expr)                          \
  do {                                              \
    hipError_t _e = (expr);                         \
    if (_e != hipSuccess) return PEEL_EHIP;         \
  } while (0)

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Carves consecutive 256-byte aligned pieces out of a caller workspace.
struct Carver {
  char *base;
  size_t used = 0;
  explicit Carver(void *p) : base(static_cast<char *>(p)) {}
  template <typename T>
  T *take(size_t count) {
    T *p = reinterpret_cast<T *>(base + used);
    used = align_up(used + count * sizeof(T));
    return p;
  }
};

struct DeviceInfo {
  int id = -1;
  int cus = 0;
  int blocks_per_cu_cap = 0;         // PEEL_BLOCKS_PER_CU, 0 = occupancy only
  uint64_t wall_khz = 0;             // device wall clock rate
  uint64_t team_limit_ticks = 0;     // longest wait while a persistent team forms (10 s)
  uint64_t team_quiet_ticks = 0;     // PEEL_TEAM_QUIET_US of device wall clock (5 us)
  bool debug = false;                // PEEL_DEBUG: launch shapes on stderr
};

inline long env_long(const char *name, long dflt) {
  const char *v = std::getenv(name);
  if (!v || !*v) return dflt;
  char *end = nullptr;
  long x = std::strtol(v, &end, 10);
  return (end && *end == 0) ? x : dflt;
}

// Properties of the current device (cached per device id).
inline const DeviceInfo &device_info() {
  static DeviceInfo cache[64];
  static std::mutex mu;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  DeviceInfo &d = cache[dev & 63];
  if (d.id != dev) {
    int cus = 0, khz = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (khz <= 0) khz = 100000;  // 100 MHz
    d.cus = cus > 0 ? cus : 1;
    d.wall_khz = (uint64_t)khz;
    d.team_limit_ticks = (uint64_t)khz * 10000ull;
    long us = env_long("PEEL_TEAM_QUIET_US", 5);
    if (us < 1) us = 1;
    d.team_quiet_ticks = (uint64_t)khz * (uint64_t)us / 1000ull + 1;
    long cap = env_long("PEEL_BLOCKS_PER_CU", 0);
    d.blocks_per_cu_cap = cap > 0 ? (int)cap : 0;
    d.debug = env_long("PEEL_DEBUG", 0) != 0;
    d.id = dev;
  }
  return d;
}

// PEEL_BARRIER=slots (read at each call): every device-wide barrier of the
// call keeps the slot groups of its first barrier, the path a team takes when
// the XCD census does not cover it (tests).
inline bool barrier_slots() {
  const char *b = std::getenv("PEEL_BARRIER");
  return b && std::strcmp(b, "slots") == 0;
}

// Device wall-clock ticks a device-wide barrier waits before the call gives
// up and reports PEEL_FLAG_TIMEOUT: PEEL_BARRIER_TIMEOUT_MS (default 10000),
// read at every call.  0 makes a barrier give up at its first poll that finds
// it still closed; every workgroup then leaves its kernel at its next barrier,
// which is how the tests reach the give-up path with every kernel ending.
inline uint64_t barrier_limit_ticks() {
  const long ms = env_long("PEEL_BARRIER_TIMEOUT_MS", 10000);
  return device_info().wall_khz * (uint64_t)(ms < 0 ? 0 : ms);
}

// Workgroups of `kernel` (kBlock threads) that fit on the device at once.
inline int coresident_blocks(const void *kernel, int block, size_t lds_bytes) {
  const DeviceInfo &d = device_info();
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds_bytes) != hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  const int occ = per_cu;
  if (d.blocks_per_cu_cap > 0 && per_cu > d.blocks_per_cu_cap) per_cu = d.blocks_per_cu_cap;
  if (d.debug)
    std::fprintf(stderr, "[peel] occupancy %d blocks/CU, using %d x %d CUs\n", occ, per_cu, d.cus);
  return per_cu * d.cus;
}

inline unsigned grid_for(uint64_t items, int per_block, unsigned cap = 1u << 20) {
  uint64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return static_cast<unsigned>(g);
}

}  // namespace peel

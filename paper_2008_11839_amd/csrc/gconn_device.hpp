// gconn_device.hpp -- device helpers shared by the gconn kernels: wave64
// primitives (all lanes of a wave must be active where noted), SplitMix64,
// plain root lookup, and the finish-phase work lists.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <utility>
#include <vector>

#include "gconn_internal.hpp"
#include "gconn_rules.hpp"

namespace gconn {

// --------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

// Wave-uniform iteration: returns the first item handled by this wave.
__device__ __forceinline__ uint64_t wave_base() {
  return ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~63ull;
}
__device__ __forceinline__ uint64_t gtid() {
  return (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
}
__device__ __forceinline__ uint64_t wave_stride() { return (uint64_t)gridDim.x * blockDim.x; }
__device__ __forceinline__ uint64_t wave_index() { return gtid() >> 6; }
__device__ __forceinline__ uint64_t wave_count() { return ((uint64_t)gridDim.x * blockDim.x) >> 6; }

// All 64 lanes must be active for the wave-wide helpers below.
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
  return x;
}
__device__ __forceinline__ unsigned long long wave_max(unsigned long long x) {
  for (int d = 32; d >= 1; d >>= 1) {
    unsigned long long y = __shfl_xor(x, d);
    x = y > x ? y : x;
  }
  return x;
}
// Exclusive prefix sum of cnt over the wave; *total receives the wave sum.
__device__ __forceinline__ uint32_t wave_exclusive(uint32_t cnt, uint32_t* total) {
  uint32_t x = cnt;
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d);
    if (lane() >= (uint32_t)d) x += y;
  }
  *total = __shfl(x, 63);
  return x - cnt;
}
// Reserve cnt slots per lane in a global list; returns this lane's first slot.
__device__ __forceinline__ uint32_t wave_reserve(uint32_t* counter, uint32_t cnt) {
  uint32_t total;
  uint32_t off = wave_exclusive(cnt, &total);
  uint32_t base = 0;
  if (total && lane() == 0) base = atomicAdd(counter, total);
  base = __shfl(base, 0);
  return base + off;
}
// One slot per lane with pred set; one atomic per wave (lanes may be inactive).
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool pred, bool* any) {
  const unsigned long long mask = __ballot(pred);
  *any = mask != 0;
  if (!mask) return 0;
  const uint32_t leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane() == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
  base = __shfl(base, leader);
  return base + (uint32_t)__popcll(mask & ((1ull << lane()) - 1));
}

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t state0, uint64_t i) {
  uint64_t z = state0 + (i + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Root by pointer jumping with plain loads: used only after a kernel boundary,
// with no concurrent links, where every value read is an ancestor.
__device__ __forceinline__ uint32_t root_plain(const uint32_t* P, uint32_t x) {
  uint32_t p = P[x];
  while (p != x) {
    x = p;
    p = P[x];
  }
  return x;
}

// --------------------------------------------------------------- work lists
struct WorkLists {
  uint32_t* small;   // [kSubLists][cap]
  uint32_t* medium;  // [kSubLists][cap]
  uint2* segs;       // (vertex, segment index)
  uint32_t cap;
};

// Append vertex v (degree deg) to its work class.  `group` is the index of the
// 64-item group this wave iteration covers (uniform over the wave); it picks
// the sub-list, so one sub-list receives at most `cap` entries.  All 64 lanes
// must be active.
__device__ __forceinline__ void wl_push(const WorkLists& wl, Ctrl* c, uint64_t group, uint32_t v,
                                        uint64_t deg, bool active) {
  const uint32_t r = (uint32_t)(group % kSubLists);
  const bool sm = active && deg <= kSmallDeg;
  const bool md = active && deg > kSmallDeg && deg <= kMedDeg;
  const bool lg = active && deg > kMedDeg;
  bool any;
  uint32_t slot = wave_append(&c->small_cnt[r * kCntPad], sm, &any);
  if (sm) wl.small[(size_t)r * wl.cap + slot] = v;
  slot = wave_append(&c->medium_cnt[r * kCntPad], md, &any);
  if (md) wl.medium[(size_t)r * wl.cap + slot] = v;
  if (__ballot(lg)) {
    const uint32_t nseg = lg ? (uint32_t)((deg + kSeg - 1) / kSeg) : 0u;
    const uint32_t first = wave_reserve(&c->seg_count, nseg);
    for (uint32_t t = 0; t < nseg; ++t) wl.segs[first + t] = make_uint2(v, t);
  }
}

// Exclusive prefix of the kSubLists counters into LDS (pre[kSubLists] = total).
// Called by every thread of the block; the first wave computes it.
__device__ __forceinline__ void wl_prefix(const uint32_t* cnt, uint32_t* pre) {
  if (threadIdx.x < 64) {
    uint32_t total;
    const uint32_t x = cnt[lane() * kCntPad];
    pre[lane()] = wave_exclusive(x, &total);
    if (lane() == 0) pre[kSubLists] = total;
  }
}
// Entry i (< pre[kSubLists]) of the concatenated sub-lists.
__device__ __forceinline__ uint32_t wl_get(const uint32_t* list, uint32_t cap, const uint32_t* pre,
                                           uint32_t i) {
  uint32_t lo = 0, hi = kSubLists;  // invariant pre[lo] <= i < pre[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (pre[mid] <= i) lo = mid;
    else hi = mid;
  }
  return list[(size_t)lo * cap + (i - pre[lo])];
}

// --------------------------------------------------------------- launches
// Resident workgroups for a persistent launch of `kernel` (all CUs x what the
// occupancy calculator allows), cached per kernel and block size.
template <class K>
inline uint32_t persistent_grid(K kernel, uint32_t block) {
  static std::mutex mu;
  static std::vector<std::pair<std::pair<const void*, uint32_t>, uint32_t>> cache;
  const void* key = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lock(mu);
  for (auto& e : cache)
    if (e.first.first == key && e.first.second == block) return e.second;
  int dev = 0, cus = 256, per_cu = 8;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    cus = 256;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, (int)block, 0) != hipSuccess ||
      per_cu < 1) {
    (void)hipGetLastError();
    per_cu = 1;
  }
  const uint32_t g = (uint32_t)cus * (uint32_t)per_cu;
  cache.push_back({{key, block}, g});
  return g;
}

}  // namespace gconn

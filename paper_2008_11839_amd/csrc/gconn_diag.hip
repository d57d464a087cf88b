// gconn_diag.hip -- random-access ceilings of the chip, the yardstick of the
// union-find kernels.  The union passes read and CAS 4-byte parent words at
// data-dependent addresses, so their speed is set by how many such accesses
// the memory system serves per second, not by streaming bandwidth.  These
// kernels issue exactly that traffic on a caller's table: independent random
// 4-byte loads (cached, or device-coherent), or random 4-byte CAS, with
// several accesses in flight per lane, and nothing else.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>

#include "gconn_internal.hpp"

namespace gconn {
namespace {

constexpr int kInFlight = 8;  // independent accesses per lane per step

// Counter-based 64-bit mix (SplitMix64 finaliser) of a lane's step index.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// kind 0: cached loads, 1: device-coherent loads, 2: CAS (the word's own
// value to itself, so the table is unchanged and every CAS succeeds).
template <int Kind>
__global__ void __launch_bounds__(256) k_random_access(uint32_t* T, uint64_t mask, uint64_t steps,
                                                       uint64_t seed, uint32_t* sink) {
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (uint64_t s = 0; s < steps; ++s) {
    uint32_t idx[kInFlight];
#pragma unroll
    for (int j = 0; j < kInFlight; ++j)
      idx[j] = (uint32_t)(mix64(seed + (tid * steps + s) * kInFlight + j) & mask);
    uint32_t val[kInFlight];
#pragma unroll
    for (int j = 0; j < kInFlight; ++j) {
      if constexpr (Kind == 0) {
        val[j] = __hip_atomic_load(&T[idx[j]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      } else if constexpr (Kind == 1) {
        val[j] = __hip_atomic_load(&T[idx[j]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        uint32_t e = idx[j];  // T[i] == i
        __hip_atomic_compare_exchange_strong(&T[idx[j]], &e, idx[j], __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        val[j] = e;
      }
    }
#pragma unroll
    for (int j = 0; j < kInFlight; ++j) acc ^= val[j];
  }
  sink[tid] = acc;
}

}  // namespace
}  // namespace gconn

using namespace gconn;


extern "C" gconn_status gconn_diag_random_access(uint32_t* table, uint64_t words, int kind,
                                                 uint64_t accesses, uint32_t* sink,
                                                 uint32_t sink_words, void* stream) {
  clear_error();
  if (!table || !sink) return fail(GCONN_EINVAL, "table or sink is NULL");
  if (words == 0 || (words & (words - 1)) != 0)
    return fail(GCONN_EINVAL, "words must be a power of two");
  if (kind < 0 || kind > 2) return fail(GCONN_EINVAL, "kind must be 0, 1 or 2");
  const uint32_t block = 256;
  const uint64_t lanes = sink_words / block * block;
  if (lanes == 0) return fail(GCONN_EINVAL, "sink must hold at least 256 words");
  const uint64_t steps = accesses / (lanes * kInFlight);
  if (steps == 0) return fail(GCONN_EINVAL, "accesses must be at least 8 per sink word");
  GCONN_TRY(check_device_ptr(table, "table"));
  GCONN_TRY(check_device_ptr(sink, "sink"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t grid = (uint32_t)(lanes / block);
  const uint64_t seed = 0x5eedull;
  switch (kind) {
    case 0: k_random_access<0><<<grid, block, 0, s>>>(table, words - 1, steps, seed, sink); break;
    case 1: k_random_access<1><<<grid, block, 0, s>>>(table, words - 1, steps, seed, sink); break;
    default: k_random_access<2><<<grid, block, 0, s>>>(table, words - 1, steps, seed, sink); break;
  }
  GCONN_LAUNCHED("k_random_access");
  return GCONN_OK;
}

// persist.h -- helpers of the persistent (lane-refill) kernels (library-internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kparams.h"

namespace dqj {
namespace persist {

__device__ __forceinline__ int rank_in(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// A wave-uniform float, kept in a scalar register.
__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

// The frame table is never written while a launch runs: reading it through the
// constant address space lets uniform reads become scalar loads. (The host pass of the
// compiler only needs the type to exist.)
#if defined(__HIP_DEVICE_COMPILE__)
typedef const __attribute__((address_space(4))) FrameDesc *ConstFrame;
typedef const __attribute__((address_space(4))) LaunchHeader *ConstHeader;
#else
typedef const FrameDesc *ConstFrame;
typedef const LaunchHeader *ConstHeader;
#endif

template <bool BATCH>
struct FramePtr {
  typedef const FrameDesc *type;
};
template <>
struct FramePtr<true> {
  typedef ConstFrame type;
};

// Frame of a global tile index (frames are in tile order).
__device__ __forceinline__ int find_frame(ConstFrame table, int nframes, uint32_t tile) {
  int lo = 0, hi = nframes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].tile_begin <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

}  // namespace persist
}  // namespace dqj

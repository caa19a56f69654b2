// kc_device.h -- device helpers shared by the gfx950 kernel sources: wave
// reductions and the range search over an LDS copy of the range fences.
#pragma once

#include "kc_internal.h"

namespace kc {

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

// Adds a wave's closure-scan counts into its slot (lane 0 only).
__device__ __forceinline__ void add_scan_counts(unsigned long long* counts, uint32_t slot, uint32_t n_ptr,
                                                uint32_t n_in) {
  unsigned long long* c = counts + (size_t)(slot % kScanSlots) * kScanSlotStride;
  if (n_ptr) atomicAdd(c, (unsigned long long)n_ptr);
  if (n_in) atomicAdd(c + 1, (unsigned long long)n_in);
}

// ---------------------------------------------------------- range search --
struct FenceLds {
  uint64_t base[kFences];
  uint64_t end[kFences];
  uint16_t bucket[kBuckets];
};

__device__ __forceinline__ void load_fences(FenceLds& f, const RangeTable& rt, uint32_t tid,
                                            uint32_t nthreads) {
  for (uint32_t i = tid; i < rt.n_fence; i += nthreads) {
    const uint32_t r = i * rt.stride;
    f.base[i] = rt.base[r];
    f.end[i] = rt.end[r];
  }
  if (rt.n != 0u)
    for (uint32_t i = tid; i < kBuckets; i += nthreads) f.bucket[i] = rt.bucket[i];
}

// Last fence whose base is at or below w, for lo <= w < lo + span: start at the
// bucket's entry and search only up to the next bucket's (usually no step).
__device__ __forceinline__ uint32_t fence_of(uint64_t w, const FenceLds& f, const RangeTable& rt) {
  const uint32_t b = (uint32_t)((w - rt.lo) >> rt.shift);
  uint32_t i = f.bucket[b];
  uint32_t j = b + 1u < kBuckets ? f.bucket[b + 1u] : rt.n_fence - 1u;
  while (i < j) {
    const uint32_t m = (i + j + 1u) >> 1;
    if (f.base[m] <= w) i = m; else j = m - 1u;
  }
  return i;
}

// Index of the range holding w, or -1.
__device__ __forceinline__ int32_t range_index(uint64_t w, const FenceLds& f, const RangeTable& rt) {
  if (rt.n == 0u || w - rt.lo >= rt.span) return -1;  // below the lowest base wraps to a large offset
  const uint32_t i = fence_of(w, f, rt);
  if (rt.stride == 1u) return w < f.end[i] ? (int32_t)i : -1;
  uint32_t a = i * rt.stride;
  uint32_t b = min(a + rt.stride, rt.n);
  while (b - a > 1u) {
    const uint32_t m = (a + b) >> 1;
    if (ld8g(rt.base + m) <= w) a = m; else b = m;
  }
  // typed global: merged with the LDS read above, the two would become one
  // flat load, whose wait also waits for every global load in flight
  return w < ld8g(rt.end + a) ? (int32_t)a : -1;
}

// True iff w lies in [base_r, end_r) for some range r.
__device__ __forceinline__ bool in_ranges(uint64_t w, const FenceLds& f, const RangeTable& rt) {
  return range_index(w, f, rt) >= 0;
}

}  // namespace kc

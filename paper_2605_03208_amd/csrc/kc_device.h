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

// ---------------------------------------------------------- range search --
struct FenceLds {
  uint64_t base[kFences];
  uint64_t end[kFences];
};

__device__ __forceinline__ void load_fences(FenceLds& f, const RangeTable& rt, uint32_t tid,
                                            uint32_t nthreads) {
  for (uint32_t i = tid; i < rt.n_fence; i += nthreads) {
    const uint32_t r = i * rt.stride;
    f.base[i] = rt.base[r];
    f.end[i] = rt.end[r];
  }
}

// True iff w lies in [base_r, end_r) for some range r.
__device__ __forceinline__ bool in_ranges(uint64_t w, const FenceLds& f, const RangeTable& rt) {
  if (rt.n == 0u || w < f.base[0]) return false;
  uint32_t i = 0;
#pragma unroll
  for (uint32_t step = kFences / 2; step > 0; step >>= 1)
    if (i + step < rt.n_fence && f.base[i + step] <= w) i += step;
  if (rt.stride == 1u) return w < f.end[i];
  uint32_t a = i * rt.stride;
  uint32_t b = min(a + rt.stride, rt.n);
  while (b - a > 1u) {
    const uint32_t m = (a + b) >> 1;
    if (rt.base[m] <= w) a = m; else b = m;
  }
  return w < rt.end[a];
}

// Index of the range holding w, or -1.
__device__ __forceinline__ int32_t range_index(uint64_t w, const FenceLds& f, const RangeTable& rt) {
  if (rt.n == 0u || w < f.base[0]) return -1;
  uint32_t i = 0;
#pragma unroll
  for (uint32_t step = kFences / 2; step > 0; step >>= 1)
    if (i + step < rt.n_fence && f.base[i + step] <= w) i += step;
  if (rt.stride == 1u) return w < f.end[i] ? (int32_t)i : -1;
  uint32_t a = i * rt.stride;
  uint32_t b = min(a + rt.stride, rt.n);
  while (b - a > 1u) {
    const uint32_t m = (a + b) >> 1;
    if (rt.base[m] <= w) a = m; else b = m;
  }
  return w < rt.end[a] ? (int32_t)a : -1;
}

}  // namespace kc

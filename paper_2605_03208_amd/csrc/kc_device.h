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

// The search over fences held in LDS (base, end and bucket arrays of a fence
// table with the given stride): index of the range holding w, or -1.  The
// last fence whose base is at or below w starts at the bucket's entry and is
// searched only up to the next bucket's (usually no step); with a stride above
// one, the ranges of that fence are searched in global memory.
__device__ __forceinline__ int32_t search_fences(uint64_t w, const uint64_t* fbase, const uint64_t* fend,
                                                 const uint16_t* fbucket, uint32_t stride, uint32_t n_fence,
                                                 const RangeTable& rt) {
  if (rt.n == 0u || w - rt.lo >= rt.span) return -1;  // below the lowest base wraps to a large offset
  const uint32_t bk = (uint32_t)((w - rt.lo) >> rt.shift);
  uint32_t i = fbucket[bk];
  uint32_t j = bk + 1u < kBuckets ? fbucket[bk + 1u] : n_fence - 1u;
  while (i < j) {
    const uint32_t m = (i + j + 1u) >> 1;
    if (fbase[m] <= w) i = m; else j = m - 1u;
  }
  if (stride == 1u) return w < fend[i] ? (int32_t)i : -1;
  uint32_t a = i * stride;
  uint32_t b = min(a + stride, rt.n);
  while (b - a > 1u) {
    const uint32_t m = (a + b) >> 1;
    if (ld8g(rt.base + m) <= w) a = m; else b = m;
  }
  // typed global: merged with the LDS read above, the two would become one
  // flat load, whose wait also waits for every global load in flight
  return w < ld8g(rt.end + a) ? (int32_t)a : -1;
}

// The same search for a value that is the same in every lane of the wave,
// straight from the range set's arrays through the scalar cache (they are a
// few KiB and read-only while a kernel runs), for kernels that search once
// per wave and would rather not load a fence table into LDS: the bucket index
// gives the fences (every stride-th range) to search, then the ranges of that
// fence are searched.  Returns the range index (or -1) and its base and end.
#define KC_CONST __attribute__((address_space(4)))
struct RangeHit {
  int32_t a;
  uint64_t base, end;
};
__device__ __forceinline__ RangeHit range_find_uniform(uint64_t w, const RangeTable& rt) {
  RangeHit h{-1, 0, 0};
  if (rt.n == 0u || w - rt.lo >= rt.span) return h;
  const KC_CONST uint64_t* base = (const KC_CONST uint64_t*)rt.base;
  const KC_CONST uint64_t* end = (const KC_CONST uint64_t*)rt.end;
  const KC_CONST uint32_t* bucket2 = (const KC_CONST uint32_t*)rt.bucket;  // two 16-bit entries a word
  const auto bucket = [&](uint32_t k) -> uint32_t {
    const uint32_t v = bucket2[k >> 1];
    return (k & 1u) ? (v >> 16) : (v & 0xFFFFu);
  };
  const uint32_t bk = __builtin_amdgcn_readfirstlane((uint32_t)((w - rt.lo) >> rt.shift));
  uint32_t i = bucket(bk);
  uint32_t j = bk + 1u < kBuckets ? bucket(bk + 1u) : rt.n_fence - 1u;
  while (i < j) {
    const uint32_t m = (i + j + 1u) >> 1;
    if (base[(uint64_t)m * rt.stride] <= w) i = m; else j = m - 1u;
  }
  uint32_t lo = i * rt.stride;
  uint32_t hi = min(lo + rt.stride, rt.n);
  while (hi - lo > 1u) {
    const uint32_t m = (lo + hi) >> 1;
    if (base[m] <= w) lo = m; else hi = m;
  }
  h.base = base[lo];
  h.end = end[lo];
  if (w < h.end) h.a = (int32_t)lo;
  return h;
}

// Index of the range holding w, or -1 (table of up to kFences fences).
__device__ __forceinline__ int32_t range_index(uint64_t w, const FenceLds& f, const RangeTable& rt) {
  return search_fences(w, f.base, f.end, f.bucket, rt.stride, rt.n_fence, rt);
}

// True iff w lies in [base_r, end_r) for some range r.
__device__ __forceinline__ bool in_ranges(uint64_t w, const FenceLds& f, const RangeTable& rt) {
  return range_index(w, f, rt) >= 0;
}

// ------------------------------------------------------------ wide table --
// Kernels whose workgroups hold several independent waves share one copy of
// up to kWideFences fences in dynamic LDS: n_fence_w bases, n_fence_w ends,
// then the kBuckets-entry bucket index.
extern __shared__ __attribute__((aligned(16))) uint64_t kc_wide_lds[];
constexpr uint32_t kWideWaves = 8;  // most waves per workgroup of the kernels that use it

// Workgroups for a grid of `waves` waves: up to kWideWaves waves each, but
// about one workgroup per CU when the grid is small (spread over the CUs
// rather than packed onto a few).
inline void wide_shape(uint32_t waves, uint32_t n_cu, uint32_t* blocks, uint32_t* waves_per_block,
                       uint32_t max_waves = kWideWaves) {
  waves = waves < 1u ? 1u : waves;
  uint32_t b = (waves + max_waves - 1) / max_waves;
  if (b < n_cu) b = waves < n_cu ? waves : n_cu;
  *waves_per_block = (waves + b - 1) / b;
  *blocks = (waves + *waves_per_block - 1) / *waves_per_block;
}

inline size_t wide_lds_bytes(const RangeTable& rt) { return 16u * (size_t)rt.n_fence_w + 2u * kBuckets; }

__device__ __forceinline__ void load_wide_fences(const RangeTable& rt, uint32_t tid, uint32_t nthreads) {
  const uint32_t nf = rt.n_fence_w;
  for (uint32_t i = tid; i < nf; i += nthreads) {
    const uint32_t r = i * rt.stride_w;
    kc_wide_lds[i] = rt.base[r];
    kc_wide_lds[nf + i] = rt.end[r];
  }
  if (rt.n != 0u) {
    uint16_t* bucket = reinterpret_cast<uint16_t*>(kc_wide_lds + 2u * nf);
    for (uint32_t i = tid; i < kBuckets; i += nthreads) bucket[i] = rt.bucket_w[i];
  }
}

// Orders a wave's own LDS accesses across lanes: the LDS executes one wave's
// operations in program order, so only the compiler must not move them.
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ int32_t wide_range_index(uint64_t w, const RangeTable& rt) {
  const uint32_t nf = rt.n_fence_w;
  return search_fences(w, kc_wide_lds, kc_wide_lds + nf, reinterpret_cast<const uint16_t*>(kc_wide_lds + 2u * nf),
                       rt.stride_w, nf, rt);
}

}  // namespace kc

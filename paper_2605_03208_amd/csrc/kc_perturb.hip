// kc_perturb.hip -- candidate materialisation for the validation server: a
// golden copy moved by a seeded perturbation, so that a request of (golden id,
// tolerance, seed) stands for a reproducer's output buffer (Sec. 4.5.2, and
// reproducers feeding tuning agents, Sec. 1 and Sec. 6).
//
// In buffer b of a typed arena (element offset o_b, length n_b, seed s_b) and
// block size B, block j < floor(n_b / B) moves element o_b + j*B + (h1 mod B)
// by 1 + (h2 mod kmax) steps, towards -inf when bit 20 of h2 is set, where
//   h1 = mix32(s_b * 0x9E37 + j * 0x85EB + 1),  h2 = mix32(h1 + s_b + 0x27D4EB2F)
// and mix32 is two rounds of x = ((x >> 16) ^ x) * 0x45D9F3B mod 2^32 and a
// final xor-shift.  A float steps in the sign-magnitude order of its bits
// (+0 and -0 both rank 0), clamped at +-inf (the largest finite code where the
// format has no inf); NaN codes stay.  An integer moves by the step, clamped
// to its range.  One thread per moved element; the moved elements of one call
// are distinct (one per block, blocks disjoint), so there is no write race.
#include <algorithm>

#include "kc_internal.h"

namespace kc {
namespace {

constexpr uint32_t kPerturbBufs = 96;  // buffers per launch (kernel arguments stay below 4 KiB)
constexpr uint32_t kPerturbThreads = 256;

struct PerturbArgs {
  uint64_t off[kPerturbBufs];   // element offset of each buffer
  uint64_t end[kPerturbBufs];   // inclusive prefix of moved elements (blocks) per buffer
  uint32_t seed[kPerturbBufs];  // already reduced to 31 bits
  uint64_t total;               // moved elements in this launch
  uint64_t block;
  uint32_t n, kmax;
  uint32_t width;               // element bytes: 1, 2, 4, 8
  uint32_t is_int;              // two's complement integer
  uint64_t limit;               // float: code of +inf (or the largest finite); int: unused
  uint32_t nan_is_neg_zero;     // fnuz formats: the code 0x80 is the NaN, and there is no -0
};

__device__ __forceinline__ uint64_t mix32(uint64_t x) {
  constexpr uint64_t m = 0xFFFFFFFFull;
  x &= m;
  x = (((x >> 16) ^ x) * 0x45D9F3Bull) & m;
  x = (((x >> 16) ^ x) * 0x45D9F3Bull) & m;
  return ((x >> 16) ^ x) & m;
}

__device__ __forceinline__ uint64_t load_elem(uint64_t addr, uint32_t width) {
  switch (width) {
    case 1: return *(const KC_GLOBAL uint8_t*)addr;
    case 2: return *(const KC_GLOBAL uint16_t*)addr;
    case 4: return *(const KC_GLOBAL uint32_t*)addr;
    default: return *(const KC_GLOBAL uint64_t*)addr;
  }
}

__device__ __forceinline__ void store_elem(uint64_t addr, uint32_t width, uint64_t v) {
  switch (width) {
    case 1: *(KC_GLOBAL uint8_t*)addr = (uint8_t)v; break;
    case 2: *(KC_GLOBAL uint16_t*)addr = (uint16_t)v; break;
    case 4: *(KC_GLOBAL uint32_t*)addr = (uint32_t)v; break;
    default: *(KC_GLOBAL uint64_t*)addr = v; break;
  }
}

// The bits of an element moved by k steps.
__device__ __forceinline__ uint64_t step_bits(uint64_t b, int64_t k, const PerturbArgs& a) {
  const uint32_t nbits = 8u * a.width;
  const uint64_t sign = 1ull << (nbits - 1u);
  if (a.is_int) {
    const int64_t lo = nbits == 64u ? INT64_MIN : -(int64_t)sign;
    const int64_t hi = nbits == 64u ? INT64_MAX : (int64_t)sign - 1;
    const int64_t v = nbits == 64u ? (int64_t)b : (int64_t)(b ^ sign) - (int64_t)sign;  // sign-extend
    int64_t o;
    if (__builtin_add_overflow(v, k, &o)) o = k > 0 ? hi : lo;
    o = o < lo ? lo : (o > hi ? hi : o);
    return (uint64_t)o & (nbits == 64u ? ~0ull : (sign << 1) - 1ull);
  }
  const uint64_t mag = b & (sign - 1ull);
  const bool nan = a.nan_is_neg_zero ? (b == sign) : (mag > a.limit);
  if (nan) return b;
  const int64_t lim = (int64_t)a.limit;
  int64_t o = ((b & sign) ? -(int64_t)mag : (int64_t)mag) + k;  // |mag| < 2^63, |k| small: no overflow
  o = o < -lim ? -lim : (o > lim ? lim : o);
  return o < 0 ? ((uint64_t)(-o) | sign) : (uint64_t)o;
}

__global__ __launch_bounds__(kPerturbThreads) void k_perturb(uint8_t* arena, PerturbArgs a) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < a.total;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t lo = 0, hi = a.n - 1u;  // first buffer whose prefix end exceeds i
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (a.end[mid] > i) hi = mid; else lo = mid + 1u;
    }
    const uint64_t start = lo == 0u ? 0ull : a.end[lo - 1u];
    const uint64_t j = i - start, sd = a.seed[lo];
    const uint64_t h1 = mix32(sd * 0x9E37ull + j * 0x85EBull + 1ull);
    const uint64_t h2 = mix32(h1 + sd + 0x27D4EB2Full);
    const uint64_t pos = a.off[lo] + j * a.block + h1 % a.block;
    int64_t k = 1 + (int64_t)(h2 % a.kmax);
    if ((h2 >> 20) & 1ull) k = -k;
    const uint64_t p = (uint64_t)arena + pos * a.width;
    store_elem(p, a.width, step_bits(load_elem(p, a.width), k, a));
  }
}

// Element width, integer flag, clamp code and NaN form of each element type.
bool perturb_format(uint32_t dtype, PerturbArgs& a) {
  a.is_int = 0;
  a.nan_is_neg_zero = 0;
  switch (dtype) {
    case KC_F32: a.width = 4; a.limit = 0x7F800000ull; return true;
    case KC_BF16: a.width = 2; a.limit = 0x7F80ull; return true;
    case KC_F16: a.width = 2; a.limit = 0x7C00ull; return true;
    case KC_F64: a.width = 8; a.limit = 0x7FF0000000000000ull; return true;
    case KC_FP8_E4M3FN: a.width = 1; a.limit = 0x7Eull; return true;  // no inf: the largest finite
    case KC_FP8_E5M2: a.width = 1; a.limit = 0x7Cull; return true;
    case KC_FP8_E4M3FNUZ:
    case KC_FP8_E5M2FNUZ: a.width = 1; a.limit = 0x7Full; a.nan_is_neg_zero = 1; return true;
    case KC_I8: a.width = 1; a.is_int = 1; return true;
    case KC_I16: a.width = 2; a.is_int = 1; return true;
    case KC_I32: a.width = 4; a.is_int = 1; return true;
    case KC_I64: a.width = 8; a.is_int = 1; return true;
    default: return false;
  }
}

}  // namespace
}  // namespace kc

using namespace kc;

extern "C" {

int kc_perturb(kc_ctx* c, void* arena_d, uint64_t arena_elems, uint32_t dtype, const kc_perturb_buf* bufs,
               uint32_t n_bufs, uint64_t block, uint32_t kmax, void* stream) {
  if (c == nullptr || (n_bufs > 0 && (bufs == nullptr || arena_d == nullptr)) || block == 0 || kmax == 0)
    return KC_EINVAL;
  PerturbArgs a{};
  if (!perturb_format(dtype, a)) return KC_EDTYPE;
  for (uint32_t b = 0; b < n_bufs; ++b)
    if (bufs[b].offset > arena_elems || bufs[b].length > arena_elems - bufs[b].offset) return KC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(arena_d) & (a.width - 1u)) != 0) return KC_EALIGN;
  a.block = block;
  a.kmax = kmax;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (uint32_t b0 = 0; b0 < n_bufs;) {
    a.n = 0;
    a.total = 0;
    for (; b0 < n_bufs && a.n < kPerturbBufs; ++b0) {
      const uint64_t m = bufs[b0].length / block;
      if (m == 0) continue;
      a.off[a.n] = bufs[b0].offset;
      a.seed[a.n] = bufs[b0].seed & 0x7FFFFFFFu;
      a.total += m;
      a.end[a.n] = a.total;
      ++a.n;
    }
    if (a.total == 0) continue;
    const uint64_t want = (a.total + kPerturbThreads - 1) / kPerturbThreads;
    const uint32_t grid = (uint32_t)std::min<uint64_t>(want, 4ull * c->n_cu);
    hipLaunchKernelGGL(k_perturb, dim3(grid), dim3(kPerturbThreads), 0, s, static_cast<uint8_t*>(arena_d), a);
    KC_HIP(hipGetLastError());
  }
  return KC_OK;
}

}  // extern "C"

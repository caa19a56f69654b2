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

// How an element type steps: its width and the codes that bound a move.
struct PerturbFmt {
  uint32_t width;               // element bytes: 1, 2, 4, 8
  uint32_t is_int;              // two's complement integer
  uint64_t limit;               // float: code of +inf (or the largest finite); int: unused
  uint32_t nan_is_neg_zero;     // fnuz formats: the code 0x80 is the NaN, and there is no -0
};

struct PerturbArgs {
  uint64_t off[kPerturbBufs];   // element offset of each buffer
  uint64_t end[kPerturbBufs];   // inclusive prefix of moved elements (blocks) per buffer
  uint32_t seed[kPerturbBufs];  // already reduced to 31 bits
  uint64_t total;               // moved elements in this launch
  uint64_t block;
  uint32_t n, kmax;
  PerturbFmt f;
};

// The buffers of one materialisation launch: golden sources, destinations in
// the arena, and the inclusive prefix of their 16-byte vectors.
constexpr uint32_t kMatBufs = 56;  // buffers per launch (kernel arguments stay below 4 KiB)
struct MatArgs {
  uint64_t src[kMatBufs];       // golden buffer (16-byte aligned)
  uint64_t dst[kMatBufs];       // its place in the arena (16-byte aligned)
  uint64_t len[kMatBufs];       // elements
  uint64_t vend[kMatBufs];      // inclusive prefix of 16-byte vectors
  uint32_t seed[kMatBufs];      // already reduced to 31 bits
  uint64_t total;               // vectors in this launch
  uint64_t block;
  uint32_t n, kmax;
  PerturbFmt f;
};
static_assert(sizeof(MatArgs) <= 3584, "kernel arguments");

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
__device__ __forceinline__ uint64_t step_bits(uint64_t b, int64_t k, const PerturbFmt& a) {
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

// The move of block j of a buffer (seed sd): the index of the element it
// moves inside the buffer, and its signed step.
__device__ __forceinline__ void block_move(uint64_t sd, uint64_t j, uint64_t block, uint32_t kmax, uint64_t& pos,
                                           int64_t& k) {
  const uint64_t h1 = mix32(sd * 0x9E37ull + j * 0x85EBull + 1ull);
  const uint64_t h2 = mix32(h1 + sd + 0x27D4EB2Full);
  pos = j * block + h1 % block;
  k = 1 + (int64_t)(h2 % kmax);
  if ((h2 >> 20) & 1ull) k = -k;
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
    uint64_t pos;
    int64_t k;
    block_move(a.seed[lo], i - start, a.block, a.kmax, pos, k);
    const uint64_t p = (uint64_t)arena + (a.off[lo] + pos) * a.f.width;
    store_elem(p, a.f.width, step_bits(load_elem(p, a.f.width), k, a.f));
  }
}

// Element width, integer flag, clamp code and NaN form of each element type.
bool perturb_format(uint32_t dtype, PerturbFmt& a) {
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

// Element e (of width w) of 16 bytes held as four words, read and written.
__device__ __forceinline__ uint64_t vec_get(const uint32_t (&x)[4], uint32_t e, uint32_t w) {
  const uint32_t byte = e * w, wi = byte >> 2, sh = (byte & 3u) * 8u;
  if (w == 8u) return ((uint64_t)x[wi + 1] << 32) | x[wi];
  if (w == 4u) return x[wi];
  return (x[wi] >> sh) & (w == 2u ? 0xFFFFu : 0xFFu);
}
__device__ __forceinline__ void vec_set(uint32_t (&x)[4], uint32_t e, uint32_t w, uint64_t v) {
  const uint32_t byte = e * w, wi = byte >> 2, sh = (byte & 3u) * 8u;
  if (w == 8u) {
    x[wi] = (uint32_t)v;
    x[wi + 1] = (uint32_t)(v >> 32);
  } else if (w == 4u) {
    x[wi] = (uint32_t)v;
  } else {
    const uint32_t m = (w == 2u ? 0xFFFFu : 0xFFu) << sh;
    x[wi] = (x[wi] & ~m) | (((uint32_t)v << sh) & m);
  }
}

// Candidates in one pass: each thread copies 16-byte vectors of the goldens
// into their places in the arena and applies the moves of the (at most two)
// blocks each vector overlaps, so the arena equals a plain copy followed by
// k_perturb.  A buffer whose byte length is not a multiple of 16 ends in a
// short vector, read and written element by element, so nothing outside the
// golden is read and nothing outside the buffer's place is written.  The
// buffer table is copied into LDS once per workgroup, where each vector finds
// its buffer by binary search; a thread takes kMatUnroll vectors a round and
// issues all their loads before it moves and stores any.  The loads and
// stores are ordinary (cached): the compare that follows reads both sides.
constexpr uint32_t kMatUnroll = 4;

__global__ __launch_bounds__(kPerturbThreads) void k_materialize(MatArgs a) {
  __shared__ uint64_t s_vend[kMatBufs], s_src[kMatBufs], s_dst[kMatBufs], s_len[kMatBufs];
  __shared__ uint32_t s_seed[kMatBufs];
  for (uint32_t b = threadIdx.x; b < a.n; b += blockDim.x) {
    s_vend[b] = a.vend[b];
    s_src[b] = a.src[b];
    s_dst[b] = a.dst[b];
    s_len[b] = a.len[b];
    s_seed[b] = a.seed[b];
  }
  __syncthreads();
  const uint32_t w = a.f.width, epv = 16u / w;
  const uint64_t round = (uint64_t)blockDim.x * kMatUnroll;
  for (uint64_t base = blockIdx.x * round + threadIdx.x; base < a.total; base += (uint64_t)gridDim.x * round) {
    uint32_t buf[kMatUnroll], valid[kMatUnroll];
    uint64_t vec[kMatUnroll];
    uint32_t x[kMatUnroll][4];
#pragma unroll
    for (uint32_t u = 0; u < kMatUnroll; ++u) {
      const uint64_t i = base + (uint64_t)u * blockDim.x;
      x[u][0] = x[u][1] = x[u][2] = x[u][3] = 0u;
      valid[u] = 0u;
      buf[u] = 0u;
      vec[u] = 0u;
      if (i >= a.total) continue;
      uint32_t lo = 0, hi = a.n - 1u;  // first buffer whose vector prefix exceeds i
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_vend[mid] > i) hi = mid; else lo = mid + 1u;
      }
      const uint64_t v = i - (lo == 0u ? 0ull : s_vend[lo - 1u]);
      const uint32_t n = (uint32_t)min<uint64_t>(epv, s_len[lo] - v * epv);
      const uint64_t src = s_src[lo] + v * 16u;
      if (n == epv) {
        const uint4 in = ld16(src);
        x[u][0] = in.x; x[u][1] = in.y; x[u][2] = in.z; x[u][3] = in.w;
      } else {
        for (uint32_t e = 0; e < n; ++e) vec_set(x[u], e, w, load_elem(src + e * w, w));
      }
      buf[u] = lo;
      vec[u] = v;
      valid[u] = n;
    }
#pragma unroll
    for (uint32_t u = 0; u < kMatUnroll; ++u) {
      const uint32_t n = valid[u];
      if (n == 0u) continue;
      const uint32_t lo = buf[u];
      const uint64_t e0 = vec[u] * epv, n_blocks = s_len[lo] / a.block, sd = s_seed[lo];
      const uint64_t j0 = e0 / a.block, j1 = (e0 + n - 1u) / a.block;
      for (uint64_t j = j0; j <= j1 && j < n_blocks; ++j) {
        uint64_t pos;
        int64_t k;
        block_move(sd, j, a.block, a.kmax, pos, k);
        if (pos >= e0 && pos < e0 + n) {
          const uint32_t e = (uint32_t)(pos - e0);
          vec_set(x[u], e, w, step_bits(vec_get(x[u], e, w), k, a.f));
        }
      }
      const uint64_t dst = s_dst[lo] + vec[u] * 16u;
      if (n == epv) {
        st16(dst, make_uint4(x[u][0], x[u][1], x[u][2], x[u][3]));
      } else {
        for (uint32_t e = 0; e < n; ++e) store_elem(dst + e * w, w, vec_get(x[u], e, w));
      }
    }
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
  if (!perturb_format(dtype, a.f)) return KC_EDTYPE;
  for (uint32_t b = 0; b < n_bufs; ++b)
    if (bufs[b].offset > arena_elems || bufs[b].length > arena_elems - bufs[b].offset) return KC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(arena_d) & (a.f.width - 1u)) != 0) return KC_EALIGN;
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

int kc_materialize(kc_ctx* c, void* arena_d, uint64_t arena_elems, uint32_t dtype, const kc_materialize_buf* bufs,
                   uint32_t n_bufs, uint64_t block, uint32_t kmax, void* stream) {
  if (c == nullptr || (n_bufs > 0 && (bufs == nullptr || arena_d == nullptr)) || block == 0 || kmax == 0)
    return KC_EINVAL;
  MatArgs a{};
  if (!perturb_format(dtype, a.f)) return KC_EDTYPE;
  const uint64_t w = a.f.width;
  for (uint32_t b = 0; b < n_bufs; ++b) {
    const kc_materialize_buf& m = bufs[b];
    if (m.offset > arena_elems || m.length > arena_elems - m.offset) return KC_EINVAL;
    if (m.length > 0 && m.src_d == nullptr) return KC_EINVAL;
    if (((reinterpret_cast<uintptr_t>(m.src_d) | (reinterpret_cast<uintptr_t>(arena_d) + m.offset * w)) & 15u) != 0)
      return KC_EALIGN;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  a.block = block;
  a.kmax = kmax;
  for (uint32_t b0 = 0; b0 < n_bufs;) {
    a.n = 0;
    a.total = 0;
    for (; b0 < n_bufs && a.n < kMatBufs; ++b0) {
      const kc_materialize_buf& m = bufs[b0];
      const uint64_t vecs = (m.length * w + 15u) / 16u;
      if (vecs == 0) continue;
      a.src[a.n] = reinterpret_cast<uint64_t>(m.src_d);
      a.dst[a.n] = reinterpret_cast<uint64_t>(arena_d) + m.offset * w;
      a.len[a.n] = m.length;
      a.seed[a.n] = m.seed & 0x7FFFFFFFu;
      a.total += vecs;
      a.vend[a.n] = a.total;
      ++a.n;
    }
    if (a.total == 0) continue;
    const uint64_t want = (a.total + kPerturbThreads * kMatUnroll - 1) / (kPerturbThreads * kMatUnroll);
    const uint32_t grid = (uint32_t)std::min<uint64_t>(want, 8ull * c->n_cu);
    hipLaunchKernelGGL(k_materialize, dim3(grid), dim3(kPerturbThreads), 0, s, a);
    KC_HIP(hipGetLastError());
  }
  return KC_OK;
}

}  // extern "C"

// kc_compare.hip -- gfx950 typed compare of candidate / golden buffer pairs.
//
// One persistent launch walks a tile list that covers every pair (uneven
// sizes, mixed element types).  A 256-thread workgroup takes a tile of up to
// tile_bytes of each side, streams it with 16-byte loads, and keeps a fast
// path for runs whose 16 bytes are bitwise equal and hold no NaN; anything
// else goes element by element through the exact path (ULP distance, fp64
// abs / rel error, NaN classes).  Tile partials go to per-pair accumulators
// with integer atomics (max of non-negative doubles via their bit patterns,
// first mismatch via max of its complement); tiles with nothing but equal
// elements flush nothing.  A second small kernel writes each pair's report
// once the pass has finished.
#include "kc_internal.h"

namespace kc {
namespace {

constexpr uint32_t kThreads = 256;
constexpr uint32_t kUnroll = 4;
constexpr uint32_t kBins = 48;

// Element formats.  B holds one element's encoding; kind 0 = floating point
// in sign-magnitude order, 1 = two's complement integer, 2 = raw bytes.
template <uint32_t DT> struct Fmt;
template <> struct Fmt<KC_F32> {
  using B = uint32_t;
  static constexpr uint32_t size = 4, kind = 0;
  static constexpr B mag = 0x7FFFFFFFu;
  __device__ static bool nan(B b) { return (b & mag) > 0x7F800000u; }
  __device__ static bool inf(B b) { return (b & mag) == 0x7F800000u; }
  __device__ static double value(B b) { return (double)__uint_as_float(b); }
};
template <> struct Fmt<KC_F64> {
  using B = uint64_t;
  static constexpr uint32_t size = 8, kind = 0;
  static constexpr B mag = 0x7FFFFFFFFFFFFFFFull;
  __device__ static bool nan(B b) { return (b & mag) > 0x7FF0000000000000ull; }
  __device__ static bool inf(B b) { return (b & mag) == 0x7FF0000000000000ull; }
  __device__ static double value(B b) { return __longlong_as_double((long long)b); }
};
template <> struct Fmt<KC_BF16> {
  using B = uint32_t;
  static constexpr uint32_t size = 2, kind = 0;
  static constexpr B mag = 0x7FFFu;
  __device__ static bool nan(B b) { return (b & mag) > 0x7F80u; }
  __device__ static bool inf(B b) { return (b & mag) == 0x7F80u; }
  __device__ static double value(B b) { return (double)__uint_as_float(b << 16); }
};
// value of a finite small-float encoding: subnormal when the exponent is 0
__device__ __forceinline__ double small_value(uint32_t e, uint32_t m, uint32_t mbits, int bias) {
  return e == 0u ? (double)m * __builtin_ldexp(1.0, 1 - bias - (int)mbits)
                 : (double)(m | (1u << mbits)) * __builtin_ldexp(1.0, (int)e - bias - (int)mbits);
}
template <> struct Fmt<KC_F16> {
  using B = uint32_t;
  static constexpr uint32_t size = 2, kind = 0;
  static constexpr B mag = 0x7FFFu;
  __device__ static bool nan(B b) { return (b & mag) > 0x7C00u; }
  __device__ static bool inf(B b) { return (b & mag) == 0x7C00u; }
  __device__ static double value(B b) {
    const uint32_t e = (b >> 10) & 0x1Fu;
    const double v = e == 31u ? __builtin_inf() : small_value(e, b & 0x3FFu, 10, 15);  // NaN never decoded
    return (b & 0x8000u) ? -v : v;
  }
};
template <> struct Fmt<KC_FP8_E4M3FN> {
  using B = uint32_t;
  static constexpr uint32_t size = 1, kind = 0;
  static constexpr B mag = 0x7Fu;
  __device__ static bool nan(B b) { return (b & mag) == 0x7Fu; }
  __device__ static bool inf(B) { return false; }
  __device__ static double value(B b) {
    const double v = small_value((b >> 3) & 0xFu, b & 0x7u, 3, 7);
    return (b & 0x80u) ? -v : v;
  }
};
template <> struct Fmt<KC_FP8_E4M3FNUZ> {
  using B = uint32_t;
  static constexpr uint32_t size = 1, kind = 0;
  static constexpr B mag = 0x7Fu;
  __device__ static bool nan(B b) { return b == 0x80u; }
  __device__ static bool inf(B) { return false; }
  __device__ static double value(B b) {
    const double v = small_value((b >> 3) & 0xFu, b & 0x7u, 3, 8);
    return (b & 0x80u) ? -v : v;
  }
};
template <> struct Fmt<KC_FP8_E5M2> {
  using B = uint32_t;
  static constexpr uint32_t size = 1, kind = 0;
  static constexpr B mag = 0x7Fu;
  __device__ static bool nan(B b) { return (b & mag) > 0x7Cu; }
  __device__ static bool inf(B b) { return (b & mag) == 0x7Cu; }
  __device__ static double value(B b) {
    const uint32_t e = (b >> 2) & 0x1Fu;
    const double v = e == 31u ? __builtin_inf() : small_value(e, b & 0x3u, 2, 15);
    return (b & 0x80u) ? -v : v;
  }
};
template <> struct Fmt<KC_FP8_E5M2FNUZ> {
  using B = uint32_t;
  static constexpr uint32_t size = 1, kind = 0;
  static constexpr B mag = 0x7Fu;
  __device__ static bool nan(B b) { return b == 0x80u; }
  __device__ static bool inf(B) { return false; }
  __device__ static double value(B b) {
    const double v = small_value((b >> 2) & 0x1Fu, b & 0x3u, 2, 16);
    return (b & 0x80u) ? -v : v;
  }
};
template <uint32_t SIZE, typename BT> struct IntFmt {
  using B = BT;
  static constexpr uint32_t size = SIZE, kind = 1;
  static constexpr B mag = 0;
  __device__ static bool nan(B) { return false; }
  __device__ static bool inf(B) { return false; }
  __device__ static int64_t sext(B b) {
    if (SIZE == 1) return (int64_t)(int8_t)(uint8_t)b;
    if (SIZE == 2) return (int64_t)(int16_t)(uint16_t)b;
    if (SIZE == 4) return (int64_t)(int32_t)(uint32_t)b;
    return (int64_t)b;
  }
  __device__ static double value(B b) { return (double)sext(b); }
};
template <> struct Fmt<KC_I8> : IntFmt<1, uint32_t> {};
template <> struct Fmt<KC_I16> : IntFmt<2, uint32_t> {};
template <> struct Fmt<KC_I32> : IntFmt<4, uint32_t> {};
template <> struct Fmt<KC_I64> : IntFmt<8, uint64_t> {};
template <> struct Fmt<KC_U8> {
  using B = uint32_t;
  static constexpr uint32_t size = 1, kind = 2;
  static constexpr B mag = 0xFFu;
  __device__ static bool nan(B) { return false; }
  __device__ static bool inf(B) { return false; }
  __device__ static double value(B) { return 0.0; }
};

// Zero byte anywhere in a 32-bit word.
__device__ __forceinline__ bool has_zero_byte(uint32_t y) { return ((y - 0x01010101u) & ~y & 0x80808080u) != 0u; }

// Any NaN encoding among the elements packed in 16 bytes.
template <uint32_t DT> __device__ __forceinline__ bool vec_has_nan(const uint4& v) {
  if (Fmt<DT>::kind != 0) return false;
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  bool any = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t x = w[i];
    if (DT == KC_F32) any |= (x & 0x7FFFFFFFu) > 0x7F800000u;
    if (DT == KC_BF16) any |= (x & 0x7FFFu) > 0x7F80u || ((x >> 16) & 0x7FFFu) > 0x7F80u;
    if (DT == KC_F16) any |= (x & 0x7FFFu) > 0x7C00u || ((x >> 16) & 0x7FFFu) > 0x7C00u;
    if (DT == KC_FP8_E4M3FN) any |= has_zero_byte((x & 0x7F7F7F7Fu) ^ 0x7F7F7F7Fu);  // magnitude 0x7F
    if (DT == KC_FP8_E4M3FNUZ || DT == KC_FP8_E5M2FNUZ) any |= has_zero_byte(x ^ 0x80808080u);  // byte 0x80
    if (DT == KC_FP8_E5M2) any |= (((x & 0x7F7F7F7Fu) + 0x03030303u) & 0x80808080u) != 0u;    // magnitude > 0x7C
    if (DT == KC_F64 && (i & 1)) {  // high word of a binary64 element
      const uint32_t hi = x & 0x7FFFFFFFu;
      any |= hi > 0x7FF00000u || (hi == 0x7FF00000u && w[i - 1] != 0u);
    }
  }
  return any;
}

struct Partial {
  uint32_t mis_elems, mis_bytes, nan_both, nan_c, nan_g, over, not_close;
  double max_abs, max_rel;
  uint64_t first;
};

struct Tol {
  uint32_t ulp;
  double atol, rtol;
};

__device__ __forceinline__ uint32_t ulp_bin(uint64_t d) {
  if (d <= 16u) return (uint32_t)d;
  const uint32_t b = 12u + (64u - (uint32_t)__clzll(d - 1ull));  // 12 + ceil(log2 d)
  return b < kBins - 1u ? b : kBins - 1u;
}

template <typename B> __device__ __forceinline__ uint32_t diff_bytes(B a, B b) {
  const B x = a ^ b;
  uint32_t n = 0;
#pragma unroll
  for (uint32_t i = 0; i < sizeof(B); ++i) n += (uint32_t)(((x >> (8u * i)) & 0xFFu) != 0u);
  return n;
}

// Exact per-element path.
template <uint32_t DT>
__device__ __forceinline__ void element(typename Fmt<DT>::B c, typename Fmt<DT>::B g, uint64_t idx, const Tol& tol,
                                        Partial& p, uint32_t* hist) {
  using F = Fmt<DT>;
  if (c != g) {
    ++p.mis_elems;
    p.mis_bytes += diff_bytes(c, g);
    if (idx < p.first) p.first = idx;
  }
  if constexpr (F::kind == 2) return;
  const bool nc = F::nan(c), ng = F::nan(g);
  if (nc || ng) {
    if (nc && ng) ++p.nan_both;
    else if (nc) ++p.nan_c;
    else ++p.nan_g;
    return;
  }
  uint64_t d;
  if constexpr (F::kind == 1) {
    const int64_t ci = F::sext(c), gi = F::sext(g);
    d = ci >= gi ? (uint64_t)ci - (uint64_t)gi : (uint64_t)gi - (uint64_t)ci;  // exact below 2^64
  } else {
    constexpr typename F::B sb = (typename F::B)1 << (8u * F::size - 1u);
    const uint64_t mc = (uint64_t)(c & F::mag), mg = (uint64_t)(g & F::mag);
    d = ((c ^ g) & sb) == 0 ? (mc > mg ? mc - mg : mg - mc) : mc + mg;  // across zero: the two magnitudes
  }
  if (d > tol.ulp) ++p.over;
  if (d != 0u) atomicAdd(&hist[ulp_bin(d)], 1u);
  if (c == g) return;
  const double vc = F::value(c), vg = F::value(g);
  const double a = F::kind == 1 ? (double)d : __builtin_fabs(vc - vg);
  if (a > p.max_abs) p.max_abs = a;
  if (vg != 0.0 && !F::inf(g)) {
    const double r = a / __builtin_fabs(vg);
    if (r > p.max_rel) p.max_rel = r;
  }
  // tolerance test: an infinity is close only to an equal value
  if (F::inf(c) || F::inf(g)) {
    if (vc != vg) ++p.not_close;
  } else {
    const double bound = tol.atol + tol.rtol * __builtin_fabs(vg);
    if (a > bound) ++p.not_close;
  }
}

template <uint32_t DT>
__device__ __forceinline__ typename Fmt<DT>::B elem_of(const uint4& v, uint32_t e) {
  constexpr uint32_t sz = Fmt<DT>::size;
  if (sz == 8) {
    return e == 0 ? (typename Fmt<DT>::B)(((uint64_t)v.y << 32) | v.x)
                  : (typename Fmt<DT>::B)(((uint64_t)v.w << 32) | v.z);
  }
  const uint32_t w = e * sz / 4u;
  const uint32_t word = w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
  if (sz == 4) return word;
  if (sz == 2) return (e & 1u) ? (word >> 16) : (word & 0xFFFFu);
  return (word >> (8u * (e & 3u))) & 0xFFu;
}

template <uint32_t DT>
__device__ __forceinline__ void vec16(const uint4& c, const uint4& g, uint64_t e0, const Tol& tol, Partial& p,
                                      uint32_t* hist) {
  const bool eq = c.x == g.x && c.y == g.y && c.z == g.z && c.w == g.w;
  if (eq && !vec_has_nan<DT>(g)) return;
  constexpr uint32_t epv = 16u / Fmt<DT>::size;
#pragma unroll
  for (uint32_t e = 0; e < epv; ++e) element<DT>(elem_of<DT>(c, e), elem_of<DT>(g, e), e0 + e, tol, p, hist);
}

template <uint32_t DT>
__device__ __forceinline__ void tile_body(const CmpPairDev& pr, uint64_t b0, uint64_t b1, Partial& p, uint32_t* hist) {
  using B = typename Fmt<DT>::B;
  constexpr uint32_t es = Fmt<DT>::size;
  const uint64_t nvec = (b1 - b0) / 16u;
  const uint32_t tid = threadIdx.x;
  const Tol tol{pr.tol, pr.atol, pr.rtol};
  for (uint64_t v0 = tid; v0 < nvec; v0 += (uint64_t)kThreads * kUnroll) {
    uint4 c[kUnroll], g[kUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
      const uint64_t v = v0 + (uint64_t)u * kThreads;
      if (v < nvec) {
        c[u] = ld16nt((uint64_t)(pr.cand + b0 + v * 16u));
        g[u] = ld16nt((uint64_t)(pr.gold + b0 + v * 16u));
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kUnroll; ++u) {
      const uint64_t v = v0 + (uint64_t)u * kThreads;
      if (v < nvec) vec16<DT>(c[u], g[u], (b0 + v * 16u) / es, tol, p, hist);
    }
  }
  // bytes past the last whole 16-byte run: element by element
  if (tid == 0) {
    const KC_GLOBAL uint8_t* cb = (const KC_GLOBAL uint8_t*)pr.cand;
    const KC_GLOBAL uint8_t* gb = (const KC_GLOBAL uint8_t*)pr.gold;
    for (uint64_t b = b0 + nvec * 16u; b < b1; b += es) {
      B cv = 0, gv = 0;
      for (uint32_t i = 0; i < es; ++i) {
        cv |= (B)cb[b + i] << (8u * i);
        gv |= (B)gb[b + i] << (8u * i);
      }
      element<DT>(cv, gv, b / es, tol, p, hist);
    }
  }
}

// One element of `es` bytes at a naturally aligned address, zero-extended.
template <typename B, uint32_t ES>
__device__ __forceinline__ B load_elem(const uint8_t* base, uint64_t e) {
  const uint64_t a = (uint64_t)base + e * ES;
  if (ES == 1) return (B)*(const KC_GLOBAL uint8_t*)a;
  if (ES == 2) return (B)*(const KC_GLOBAL uint16_t*)a;
  if (ES == 4) return (B)*(const KC_GLOBAL uint32_t*)a;
  return (B)*(const KC_GLOBAL uint64_t*)a;
}

// A pair whose buffers are element-aligned but not both 16-byte aligned (a
// view at an odd element offset): element-sized loads, consecutive threads on
// consecutive elements; equal NaN-free elements skip the exact path.
template <uint32_t DT>
__device__ __forceinline__ void tile_body_elems(const CmpPairDev& pr, uint64_t b0, uint64_t b1, Partial& p,
                                                uint32_t* hist) {
  using F = Fmt<DT>;
  using B = typename F::B;
  constexpr uint32_t es = F::size;
  const Tol tol{pr.tol, pr.atol, pr.rtol};
  const uint64_t e1 = b1 / es;
  for (uint64_t e = b0 / es + threadIdx.x; e < e1; e += kThreads) {
    const B c = load_elem<B, es>(pr.cand, e), g = load_elem<B, es>(pr.gold, e);
    if (c == g && !F::nan(g)) continue;
    element<DT>(c, g, e, tol, p, hist);
  }
}

template <uint32_t DT>
__device__ __forceinline__ void tile_any(const CmpPairDev& pr, uint64_t b0, uint64_t b1, Partial& p, uint32_t* hist) {
  if ((((uint64_t)pr.cand | (uint64_t)pr.gold) & 15u) != 0u) tile_body_elems<DT>(pr, b0, b1, p, hist);
  else tile_body<DT>(pr, b0, b1, p, hist);
}

__device__ __forceinline__ uint64_t dbl_bits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double bits_dbl(uint64_t x) { return __longlong_as_double((long long)x); }

template <typename T>
__device__ __forceinline__ T wave_reduce_sum(T x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}
__device__ __forceinline__ uint64_t wave_reduce_max_u64(uint64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t y = __shfl_xor(x, d, 64);
    x = y > x ? y : x;
  }
  return x;
}

// One tile of one pair: the workgroup streams its bytes, then flushes what it
// found into the pair's accumulators (nothing when every element was equal).
// hist (48 bins) is zero on entry and left zero; red is a 4 x 10 exchange area.
__device__ __forceinline__ void compare_tile(const CmpPairDev& pr, uint64_t tile_idx, uint32_t tile_bytes,
                                             unsigned long long* acc, uint32_t* hist, uint64_t (*red)[10]) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  Partial p{0, 0, 0, 0, 0, 0, 0, 0.0, 0.0, ~0ull};
  const uint64_t nbytes = pr.n_elems * pr.esize;
  const uint64_t b0 = tile_idx * tile_bytes;
  const uint64_t b1 = b0 + tile_bytes < nbytes ? b0 + tile_bytes : nbytes;
  if (b0 < b1) {
    switch (pr.dtype) {
      case KC_F32: tile_any<KC_F32>(pr, b0, b1, p, hist); break;
      case KC_BF16: tile_any<KC_BF16>(pr, b0, b1, p, hist); break;
      case KC_F16: tile_any<KC_F16>(pr, b0, b1, p, hist); break;
      case KC_FP8_E4M3FN: tile_any<KC_FP8_E4M3FN>(pr, b0, b1, p, hist); break;
      case KC_F64: tile_any<KC_F64>(pr, b0, b1, p, hist); break;
      case KC_FP8_E4M3FNUZ: tile_any<KC_FP8_E4M3FNUZ>(pr, b0, b1, p, hist); break;
      case KC_FP8_E5M2: tile_any<KC_FP8_E5M2>(pr, b0, b1, p, hist); break;
      case KC_FP8_E5M2FNUZ: tile_any<KC_FP8_E5M2FNUZ>(pr, b0, b1, p, hist); break;
      case KC_I8: tile_any<KC_I8>(pr, b0, b1, p, hist); break;
      case KC_I16: tile_any<KC_I16>(pr, b0, b1, p, hist); break;
      case KC_I32: tile_any<KC_I32>(pr, b0, b1, p, hist); break;
      case KC_I64: tile_any<KC_I64>(pr, b0, b1, p, hist); break;
      default: tile_any<KC_U8>(pr, b0, b1, p, hist); break;
    }
  }
  // Every non-equal element bumps mis_elems or a NaN class, so a tile with
  // all of these zero contributed nothing but equal elements.
  const bool any = (p.mis_elems | p.nan_both | p.nan_c | p.nan_g) != 0u;
  if (!__syncthreads_or(any)) return;
  const uint64_t v0 = wave_reduce_sum<uint32_t>(p.mis_elems);
  const uint64_t v1 = wave_reduce_sum<uint32_t>(p.mis_bytes);
  const uint64_t v2 = wave_reduce_sum<uint32_t>(p.nan_both);
  const uint64_t v3 = wave_reduce_sum<uint32_t>(p.nan_c);
  const uint64_t v4 = wave_reduce_sum<uint32_t>(p.nan_g);
  const uint64_t v5 = wave_reduce_sum<uint32_t>(p.over);
  const uint64_t v6 = wave_reduce_max_u64(dbl_bits(p.max_abs));
  const uint64_t v7 = wave_reduce_max_u64(dbl_bits(p.max_rel));
  const uint64_t v8 = wave_reduce_max_u64(~p.first);
  const uint64_t v9 = wave_reduce_sum<uint32_t>(p.not_close);
  if (lane == 0) {
    red[wave][0] = v0; red[wave][1] = v1; red[wave][2] = v2; red[wave][3] = v3; red[wave][4] = v4;
    red[wave][5] = v5; red[wave][6] = v6; red[wave][7] = v7; red[wave][8] = v8; red[wave][9] = v9;
  }
  __syncthreads();
  if (tid < 10) {  // thread i folds slot i over the four waves and flushes it
    const uint32_t i = tid;
    const bool is_sum = i < 6 || i == 9;
    uint64_t x = red[0][i];
#pragma unroll
    for (uint32_t w = 1; w < 4; ++w) {
      const uint64_t y = red[w][i];
      x = is_sum ? x + y : (y > x ? y : x);
    }
    if (x) {
      if (i < 6) atomicAdd(&acc[kAccMisElems + i], (unsigned long long)x);
      else if (i == 9) atomicAdd(&acc[kAccNotClose], (unsigned long long)x);
      else atomicMax(&acc[kAccMaxAbs + (i - 6)], (unsigned long long)x);
    }
  }
  if (tid < kBins) {
    const uint32_t h = hist[tid];
    if (h) {
      atomicAdd(&acc[kAccHist + tid], (unsigned long long)h);
      hist[tid] = 0u;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_compare(const CmpPairDev* pairs, const CmpTileDev* tiles,
                                                 uint32_t n_tiles, uint32_t tile_bytes,
                                                 unsigned long long* acc_all) {
  __shared__ uint32_t hist[48];
  __shared__ uint64_t red[4][10];
  if (threadIdx.x < 48) hist[threadIdx.x] = 0u;  // stays zero between tiles: flushed bins are reset
  __syncthreads();
  for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const CmpTileDev tl = tiles[t];
    compare_tile(pairs[tl.pair], tl.idx, tile_bytes, acc_all + (uint64_t)tl.pair * kAccWords, hist, red);
  }
}

// The same pass over the pairs carried in the kernel arguments: tile t
// belongs to the first pair whose inclusive tile prefix exceeds t.
__global__ __launch_bounds__(256) void k_compare_args(CmpArgPairs a, uint32_t tile_bytes,
                                                      unsigned long long* acc_all) {
  __shared__ uint32_t hist[48];
  __shared__ uint64_t red[4][10];
  if (threadIdx.x < 48) hist[threadIdx.x] = 0u;
  __syncthreads();
  for (uint32_t t = blockIdx.x; t < a.n_tiles; t += gridDim.x) {
    uint32_t lo = 0, hi = a.n - 1u;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (a.tile_end[mid] > t) hi = mid; else lo = mid + 1u;
    }
    const uint32_t start = lo == 0u ? 0u : a.tile_end[lo - 1u];
    compare_tile(a.pair[lo], t - start, tile_bytes, acc_all + (uint64_t)lo * kAccWords, hist, red);
  }
}

// One pair's report from its accumulators, which are zeroed again.
__device__ __forceinline__ void finalize_pair(const CmpPairDev& pr, unsigned long long* acc, kc_cmp_result* r) {
  const uint64_t nb = acc[kAccNanBoth], ncand = acc[kAccNanCand], ngold = acc[kAccNanGold], over = acc[kAccOverTol];
  r->n_elems = pr.n_elems;
  r->n_mismatch_elems = acc[kAccMisElems];
  r->n_mismatch_bytes = acc[kAccMisBytes];
  r->first_mismatch = ~(uint64_t)acc[kAccFirstInv];
  r->n_nan_both = nb;
  r->n_nan_cand_only = ncand;
  r->n_nan_gold_only = ngold;
  r->n_over_tol = over;
  r->max_abs = bits_dbl(acc[kAccMaxAbs]);
  r->max_rel = bits_dbl(acc[kAccMaxRel]);
  uint64_t rest = 0;
  for (uint32_t b = 1; b < 48; ++b) {
    const uint64_t h = b < kBins ? (uint64_t)acc[kAccHist + b] : 0ull;
    r->ulp_hist[b] = h;
    rest += h;
  }
  const uint64_t not_close = acc[kAccNotClose];
  r->n_not_close = not_close;
  if (pr.dtype == KC_U8) {
    r->ulp_hist[0] = 0;
    r->pass = r->n_mismatch_elems == 0 ? 1u : 0u;
    r->pass_close = r->pass;
  } else {
    r->ulp_hist[0] = pr.n_elems - nb - ncand - ngold - rest;
    r->pass = (over == 0 && ncand == 0 && ngold == 0) ? 1u : 0u;
    r->pass_close = (not_close == 0 && ncand == 0 && ngold == 0) ? 1u : 0u;
  }
  r->status = 0u;
  r->reserved = 0u;
  for (uint32_t w = 0; w < kAccWords; ++w) acc[w] = 0ull;  // ready for the next call
}

// One thread per pair turns the accumulators into the report and zeroes them.
__global__ __launch_bounds__(256) void k_compare_finalize(const CmpPairDev* pairs, uint32_t n_pairs,
                                                          unsigned long long* acc_all, kc_cmp_result* res) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pairs) return;
  finalize_pair(pairs[i], acc_all + (uint64_t)i * kAccWords, res + i);
}

__global__ __launch_bounds__(64) void k_compare_args_finalize(CmpArgPairs a, unsigned long long* acc_all,
                                                              kc_cmp_result* res) {
  const uint32_t i = threadIdx.x;
  if (i >= a.n) return;
  finalize_pair(a.pair[i], acc_all + (uint64_t)i * kAccWords, res + i);
}

}  // namespace

hipError_t launch_compare(const CmpPairDev* pairs, const CmpTileDev* tiles, uint32_t n_tiles,
                          uint32_t tile_bytes, unsigned long long* acc, uint32_t grid, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  grid = grid < 1u ? 1u : (grid > n_tiles ? n_tiles : grid);
  hipLaunchKernelGGL(k_compare, dim3(grid), dim3(kThreads), 0, s, pairs, tiles, n_tiles, tile_bytes, acc);
  return hipGetLastError();
}

hipError_t launch_compare_finalize(const CmpPairDev* pairs, uint32_t n_pairs, unsigned long long* acc,
                                   kc_cmp_result* res, hipStream_t s) {
  if (n_pairs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_compare_finalize, dim3((n_pairs + 255) / 256), dim3(256), 0, s, pairs, n_pairs, acc, res);
  return hipGetLastError();
}

hipError_t launch_compare_args(const CmpArgPairs& a, uint32_t tile_bytes, unsigned long long* acc,
                               kc_cmp_result* res, uint32_t grid, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  grid = grid < 1u ? 1u : (grid > a.n_tiles ? a.n_tiles : grid);
  hipLaunchKernelGGL(k_compare_args, dim3(grid), dim3(kThreads), 0, s, a, tile_bytes, acc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  static_assert(kArgPairs <= 64, "one finalize thread per pair");
  hipLaunchKernelGGL(k_compare_args_finalize, dim3(1), dim3(64), 0, s, a, acc, res);
  return hipGetLastError();
}

}  // namespace kc

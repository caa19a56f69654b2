/*
 * kco.c -- CPU oracle for the snapshot / validation hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see kco.h).  Plain, slow, single-threaded C99,
 * compiled without fast-math and with FP contraction off so that every fp64
 * operation is one IEEE-754 round-to-nearest-even operation.
 */
#include "kco.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define PAGE 4096u

/* ------------------------------------------------------------------------ */
/* XXH64, written from the public xxHash specification (Y. Collet): four     */
/* accumulators over 32-byte stripes, merge, length, tail, avalanche.        */
/* ------------------------------------------------------------------------ */

static const uint64_t PRIME1 = 0x9E3779B185EBCA87ULL;
static const uint64_t PRIME2 = 0xC2B2AE3D27D4EB4FULL;
static const uint64_t PRIME3 = 0x165667B19E3779F9ULL;
static const uint64_t PRIME4 = 0x85EBCA77C2B2AE63ULL;
static const uint64_t PRIME5 = 0x27D4EB2F165667C5ULL;

static uint64_t rotate_left(uint64_t x, unsigned r) {
  return (x << r) | (x >> (64u - r));
}

static uint64_t read_u64_le(const uint8_t *p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; --i) v = (v << 8) | (uint64_t)p[i];
  return v;
}

static uint32_t read_u32_le(const uint8_t *p) {
  uint32_t v = 0;
  for (int i = 3; i >= 0; --i) v = (v << 8) | (uint32_t)p[i];
  return v;
}

static uint64_t xxh_round(uint64_t acc, uint64_t lane) {
  acc = acc + lane * PRIME2;
  acc = rotate_left(acc, 31);
  return acc * PRIME1;
}

static uint64_t xxh_merge_accumulator(uint64_t acc, uint64_t v) {
  acc = acc ^ xxh_round(0, v);
  return acc * PRIME1 + PRIME4;
}

uint64_t kco_xxh64(const void *data, uint64_t len, uint64_t seed) {
  const uint8_t *p = (const uint8_t *)data;
  uint64_t remaining = len;
  uint64_t acc;
  if (len >= 32) {
    uint64_t v1 = seed + PRIME1 + PRIME2;
    uint64_t v2 = seed + PRIME2;
    uint64_t v3 = seed;
    uint64_t v4 = seed - PRIME1;
    while (remaining >= 32) {
      v1 = xxh_round(v1, read_u64_le(p + 0));
      v2 = xxh_round(v2, read_u64_le(p + 8));
      v3 = xxh_round(v3, read_u64_le(p + 16));
      v4 = xxh_round(v4, read_u64_le(p + 24));
      p += 32;
      remaining -= 32;
    }
    acc = rotate_left(v1, 1) + rotate_left(v2, 7) + rotate_left(v3, 12) +
          rotate_left(v4, 18);
    acc = xxh_merge_accumulator(acc, v1);
    acc = xxh_merge_accumulator(acc, v2);
    acc = xxh_merge_accumulator(acc, v3);
    acc = xxh_merge_accumulator(acc, v4);
  } else {
    acc = seed + PRIME5;
  }
  acc += len;
  while (remaining >= 8) {
    acc ^= xxh_round(0, read_u64_le(p));
    acc = rotate_left(acc, 27) * PRIME1 + PRIME4;
    p += 8;
    remaining -= 8;
  }
  if (remaining >= 4) {
    acc ^= (uint64_t)read_u32_le(p) * PRIME1;
    acc = rotate_left(acc, 23) * PRIME2 + PRIME3;
    p += 4;
    remaining -= 4;
  }
  while (remaining > 0) {
    acc ^= (uint64_t)(*p) * PRIME5;
    acc = rotate_left(acc, 11) * PRIME1;
    p += 1;
    remaining -= 1;
  }
  acc ^= acc >> 33;
  acc *= PRIME2;
  acc ^= acc >> 29;
  acc *= PRIME3;
  acc ^= acc >> 32;
  return acc;
}

/* ------------------------------------------------------------------------ */
/* Range table: the pointer-to-size map of tracked allocations               */
/* (paper Sec. 4.1.1), as sorted, disjoint (base, size) with a page-aligned  */
/* base.  A range spans ceil(size / 4096) pages; its last page holds the     */
/* remaining size mod 4096 bytes when that is not zero.                      */
/* ------------------------------------------------------------------------ */

/* The hash unit: a power of two from 4 KiB to 2 MiB. */
static int unit_ok(uint64_t unit) {
  return unit >= PAGE && unit <= (2u << 20) && (unit & (unit - 1)) == 0;
}

int kco_range_check_unit(const kco_range *ranges, uint32_t n, uint64_t unit,
                         uint64_t *first_page, uint64_t *n_pages) {
  uint64_t pages = 0;
  if (!unit_ok(unit)) return KCO_EINVAL;
  if (n > 0 && ranges == NULL) return KCO_EINVAL;
  if (first_page) first_page[0] = 0;
  for (uint32_t a = 0; a < n; ++a) {
    uint64_t base = ranges[a].base, size = ranges[a].size;
    if (base == 0 || size == 0) return KCO_EINVAL;
    if (base % PAGE != 0) return KCO_EALIGN;
    if (base + size < base) return KCO_EINVAL; /* wraps around 2^64 */
    if (a > 0) {
      uint64_t prev_end = ranges[a - 1].base + ranges[a - 1].size;
      if (base < prev_end) return KCO_EORDER;
    }
    pages += (size + unit - 1) / unit;
    if (first_page) first_page[a + 1] = pages;
  }
  if (n_pages) *n_pages = pages;
  return KCO_OK;
}

int kco_range_check(const kco_range *ranges, uint32_t n, uint64_t *first_page,
                    uint64_t *n_pages) {
  return kco_range_check_unit(ranges, n, PAGE, first_page, n_pages);
}

int kco_default_window(const kco_range *ranges, uint32_t n, uint64_t *lo,
                       uint64_t *hi) {
  const uint64_t margin = 1ULL << 32; /* 4 GiB either side */
  if (n == 0) {
    *lo = 0;
    *hi = 0;
    return KCO_OK;
  }
  uint64_t min_base = ranges[0].base;
  uint64_t max_end = ranges[n - 1].base + ranges[n - 1].size;
  *lo = (min_base > margin + PAGE) ? min_base - margin : PAGE;
  *hi = (max_end <= UINT64_MAX - margin) ? max_end + margin : UINT64_MAX;
  return KCO_OK;
}

static int bit_get(const uint64_t *bm, uint64_t g) {
  return (int)((bm[g / 64] >> (g % 64)) & 1u);
}

static void bit_set(uint64_t *bm, uint64_t g) {
  bm[g / 64] |= 1ULL << (g % 64);
}

static int page_is_zero(const uint8_t *page, uint64_t len) {
  for (uint64_t i = 0; i < len; ++i)
    if (page[i] != 0) return 0;
  return 1;
}

/* Units of a range and the bytes of its unit p (the last may be partial). */
static uint64_t range_pages(const kco_range *r, uint64_t unit) { return (r->size + unit - 1) / unit; }

static uint64_t page_len(const kco_range *r, uint64_t p, uint64_t unit) {
  uint64_t rest = r->size - p * unit;
  return rest < unit ? rest : unit;
}

/* ------------------------------------------------------------------------ */
/* Snapshot: page hash + zero + changed                                      */
/* ------------------------------------------------------------------------ */

int kco_page_hash_unit(const kco_range *ranges, const uint8_t *const *host_ptr,
                       uint32_t n, uint64_t unit, uint64_t seed, const uint64_t *prior,
                       uint64_t *hash, uint64_t *zero_bm, uint64_t *changed_bm) {
  uint64_t n_pages = 0;
  int st = kco_range_check_unit(ranges, n, unit, NULL, &n_pages);
  if (st != KCO_OK) return st;
  if (n_pages > 0 && (hash == NULL || zero_bm == NULL)) return KCO_EINVAL;
  if (prior != NULL && changed_bm == NULL) return KCO_EINVAL;
  uint64_t n_words = (n_pages + 63) / 64;
  for (uint64_t w = 0; w < n_words; ++w) {
    zero_bm[w] = 0;
    if (prior) changed_bm[w] = 0;
  }
  uint64_t g = 0;
  for (uint32_t a = 0; a < n; ++a) {
    uint64_t pages = range_pages(&ranges[a], unit);
    for (uint64_t p = 0; p < pages; ++p, ++g) {
      const uint8_t *page = host_ptr[a] + p * unit;
      uint64_t len = page_len(&ranges[a], p, unit);
      hash[g] = kco_xxh64(page, len, seed);
      if (page_is_zero(page, len)) bit_set(zero_bm, g);
      if (prior && hash[g] != prior[g]) bit_set(changed_bm, g);
    }
  }
  return KCO_OK;
}

int kco_page_hash(const kco_range *ranges, const uint8_t *const *host_ptr,
                  uint32_t n, uint64_t seed, const uint64_t *prior,
                  uint64_t *hash, uint64_t *zero_bm, uint64_t *changed_bm) {
  return kco_page_hash_unit(ranges, host_ptr, n, PAGE, seed, prior, hash, zero_bm, changed_bm);
}

/* ------------------------------------------------------------------------ */
/* Snapshot: compaction of the kept pages, ascending g                       */
/* ------------------------------------------------------------------------ */

int kco_compact_unit(const kco_range *ranges, const uint8_t *const *host_ptr,
                     uint32_t n, uint64_t unit, const uint64_t *zero_bm,
                     const uint64_t *changed_bm, uint8_t *packed, uint64_t *page_va,
                     uint64_t cap_pages, uint64_t *n_kept) {
  uint64_t n_pages = 0;
  int st = kco_range_check_unit(ranges, n, unit, NULL, &n_pages);
  if (st != KCO_OK) return st;
  if (n_kept == NULL || (n_pages > 0 && zero_bm == NULL)) return KCO_EINVAL;
  if (cap_pages > 0 && (packed == NULL || page_va == NULL)) return KCO_EINVAL;
  uint64_t g = 0, slot = 0;
  for (uint32_t a = 0; a < n; ++a) {
    uint64_t pages = range_pages(&ranges[a], unit);
    for (uint64_t p = 0; p < pages; ++p, ++g) {
      int keep = !bit_get(zero_bm, g);
      if (changed_bm != NULL) keep = keep && bit_get(changed_bm, g);
      if (!keep) continue;
      if (slot < cap_pages) { /* a partial unit is followed by zeros in its slot */
        uint64_t len = page_len(&ranges[a], p, unit);
        memcpy(packed + slot * unit, host_ptr[a] + p * unit, len);
        memset(packed + slot * unit + len, 0, unit - len);
        page_va[slot] = ranges[a].base + p * unit;
      }
      ++slot;
    }
  }
  *n_kept = slot;
  return KCO_OK;
}

int kco_compact(const kco_range *ranges, const uint8_t *const *host_ptr,
                uint32_t n, const uint64_t *zero_bm, const uint64_t *changed_bm,
                uint8_t *packed, uint64_t *page_va, uint64_t cap_pages,
                uint64_t *n_kept) {
  return kco_compact_unit(ranges, host_ptr, n, PAGE, zero_bm, changed_bm, packed, page_va,
                          cap_pages, n_kept);
}

/* ------------------------------------------------------------------------ */
/* Restore at the original VAs                                               */
/* ------------------------------------------------------------------------ */

/* Index of the range holding address va, or -1. */
static int64_t find_range(const kco_range *ranges, uint32_t n, uint64_t va) {
  uint32_t lo = 0, hi = n; /* search in [lo, hi) for last base <= va */
  if (n == 0 || va < ranges[0].base) return -1;
  while (hi - lo > 1) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (ranges[mid].base <= va)
      lo = mid;
    else
      hi = mid;
  }
  if (va - ranges[lo].base < ranges[lo].size) return (int64_t)lo;
  return -1;
}

int kco_restore_unit(const kco_range *ranges, uint8_t *const *host_ptr, uint32_t n,
                     uint64_t unit, const uint64_t *zero_bm, const uint64_t *changed_bm,
                     const uint8_t *packed, const uint64_t *page_va,
                     uint64_t n_kept, uint64_t cap_pages, uint64_t *n_bad) {
  uint64_t n_pages = 0;
  int st = kco_range_check_unit(ranges, n, unit, NULL, &n_pages);
  if (st != KCO_OK) return st;
  if (n_pages > 0 && zero_bm == NULL) return KCO_EINVAL;
  uint64_t n_copy = n_kept < cap_pages ? n_kept : cap_pages;
  if (n_copy > 0 && (packed == NULL || page_va == NULL)) return KCO_EINVAL;
  /* 1. zero-fill the selected zero pages */
  uint64_t g = 0;
  for (uint32_t a = 0; a < n; ++a) {
    uint64_t pages = range_pages(&ranges[a], unit);
    for (uint64_t p = 0; p < pages; ++p, ++g) {
      int selected = changed_bm == NULL || bit_get(changed_bm, g);
      if (selected && bit_get(zero_bm, g))
        memset(host_ptr[a] + p * unit, 0, page_len(&ranges[a], p, unit));
    }
  }
  /* 2. scatter every packed unit back to the VA the page table names: the
   * start of a unit of some range */
  uint64_t bad = 0;
  for (uint64_t s = 0; s < n_copy; ++s) {
    uint64_t va = page_va[s];
    int64_t a = find_range(ranges, n, va);
    if (a < 0 || (va - ranges[a].base) % unit != 0) {
      ++bad;
      continue;
    }
    uint64_t p = (va - ranges[a].base) / unit; /* only the unit's own bytes are written */
    memcpy(host_ptr[a] + p * unit, packed + s * unit, page_len(&ranges[a], p, unit));
  }
  if (n_bad) *n_bad = bad;
  return KCO_OK;
}

int kco_restore(const kco_range *ranges, uint8_t *const *host_ptr, uint32_t n,
                const uint64_t *zero_bm, const uint64_t *changed_bm,
                const uint8_t *packed, const uint64_t *page_va,
                uint64_t n_kept, uint64_t cap_pages, uint64_t *n_bad) {
  return kco_restore_unit(ranges, host_ptr, n, PAGE, zero_bm, changed_bm, packed, page_va,
                          n_kept, cap_pages, n_bad);
}

/* ------------------------------------------------------------------------ */
/* Closure scan                                                              */
/* ------------------------------------------------------------------------ */

int kco_closure_scan(const kco_range *ranges, const uint8_t *const *host_ptr,
                     uint32_t n, uint64_t win_lo, uint64_t win_hi,
                     kco_scan_result *res, kco_oob *oob, uint64_t oob_cap) {
  uint64_t n_pages = 0;
  int st = kco_range_check(ranges, n, NULL, &n_pages);
  if (st != KCO_OK) return st;
  if (res == NULL || (oob_cap > 0 && oob == NULL)) return KCO_EINVAL;
  if (win_lo == 0 && win_hi == 0)
    kco_default_window(ranges, n, &win_lo, &win_hi);
  else if (win_lo == 0 || win_lo >= win_hi)
    return KCO_EINVAL;
  memset(res, 0, sizeof(*res));
  for (uint32_t a = 0; a < n; ++a) {
    for (uint64_t off = 0; off + 8 <= ranges[a].size; off += 8) { /* words wholly inside */
      uint64_t w = read_u64_le(host_ptr[a] + off);
      res->n_words += 1;
      if (w < win_lo || w >= win_hi) continue;
      res->n_ptr_like += 1;
      if (find_range(ranges, n, w) >= 0) {
        res->n_in_range += 1;
      } else {
        if (res->n_oob < oob_cap) {
          oob[res->n_oob].word_va = ranges[a].base + off;
          oob[res->n_oob].value = w;
        }
        res->n_oob += 1;
      }
    }
  }
  res->n_written = (uint32_t)(res->n_oob < oob_cap ? res->n_oob : oob_cap);
  res->truncated = res->n_oob > oob_cap ? 1u : 0u;
  return KCO_OK;
}

int kco_closure_scan_range(const kco_range *ranges, uint32_t n, uint32_t a,
                           const uint8_t *host, uint64_t win_lo, uint64_t win_hi,
                           kco_scan_result *res, kco_oob *oob, uint64_t oob_cap) {
  uint64_t n_pages = 0;
  int st = kco_range_check(ranges, n, NULL, &n_pages);
  if (st != KCO_OK) return st;
  if (a >= n || host == NULL || res == NULL || (oob_cap > 0 && oob == NULL))
    return KCO_EINVAL;
  if (win_lo == 0 && win_hi == 0)
    kco_default_window(ranges, n, &win_lo, &win_hi);
  else if (win_lo == 0 || win_lo >= win_hi)
    return KCO_EINVAL;
  memset(res, 0, sizeof(*res));
  /* the words of range a only, each tested against every range */
  for (uint64_t off = 0; off + 8 <= ranges[a].size; off += 8) {
    uint64_t w = read_u64_le(host + off);
    res->n_words += 1;
    if (w < win_lo || w >= win_hi) continue;
    res->n_ptr_like += 1;
    if (find_range(ranges, n, w) >= 0) {
      res->n_in_range += 1;
    } else {
      if (res->n_oob < oob_cap) {
        oob[res->n_oob].word_va = ranges[a].base + off;
        oob[res->n_oob].value = w;
      }
      res->n_oob += 1;
    }
  }
  res->n_written = (uint32_t)(res->n_oob < oob_cap ? res->n_oob : oob_cap);
  res->truncated = res->n_oob > oob_cap ? 1u : 0u;
  return KCO_OK;
}

/* ------------------------------------------------------------------------ */
/* Typed compare                                                             */
/* ------------------------------------------------------------------------ */

static uint32_t elem_size(uint32_t dtype) {
  switch (dtype) {
    case KCO_F64: case KCO_I64: return 8;
    case KCO_F32: case KCO_I32: return 4;
    case KCO_BF16: case KCO_F16: case KCO_I16: return 2;
    case KCO_FP8_E4M3FN: case KCO_FP8_E4M3FNUZ: case KCO_FP8_E5M2:
    case KCO_FP8_E5M2FNUZ: case KCO_I8: case KCO_U8: return 1;
    default: return 0;
  }
}

static int is_int_type(uint32_t dtype) {
  return dtype == KCO_I8 || dtype == KCO_I16 || dtype == KCO_I32 || dtype == KCO_I64;
}

static uint64_t read_elem_bits(const uint8_t *p, uint32_t size) {
  uint64_t v = 0;
  for (int i = (int)size - 1; i >= 0; --i) v = (v << 8) | (uint64_t)p[i];
  return v;
}

/* Floating formats: the sign bit is the top bit of the element, the
 * magnitude is the rest. */
static uint64_t sign_bit(uint32_t dtype) {
  return 1ULL << (8u * elem_size(dtype) - 1u);
}

static int is_nan_bits(uint32_t dtype, uint64_t bits) {
  uint64_t mag = bits & (sign_bit(dtype) - 1u);
  switch (dtype) {
    case KCO_F64: return mag > 0x7FF0000000000000ULL;
    case KCO_F32: return mag > 0x7F800000u;
    case KCO_BF16: return mag > 0x7F80u;
    case KCO_F16: return mag > 0x7C00u;
    case KCO_FP8_E4M3FN: return mag == 0x7Fu;
    case KCO_FP8_E5M2: return mag > 0x7Cu;
    case KCO_FP8_E4M3FNUZ: case KCO_FP8_E5M2FNUZ: return bits == 0x80u;
    default: return 0; /* integers */
  }
}

/* Value of a small binary format with exponent field e (ebits wide),
 * mantissa field m (mbits wide) and the given bias: subnormal when e == 0. */
static double small_float(uint32_t e, uint32_t m, int mbits, int bias) {
  if (e == 0) return ldexp((double)m, 1 - bias - mbits);
  return ldexp((double)(m | (1u << mbits)), (int)e - bias - mbits);
}

static double decode_value(uint32_t dtype, uint64_t bits) {
  if (is_int_type(dtype)) {
    uint32_t nb = 8u * elem_size(dtype);
    int64_t v = (nb < 64 && (bits >> (nb - 1)) & 1u) ? (int64_t)(bits | (~0ULL << nb)) : (int64_t)bits;
    return (double)v;
  }
  if (dtype == KCO_F64) {
    double d;
    memcpy(&d, &bits, sizeof d); /* the host's own binary64 */
    return d;
  }
  uint64_t mag = bits & (sign_bit(dtype) - 1u);
  int negative = (bits & sign_bit(dtype)) != 0;
  double v;
  if (dtype == KCO_F32 || dtype == KCO_BF16) {
    /* bf16 is the upper half of an fp32 encoding */
    uint32_t f32 = dtype == KCO_F32 ? (uint32_t)mag : (uint32_t)(mag << 16);
    uint32_t e = f32 >> 23, m = f32 & 0x7FFFFFu;
    v = e == 255 ? INFINITY /* NaN never reaches decode */ : small_float(e, m, 23, 127);
  } else if (dtype == KCO_F16) {
    uint32_t e = (uint32_t)mag >> 10, m = (uint32_t)mag & 0x3FFu;
    v = e == 31 ? INFINITY : small_float(e, m, 10, 15);
  } else if (dtype == KCO_FP8_E5M2) {
    uint32_t e = (uint32_t)mag >> 2, m = (uint32_t)mag & 0x3u;
    v = e == 31 ? INFINITY : small_float(e, m, 2, 15);
  } else if (dtype == KCO_FP8_E5M2FNUZ) { /* every exponent is finite */
    v = small_float((uint32_t)mag >> 2, (uint32_t)mag & 0x3u, 2, 16);
  } else if (dtype == KCO_FP8_E4M3FNUZ) {
    v = small_float((uint32_t)mag >> 3, (uint32_t)mag & 0x7u, 3, 8);
  } else { /* OCP fp8 e4m3fn: bias 7, no infinities */
    v = small_float((uint32_t)mag >> 3, (uint32_t)mag & 0x7u, 3, 7);
  }
  return negative ? -v : v;
}

static int is_inf_value(uint32_t dtype, double v) {
  return !is_int_type(dtype) && isinf(v);
}

int kco_ulp(uint32_t dtype, uint64_t cand_bits, uint64_t gold_bits,
            uint64_t *dist) {
  uint32_t es = elem_size(dtype);
  if (es == 0 || dtype == KCO_U8) return KCO_EDTYPE;
  if (is_int_type(dtype)) {
    /* sign-extend, then the exact difference (it fits in 64 unsigned bits) */
    uint32_t nb = 8u * es;
    uint64_t c = cand_bits, g = gold_bits;
    if (nb < 64) {
      if ((c >> (nb - 1)) & 1u) c |= ~0ULL << nb;
      if ((g >> (nb - 1)) & 1u) g |= ~0ULL << nb;
    }
    int64_t ci = (int64_t)c, gi = (int64_t)g;
    *dist = ci >= gi ? c - g : g - c; /* modulo 2^64, exact since < 2^64 */
    return KCO_OK;
  }
  /* floats: position in sign-magnitude order; +0 and -0 coincide */
  uint64_t sb = sign_bit(dtype), mm = sb - 1u;
  uint64_t mc = cand_bits & mm, mg = gold_bits & mm;
  int sc = (cand_bits & sb) != 0, sg = (gold_bits & sb) != 0;
  if (sc == sg)
    *dist = mc > mg ? mc - mg : mg - mc;
  else
    *dist = mc + mg; /* through zero: each magnitude is below 2^63 */
  return KCO_OK;
}

uint32_t kco_ulp_bin(uint64_t dist) {
  if (dist <= 16) return (uint32_t)dist;
  uint32_t k = 0; /* smallest k with 2^k >= dist */
  while (k < 64 && (1ULL << k) < dist) ++k;
  return 12u + k < 47u ? 12u + k : 47u;
}

int kco_compare(const void *cand, const void *gold, uint64_t n_elems,
                uint32_t dtype, uint32_t ulp_tol, double atol, double rtol,
                kco_cmp_result *res) {
  if (res == NULL) return KCO_EINVAL;
  uint32_t es = elem_size(dtype);
  if (es == 0) return KCO_EDTYPE;
  if (!(atol >= 0.0) || !(rtol >= 0.0)) return KCO_EINVAL;
  if (n_elems > 0 && (cand == NULL || gold == NULL)) return KCO_EINVAL;
  memset(res, 0, sizeof(*res));
  res->n_elems = n_elems;
  res->first_mismatch = UINT64_MAX;
  const uint8_t *cb = (const uint8_t *)cand, *gb = (const uint8_t *)gold;
  for (uint64_t i = 0; i < n_elems; ++i) {
    const uint8_t *pc = cb + i * es, *pg = gb + i * es;
    uint64_t c = read_elem_bits(pc, es), g = read_elem_bits(pg, es);
    if (c != g) {
      res->n_mismatch_elems += 1;
      if (res->first_mismatch == UINT64_MAX) res->first_mismatch = i;
      for (uint32_t b = 0; b < es; ++b)
        if (pc[b] != pg[b]) res->n_mismatch_bytes += 1;
    }
    if (dtype == KCO_U8) continue;
    int nan_c = is_nan_bits(dtype, c), nan_g = is_nan_bits(dtype, g);
    if (nan_c && nan_g) {
      res->n_nan_both += 1;
      continue;
    }
    if (nan_c) {
      res->n_nan_cand_only += 1;
      continue;
    }
    if (nan_g) {
      res->n_nan_gold_only += 1;
      continue;
    }
    uint64_t d = 0;
    kco_ulp(dtype, c, g, &d);
    res->ulp_hist[kco_ulp_bin(d)] += 1;
    if (d > ulp_tol) res->n_over_tol += 1;
    if (c == g) continue; /* identical encodings: abs 0, rel 0 */
    double vc = decode_value(dtype, c), vg = decode_value(dtype, g);
    double abs_err;
    if (is_int_type(dtype))
      abs_err = (double)d; /* exact difference, one rounding */
    else
      abs_err = fabs(vc - vg);
    if (abs_err > res->max_abs) res->max_abs = abs_err;
    if (vg != 0.0 && !is_inf_value(dtype, vg)) {
      double rel = abs_err / fabs(vg);
      if (rel > res->max_rel) res->max_rel = rel;
    }
    int close;
    if (is_inf_value(dtype, vc) || is_inf_value(dtype, vg))
      close = vc == vg;
    else
      close = abs_err <= atol + rtol * fabs(vg);
    if (!close) res->n_not_close += 1;
  }
  if (dtype == KCO_U8) {
    res->pass = res->n_mismatch_elems == 0;
    res->pass_close = res->pass;
  } else {
    res->pass = res->n_over_tol == 0 && res->n_nan_cand_only == 0 &&
                res->n_nan_gold_only == 0;
    res->pass_close = res->n_not_close == 0 && res->n_nan_cand_only == 0 &&
                      res->n_nan_gold_only == 0;
  }
  res->status = 0;
  return KCO_OK;
}

/* ------------------------------------------------------------------------ */
/* Pointer graph between ranges and the reachable set                        */
/* ------------------------------------------------------------------------ */

static uint64_t graph_row_words(uint32_t n) { return ((uint64_t)n + 63u) / 64u; }

int kco_pointer_graph(const kco_range *ranges, const uint8_t *const *host_ptr,
                      uint32_t n, uint64_t win_lo, uint64_t win_hi,
                      uint64_t *edge_bm) {
  uint64_t n_pages = 0;
  int st = kco_range_check(ranges, n, NULL, &n_pages);
  if (st != KCO_OK) return st;
  if (n > 0 && edge_bm == NULL) return KCO_EINVAL;
  if (win_lo == 0 && win_hi == 0)
    kco_default_window(ranges, n, &win_lo, &win_hi);
  else if (win_lo == 0 || win_lo >= win_hi)
    return KCO_EINVAL;
  uint64_t rw = graph_row_words(n);
  memset(edge_bm, 0, (size_t)(n * rw) * sizeof(uint64_t));
  for (uint32_t a = 0; a < n; ++a) {
    for (uint64_t off = 0; off + 8 <= ranges[a].size; off += 8) { /* words wholly inside */
      uint64_t w = read_u64_le(host_ptr[a] + off);
      if (!(w >= win_lo && w < win_hi)) continue; /* not pointer-like */
      int64_t b = find_range(ranges, n, w);
      if (b >= 0) bit_set(edge_bm + (uint64_t)a * rw, (uint64_t)b);
    }
  }
  return KCO_OK;
}

int kco_graph_reach(const kco_range *ranges, uint32_t n, const uint64_t *edge_bm,
                    const uint64_t *root_words, uint64_t n_root_words,
                    uint64_t *reach_bm) {
  uint64_t n_pages = 0;
  int st = kco_range_check(ranges, n, NULL, &n_pages);
  if (st != KCO_OK) return st;
  if ((n > 0 && (edge_bm == NULL || reach_bm == NULL)) || (n_root_words > 0 && root_words == NULL))
    return KCO_EINVAL;
  uint64_t rw = graph_row_words(n);
  memset(reach_bm, 0, (size_t)rw * sizeof(uint64_t));
  uint32_t *queue = (uint32_t *)malloc(((size_t)n + 1u) * sizeof(uint32_t));
  if (queue == NULL) return KCO_ENOMEM;
  uint32_t head = 0, tail = 0;
  /* the roots: every range that some root word points into */
  for (uint64_t i = 0; i < n_root_words; ++i) {
    int64_t r = find_range(ranges, n, root_words[i]);
    if (r >= 0 && !bit_get(reach_bm, (uint64_t)r)) {
      bit_set(reach_bm, (uint64_t)r);
      queue[tail++] = (uint32_t)r;
    }
  }
  /* breadth-first over the edges */
  while (head < tail) {
    uint32_t a = queue[head++];
    for (uint32_t b = 0; b < n; ++b) {
      if (bit_get(edge_bm + (uint64_t)a * rw, b) && !bit_get(reach_bm, b)) {
        bit_set(reach_bm, b);
        queue[tail++] = b;
      }
    }
  }
  free(queue);
  return KCO_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-range byte difference against a full snapshot                         */
/* ------------------------------------------------------------------------ */

int kco_region_diff_unit(const kco_range *ranges, const uint8_t *const *host_ptr,
                         uint32_t n, uint64_t unit, const uint64_t *gold_zero_bm,
                         const uint8_t *gold_packed, const uint64_t *gold_page_va,
                         uint64_t gold_n_kept, uint64_t cap_pages,
                         kco_region_diff_result *res) {
  uint64_t n_pages = 0;
  int st = kco_range_check_unit(ranges, n, unit, NULL, &n_pages);
  if (st != KCO_OK) return st;
  if (n > 0 && res == NULL) return KCO_EINVAL;
  if (n_pages > 0 && gold_zero_bm == NULL) return KCO_EINVAL;
  uint64_t n_valid = gold_n_kept < cap_pages ? gold_n_kept : cap_pages;
  if (n_valid > 0 && (gold_packed == NULL || gold_page_va == NULL)) return KCO_EINVAL;
  uint64_t g = 0, slot = 0; /* slot = non-zero units seen so far */
  for (uint32_t a = 0; a < n; ++a) {
    res[a].n_diff_bytes = 0;
    res[a].n_diff_pages = 0;
    res[a].first_diff_va = UINT64_MAX;
    res[a].n_bad_pages = 0;
    uint64_t pages = range_pages(&ranges[a], unit);
    for (uint64_t p = 0; p < pages; ++p, ++g) {
      uint64_t va = ranges[a].base + p * unit;
      uint64_t len = page_len(&ranges[a], p, unit);
      const uint8_t *gold = NULL; /* NULL: the golden unit is all zeros */
      if (!bit_get(gold_zero_bm, g)) {
        uint64_t s = slot++;
        if (s >= n_valid || gold_page_va[s] != va) {
          res[a].n_bad_pages += 1;
          continue;
        }
        gold = gold_packed + s * unit;
      }
      const uint8_t *live = host_ptr[a] + p * unit;
      uint64_t d = 0;
      for (uint64_t b = 0; b < len; ++b) {
        if (live[b] == (gold ? gold[b] : 0)) continue;
        if (res[a].first_diff_va == UINT64_MAX) res[a].first_diff_va = va + b;
        ++d;
      }
      res[a].n_diff_bytes += d;
      if (d > 0) res[a].n_diff_pages += 1;
    }
  }
  return KCO_OK;
}

int kco_region_diff(const kco_range *ranges, const uint8_t *const *host_ptr,
                    uint32_t n, const uint64_t *gold_zero_bm,
                    const uint8_t *gold_packed, const uint64_t *gold_page_va,
                    uint64_t gold_n_kept, uint64_t cap_pages,
                    kco_region_diff_result *res) {
  return kco_region_diff_unit(ranges, host_ptr, n, PAGE, gold_zero_bm, gold_packed, gold_page_va,
                              gold_n_kept, cap_pages, res);
}

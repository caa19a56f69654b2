/*
 * kco.h -- the CPU oracle for the snapshot / validation hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU leg of
 * the benchmark load the oracle.  It shares no code, header, table or
 * constant generator with the HIP library.
 *
 * Plain single-threaded C99, host pointers only, no SIMD, no threads.  Each
 * entry point computes the plain definition of one step of the method:
 *
 *   - the snapshot of every tracked allocation at its own virtual address,
 *     driven by the pointer-to-size map (paper Sec. 4.1.1 "Memory tracking",
 *     Sec. 4.2.1 snapshot of all tracked memory), here as a per-4-KiB-page
 *     XXH64 hash table, a zero-page bitmap, a changed-page bitmap against a
 *     prior hash table, and a packed snapshot of the kept pages with a
 *     page-VA table;
 *   - the restore of captured data into each region at the same virtual
 *     address (paper Sec. 4.5.1, replay stage 5; Sec. 4.2.1 address-space
 *     closure);
 *   - the closure scan: every 8-byte-aligned word that looks like a device
 *     pointer must land inside a captured range (paper Sec. 4.2.1,
 *     "Bounds of the closure", cases 1 and 3);
 *   - the output compare: differing bytes (paper Sec. 4.5.2, byte-exact
 *     comparison), and for floating-point buffers a ULP-distance report with
 *     explicit NaN accounting (paper Sec. 4.5.2, tolerance comparison).
 *
 * Conventions shared with the product ABI (same meaning, independent code):
 * a range is (base VA, size in bytes), base a multiple of 4096 and > 0,
 * size > 0, ranges sorted by base and disjoint.  A range spans
 * ceil(size / 4096) pages; when size is not a multiple of 4096 its last page
 * is partial and holds size mod 4096 bytes: its hash is the XXH64 of exactly
 * those bytes, its zero test looks at them only, its packed slot holds them
 * followed by zeros, a restore writes only them, and the closure scan reads
 * only 8-byte words that lie wholly inside the range.  Global page index g
 * numbers the pages of range 0 first, then range 1, ...  Bitmaps are arrays
 * of u64, bit (g % 64) of word (g / 64); bits past the last page are 0.
 *
 * The data of range a is read from / written to host_ptr[a] (a host copy of
 * the bytes that live at VA base_a on the device); VAs are only used as
 * values (page-VA table, pointer tests), never dereferenced.
 */
#ifndef KCO_H
#define KCO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KCO_OK = 0,
  KCO_EINVAL = -1, /* null pointer, empty range, zero base, bad window      */
  KCO_EALIGN = -2, /* base not a multiple of 4096                            */
  KCO_EORDER = -3, /* ranges unsorted or overlapping                        */
  KCO_ENOMEM = -4,
  KCO_EDTYPE = -6
};

/* Element types.  Floating formats: IEEE binary32 / binary16 / binary64,
 * bfloat16, OCP fp8 E4M3FN (bias 7, NaN = S.1111.111, no inf) and E5M2
 * (bias 15, IEEE-like inf / NaN), and the FNUZ fp8 variants E4M3FNUZ (bias 8)
 * and E5M2FNUZ (bias 16), whose only NaN is 0x80 and which have no -0 and no
 * inf.  Integers are two's complement, compared by their exact difference.
 * KCO_U8 is raw bytes (bitwise report only). */
enum {
  KCO_F32 = 0, KCO_BF16 = 1, KCO_F16 = 2, KCO_FP8_E4M3FN = 3, KCO_U8 = 4,
  KCO_F64 = 5, KCO_FP8_E4M3FNUZ = 6, KCO_FP8_E5M2 = 7, KCO_FP8_E5M2FNUZ = 8,
  KCO_I8 = 9, KCO_I16 = 10, KCO_I32 = 11, KCO_I64 = 12
};

typedef struct {
  uint64_t base, size;
} kco_range;

typedef struct {
  uint64_t n_words, n_ptr_like, n_in_range, n_oob;
  uint32_t n_written, truncated;
} kco_scan_result;

typedef struct {
  uint64_t word_va, value;
} kco_oob;

typedef struct {
  uint64_t n_elems, n_mismatch_elems, n_mismatch_bytes, first_mismatch;
  uint64_t n_nan_both, n_nan_cand_only, n_nan_gold_only, n_over_tol;
  double max_abs, max_rel;
  uint64_t ulp_hist[48];
  uint32_t pass, status;
  uint64_t n_not_close;
  uint32_t pass_close, reserved;
} kco_cmp_result;

typedef struct {
  uint64_t n_diff_bytes, n_diff_pages, first_diff_va, n_bad_pages;
} kco_region_diff_result;

/* XXH64 of len bytes at data with the given seed (public xxHash definition). */
uint64_t kco_xxh64(const void *data, uint64_t len, uint64_t seed);

/* Validate ranges; on success *n_pages = total pages and, if first_page is
 * non-null, first_page[0..n] = page prefix (first_page[n] = *n_pages). */
int kco_range_check(const kco_range *ranges, uint32_t n, uint64_t *first_page,
                    uint64_t *n_pages);

/* Hash units larger than the 4 KiB page (paper Sec. 4.2.1: whole-allocation
 * capture of large tensors, where a table entry per 4 KiB is more than a
 * snapshot needs).  The *_unit entry points below take the unit in bytes, a
 * power of two from 4096 to 2 MiB (else KCO_EINVAL), and mean by "page" one
 * unit: a range spans ceil(size / unit) units, unit p of range a starts at
 * base_a + p * unit (the base stays a multiple of 4096 only), its last unit
 * holds size mod unit bytes when that is not zero, packed slots are unit
 * bytes apart, and a restore accepts a page-table VA only if it is the start
 * of a unit of some range.  The entry points without the suffix are these
 * with unit = 4096. */
int kco_range_check_unit(const kco_range *ranges, uint32_t n, uint64_t unit,
                         uint64_t *first_page, uint64_t *n_pages);
int kco_page_hash_unit(const kco_range *ranges, const uint8_t *const *host_ptr,
                       uint32_t n, uint64_t unit, uint64_t seed, const uint64_t *prior,
                       uint64_t *hash, uint64_t *zero_bm, uint64_t *changed_bm);
int kco_compact_unit(const kco_range *ranges, const uint8_t *const *host_ptr,
                     uint32_t n, uint64_t unit, const uint64_t *zero_bm,
                     const uint64_t *changed_bm, uint8_t *packed, uint64_t *page_va,
                     uint64_t cap_pages, uint64_t *n_kept);
int kco_restore_unit(const kco_range *ranges, uint8_t *const *host_ptr, uint32_t n,
                     uint64_t unit, const uint64_t *zero_bm, const uint64_t *changed_bm,
                     const uint8_t *packed, const uint64_t *page_va,
                     uint64_t n_kept, uint64_t cap_pages, uint64_t *n_bad);
int kco_region_diff_unit(const kco_range *ranges, const uint8_t *const *host_ptr,
                         uint32_t n, uint64_t unit, const uint64_t *gold_zero_bm,
                         const uint8_t *gold_packed, const uint64_t *gold_page_va,
                         uint64_t gold_n_kept, uint64_t cap_pages,
                         kco_region_diff_result *res);

/* Pointer window used by the closure scan when the caller passes (0, 0). */
int kco_default_window(const kco_range *ranges, uint32_t n, uint64_t *lo,
                       uint64_t *hi);

/* hash[g], zero bitmap and (if prior != NULL) changed bitmap for every page. */
int kco_page_hash(const kco_range *ranges, const uint8_t *const *host_ptr,
                  uint32_t n, uint64_t seed, const uint64_t *prior,
                  uint64_t *hash, uint64_t *zero_bm, uint64_t *changed_bm);

/* Packed snapshot of kept pages (changed_bm == NULL: keep = not zero;
 * otherwise keep = changed and not zero), ascending g.  Pages past cap_pages
 * are not written; *n_kept is the true count. */
int kco_compact(const kco_range *ranges, const uint8_t *const *host_ptr,
                uint32_t n, const uint64_t *zero_bm, const uint64_t *changed_bm,
                uint8_t *packed, uint64_t *page_va, uint64_t cap_pages,
                uint64_t *n_kept);

/* Restore: zero-fill every selected zero page (all pages when changed_bm is
 * NULL, else the changed ones), then scatter packed[s] to page_va[s] for
 * s < min(n_kept, cap_pages).  A page_va that is not a page of some range is
 * skipped and counted in *n_bad. */
int kco_restore(const kco_range *ranges, uint8_t *const *host_ptr, uint32_t n,
                const uint64_t *zero_bm, const uint64_t *changed_bm,
                const uint8_t *packed, const uint64_t *page_va,
                uint64_t n_kept, uint64_t cap_pages, uint64_t *n_bad);

/* Closure scan over every 8-byte-aligned word of every range. */
int kco_closure_scan(const kco_range *ranges, const uint8_t *const *host_ptr,
                     uint32_t n, uint64_t win_lo, uint64_t win_hi,
                     kco_scan_result *res, kco_oob *oob, uint64_t oob_cap);

/* The closure scan of one range's words (range a, bytes at host), each word
 * tested against the whole range table with the same rules as
 * kco_closure_scan.  Summed over a = 0 .. n-1 the counts equal
 * kco_closure_scan's, and the lists, concatenated in range order, its list:
 * the form a scan of a pool too large for host memory takes, one range at a
 * time. */
int kco_closure_scan_range(const kco_range *ranges, uint32_t n, uint32_t a,
                           const uint8_t *host, uint64_t win_lo, uint64_t win_hi,
                           kco_scan_result *res, kco_oob *oob, uint64_t oob_cap);

/* Per-range byte difference between the live bytes of the ranges and a full
 * snapshot of the same ranges (byte-exact comparison reported per region,
 * paper Sec. 4.5.2).  The golden copy of page g is all zeros when its zero
 * bit is set; otherwise packed page s, s = number of non-zero pages before g
 * (the order kco_compact writes), accepted iff s < min(n_kept, cap_pages) and
 * page_va[s] is the VA of page g; a non-zero page without an accepted copy is
 * counted in n_bad_pages and not compared.  res[a] per range: differing
 * bytes, pages with at least one differing byte, VA of the first differing
 * byte (UINT64_MAX if none). */
int kco_region_diff(const kco_range *ranges, const uint8_t *const *host_ptr,
                    uint32_t n, const uint64_t *gold_zero_bm,
                    const uint8_t *gold_packed, const uint64_t *gold_page_va,
                    uint64_t gold_n_kept, uint64_t cap_pages,
                    kco_region_diff_result *res);

/* Pointer graph between ranges: edge_bm holds n rows of ceil(n / 64) u64
 * words; bit b of row a is set iff some 8-byte-aligned word of range a is
 * pointer-like (same window rule as kco_closure_scan) and lies inside range b.
 * This is the graph a pointer-chasing capture would follow (paper Sec. 4.2.1,
 * address-space closure, where the paper contrasts whole-memory capture with
 * chasing pointers). */
int kco_pointer_graph(const kco_range *ranges, const uint8_t *const *host_ptr,
                      uint32_t n, uint64_t win_lo, uint64_t win_hi,
                      uint64_t *edge_bm);

/* Ranges reachable from the root words (e.g. the kernel-argument words): the
 * ranges they point into, then everything reachable over edge_bm.  reach_bm
 * holds ceil(n / 64) u64 words, bit r = range r reached. */
int kco_graph_reach(const kco_range *ranges, uint32_t n, const uint64_t *edge_bm,
                    const uint64_t *root_words, uint64_t n_root_words,
                    uint64_t *reach_bm);

/* Typed compare of one candidate / golden pair of n_elems elements.  Besides
 * the ULP report, an element pair (neither NaN) is close iff
 * |c - g| <= atol + rtol * |g| in fp64, an infinity being close only to an
 * equal value (tolerance comparison with atol / rtol, paper Sec. 4.5.2).
 * For integers |c - g| is the exact difference rounded once to fp64.
 * Histogram bins: d for d <= 16, else min(12 + ceil(log2 d), 47). */
int kco_compare(const void *cand, const void *gold, uint64_t n_elems,
                uint32_t dtype, uint32_t ulp_tol, double atol, double rtol,
                kco_cmp_result *res);

/* ULP distance (floats: steps between the encodings in sign-magnitude order;
 * integers: |c - g| exactly) and histogram bin of one element pair (exposed
 * for tests).  Bits are the element's little-endian encoding, zero-extended. */
int kco_ulp(uint32_t dtype, uint64_t cand_bits, uint64_t gold_bits,
            uint64_t *dist);
uint32_t kco_ulp_bin(uint64_t dist);

#ifdef __cplusplus
}
#endif
#endif

/*
 * kc.h -- C ABI of libkc.so, the MI355X (gfx950) snapshot / validation hot
 * path behind VA-faithful kernel capture and reproducer validation.
 *
 * The method (Kerncap, arXiv 2605.03208) snapshots every tracked device
 * allocation at its original virtual address so that pointers embedded in
 * device memory stay valid on replay (Sec. 4.2.1, "address-space closure"),
 * restores that state before re-dispatch (Sec. 4.5.1, replay stage 5), and
 * validates a variant's outputs against the captured ones (Sec. 4.5.2).  This
 * library is the data-parallel core of those steps, done on the GPU:
 *
 *   kc_page_hash     XXH64 per 4 KiB page, zero-page and changed-page bitmaps
 *   kc_compact       prefix-scan compaction of kept pages + page-VA table
 *   kc_snapshot      the two above fused into one pass over the data
 *   kc_restore       zero-fill + scatter of packed pages back to their VAs
 *   kc_closure_scan  every aligned u64 that looks like a pointer must land
 *                    inside a captured range
 *   kc_compare       candidate vs golden: byte / element mismatches, first
 *                    mismatch, fp64 max abs / rel error, ULP histogram, NaNs
 *   kc_region_diff   per-range differing bytes of live memory against a
 *                    snapshot, comparing only pages whose hash changed
 *   kc_vaspace_*     device memory mapped at exactly the captured VAs in a
 *                    fresh process, for a VA-faithful restore
 *   kc_pointer_graph which range points into which (the graph pointer
 *                    chasing would follow), and kc_graph_reach, the ranges
 *                    reachable from the kernel-argument words
 *   kc_perturb       the validation server's candidates: goldens moved by a
 *                    seeded perturbation, in place on the device
 *   kc_materialize   the same candidates copied and moved in one pass
 *
 * Conventions
 *  - Pointers suffixed _d are device pointers owned by the caller; the
 *    library never frees caller memory.  Host pointers are read during the
 *    call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls enqueue work and return; outputs are valid once the stream has
 *    reached that point.  Apart from the *_create calls and kc_compare, a
 *    call allocates nothing and never synchronises, so a sequence of
 *    kc_snapshot / kc_restore / kc_closure_scan / kc_compare_pairset calls
 *    can be recorded into a HIP graph and replayed.
 *  - The return value reports synchronous argument checks and launch
 *    failures only.  Conditions found on the device (capacity overflow,
 *    truncated lists, rejected page addresses) are reported through outputs.
 *  - A kc_ctx, and any kc_rangeset made from it, is used by one host thread
 *    and one stream at a time: rangesets own the scratch their calls use.
 *  - Ranges: (base VA, size) with base > 0 a multiple of 4096, size > 0 any
 *    number of bytes, sorted by base, disjoint.  They are the pointer-to-size
 *    map of tracked allocations (Sec. 4.1.1, memory tracking).  A range spans
 *    ceil(size / 4096) pages; page g of the set numbers the pages of range 0
 *    first, then range 1, and so on.  When size is not a multiple of 4096 the
 *    range's last page is partial: only its size mod 4096 bytes belong to
 *    the range.  They alone are hashed (XXH64 of that many bytes), zero-tested
 *    and compared; its packed slot holds them followed by zeros; a restore
 *    writes them and nothing past the range's end; the closure scan and the
 *    pointer graph read only 8-byte words wholly inside the range.  Loads may
 *    touch up to 15 bytes past a range's end inside its last page (the page
 *    is mapped: device memory is mapped in whole pages); nothing is written
 *    there.
 *  - Bitmaps: u64 words, page g is bit (g % 64) of word (g / 64); a bitmap
 *    over N pages has ceil(N / 64) words and its bits past N are 0.
 *  - Limits: fewer than 2^32 pages per rangeset, fewer than 2^31 ranges.
 */
#ifndef KC_H
#define KC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KC_PAGE_SIZE 4096u
#define KC_ABI_VERSION 7
#define KC_GRAPH_MAX_RANGES 16384u /* kc_pointer_graph: at most 32 MiB of edges */
#define KC_NOALLOC_MAX_PAIRS 4096u /* kc_compare_noalloc: pairs per call (2 MiB of static scratch) */

/* Status codes. */
enum {
  KC_OK = 0,
  KC_EINVAL = -1,  /* null where non-null is required, empty range, base 0,
                      bad window, size overflow                            */
  KC_EALIGN = -2,  /* range base not 4096-aligned / buffer not aligned to its element size */
  KC_EORDER = -3,  /* ranges unsorted or overlapping                       */
  KC_ENOMEM = -4,  /* device or pinned host allocation failed             */
  KC_EHIP = -5,    /* a HIP runtime call failed; see kc_last_error()       */
  KC_EDTYPE = -6,  /* unknown element type                                 */
  KC_ELIMIT = -7,  /* a documented size limit is exceeded                  */
  KC_ERELOC = -8   /* an address range could not be placed at its VA       */
};

/* Element types understood by kc_compare.  Floating types get the ULP
 * distance (steps between the two encodings in sign-magnitude order, +0 and
 * -0 coinciding) and NaN classes; integer types get the exact difference
 * |c - g| as their distance and have no NaN; KC_U8 is compared bytewise only. */
enum {
  KC_F32 = 0,            /* IEEE binary32                                     */
  KC_BF16 = 1,           /* bfloat16 (upper half of binary32)                 */
  KC_F16 = 2,            /* IEEE binary16                                     */
  KC_FP8_E4M3FN = 3,     /* OCP fp8 E4M3: bias 7, no inf, NaN = S.1111.111    */
  KC_U8 = 4,             /* raw bytes                                         */
  KC_F64 = 5,            /* IEEE binary64                                     */
  KC_FP8_E4M3FNUZ = 6,   /* fp8 E4M3 FNUZ: bias 8, no inf, no -0, NaN = 0x80  */
  KC_FP8_E5M2 = 7,       /* OCP fp8 E5M2: bias 15, IEEE-style inf and NaN     */
  KC_FP8_E5M2FNUZ = 8,   /* fp8 E5M2 FNUZ: bias 16, no inf, no -0, NaN = 0x80 */
  KC_I8 = 9,             /* two's complement integers                         */
  KC_I16 = 10,
  KC_I32 = 11,
  KC_I64 = 12
};

typedef struct kc_ctx kc_ctx;
typedef struct kc_rangeset kc_rangeset;
typedef struct kc_pairset kc_pairset;
typedef struct kc_vaspace kc_vaspace;

typedef struct {
  uint64_t base; /* device VA of the allocation */
  uint64_t size; /* bytes                       */
} kc_range;

/* Closure-scan totals. */
typedef struct {
  uint64_t n_words;    /* aligned u64 words scanned                           */
  uint64_t n_ptr_like; /* words inside the pointer window                     */
  uint64_t n_in_range; /* pointer-like words inside some range                */
  uint64_t n_oob;      /* pointer-like words outside every range (exact)      */
  uint32_t n_written;  /* min(n_oob, oob_cap) entries written to the list     */
  uint32_t truncated;  /* 1 iff n_oob > oob_cap                               */
} kc_scan_result;

/* One out-of-range pointer-like word: where it sits and what it holds. */
typedef struct {
  uint64_t word_va;
  uint64_t value;
} kc_oob;

/* Closure-scan arguments.  A word w is pointer-like iff win_lo <= w < win_hi;
 * (0, 0) selects [min_base - 4 GiB, max_end + 4 GiB) clamped to [4096, 2^64-1].
 * Otherwise 1 <= win_lo < win_hi is required (a null word is never a pointer).
 * The list holds the first min(n_oob, oob_cap) words in ascending address. */
typedef struct {
  uint64_t win_lo, win_hi;
  kc_scan_result *res_d; /* device, one struct                          */
  kc_oob *oob_d;         /* device, oob_cap entries (may be NULL if 0)  */
  uint64_t oob_cap;
} kc_scan_args;

/* One candidate / golden pair for kc_compare.  Both buffers device memory of
 * n_elems elements of `dtype`, each aligned to the element size (else
 * KC_EALIGN).  Pairs whose buffers are both 16-byte aligned stream 16-byte
 * runs; others (views at odd element offsets) are read element by element,
 * with the same results. */
typedef struct {
  const void *cand_d;
  const void *gold_d;
  uint64_t n_elems;
  uint32_t dtype;
  uint32_t ulp_tol; /* an element fails if its ULP distance exceeds this   */
  double atol;      /* tolerance comparison (Sec. 4.5.2): an element is     */
  double rtol;      /* close iff |c - g| <= atol + rtol * |g| in fp64       */
} kc_pair;

/* Per-pair compare report (488 bytes). */
typedef struct {
  uint64_t n_elems;
  uint64_t n_mismatch_elems; /* elements whose encodings differ            */
  uint64_t n_mismatch_bytes; /* byte positions that differ                 */
  uint64_t first_mismatch;   /* lowest differing element, UINT64_MAX if none */
  uint64_t n_nan_both;       /* both NaN: passes, excluded from the rest   */
  uint64_t n_nan_cand_only;  /* fails, excluded from the rest              */
  uint64_t n_nan_gold_only;  /* fails, excluded from the rest              */
  uint64_t n_over_tol;       /* non-NaN elements with ULP distance > tol   */
  double max_abs;            /* max |c - g| in fp64 over non-NaN elements
                                (integers: exact difference, rounded once) */
  double max_rel;            /* max |c - g| / |g| over finite non-zero g   */
  uint64_t ulp_hist[48];     /* bin d for d <= 16, else
                                min(12 + ceil(log2 d), 47)                 */
  uint32_t pass;             /* no over-tolerance element and no lone NaN;
                                KC_U8: no differing byte                   */
  uint32_t status;           /* 0                                          */
  uint64_t n_not_close;      /* non-NaN elements failing the atol / rtol test
                                (an infinity is close only to itself)      */
  uint32_t pass_close;       /* no element failing it and no lone NaN;
                                KC_U8: no differing byte                   */
  uint32_t reserved;
} kc_cmp_result;

/* Per-range byte difference against a snapshot (32 bytes). */
typedef struct {
  uint64_t n_diff_bytes;  /* bytes that differ from the snapshot's copy        */
  uint64_t n_diff_pages;  /* pages with at least one differing byte            */
  uint64_t first_diff_va; /* VA of the lowest differing byte, UINT64_MAX if none */
  uint64_t n_bad_pages;   /* non-zero snapshot pages without an accepted copy:
                             not compared                                      */
} kc_region_diff_result;

/* Launch shape of one operation.  Zero fields keep the built-in choice. */
typedef struct {
  uint32_t grid_per_cu; /* persistent waves per compute unit (the compare:
                           four-wave workgroups per compute unit)           */
  uint32_t tile_bytes;  /* compare: bytes of each side per work item        */
  uint32_t per_item;    /* 1 = one launch per range / pair (no batching)    */
  uint32_t depth;       /* hashing pass without a fused scan: chunks in flight
                           per wave, 1 to 4; 2 to 4 select the pipelined,
                           skewed pass of units above 4 KiB; 0 = built-in
                           choice (2 above 4 KiB, else 1)                    */
} kc_tuning;

enum {
  KC_OP_PAGE_HASH = 0,
  KC_OP_SNAPSHOT = 1,
  KC_OP_COMPACT = 2,
  KC_OP_RESTORE = 3,
  KC_OP_CLOSURE = 4,
  KC_OP_COMPARE = 5,
  KC_OP_GRAPH = 6,
  KC_OP_REGION_DIFF = 7,
  KC_OP_COUNT = 8
};

/* ---- host-only helpers (no device needed) ---------------------------- */

/* Static text for a status code. */
const char *kc_strerror(int code);

/* Text of the last failure on this thread (HIP error name and call site). */
const char *kc_last_error(void);

/* KC_ABI_VERSION of the loaded library. */
int kc_abi_version(void);

/* Validate a range list as kc_rangeset_create does, without a device.
 * On KC_OK *n_pages (if non-NULL) is the page count. */
int kc_range_check(const kc_range *ranges, uint32_t n, uint64_t *n_pages);

/* The pointer window kc_closure_scan uses for (0, 0). */
int kc_default_window(const kc_range *ranges, uint32_t n, uint64_t *win_lo,
                      uint64_t *win_hi);

/* ---- context and range sets ------------------------------------------- */

/* Create a context on HIP device `hip_device` (made current for the call).
 * Owns launch tuning and the scratch of kc_compare. */
int kc_ctx_create(kc_ctx **out, int hip_device);
void kc_ctx_destroy(kc_ctx *ctx);

/* Set / read the launch shape of an operation (KC_OP_*). */
int kc_ctx_set_tuning(kc_ctx *ctx, uint32_t op, const kc_tuning *t);
int kc_ctx_get_tuning(const kc_ctx *ctx, uint32_t op, kc_tuning *t);

/* Kernel timing for measurement.  When on, each call records a pair of HIP
 * events on its stream around the launches of its main kernel (the hashing
 * pass of kc_page_hash / kc_snapshot, the gather of kc_compact, the scatter of
 * kc_restore, the scanning pass of kc_closure_scan, the compare pass of
 * kc_compare).  kc_ctx_kernel_ms waits for the last pair recorded for `op`
 * and returns the elapsed milliseconds (KC_EINVAL if none was recorded).
 * Off by default; leave it off while a stream is being captured. */
int kc_ctx_enable_timing(kc_ctx *ctx, int on);
int kc_ctx_kernel_ms(kc_ctx *ctx, uint32_t op, float *ms);

/* Upload a validated range list (the tracked-allocation map) and allocate
 * the scratch its calls need (about 40 bytes per page).  Synchronous.
 * Errors: KC_EINVAL / KC_EALIGN / KC_EORDER as kc_range_check, KC_ELIMIT,
 * KC_ENOMEM, KC_EHIP.  *n_pages (if non-NULL) receives the page count. */
int kc_rangeset_create(kc_ctx *ctx, const kc_range *ranges, uint32_t n,
                       kc_rangeset **out, uint64_t *n_pages);

/* The same with a hash unit larger than the 4 KiB page, for whole-allocation
 * capture of large tensors (Sec. 4.2.1: the snapshot covers whole tracked
 * allocations; a table entry per 4 KiB is more than such tensors need).
 * `unit` is a power of two from 4096 to 2 MiB (2097152), else KC_EINVAL.
 * Every call on the set then means by "page" one unit: a range spans
 * ceil(size / unit) units, unit p of range a starts at base_a + p * unit
 * (bases stay 4096-aligned only), a range's last unit holds size mod unit
 * bytes when that is not zero (hashed, zero-tested, packed and restored over
 * those bytes only; its packed slot is padded with zeros), hash tables,
 * bitmaps, page-VA tables and kept counts count units, packed slots are
 * `unit` bytes apart, a restore accepts a page-VA entry only if it is the
 * start of a unit of some range, snapshot files record the unit and load
 * only into a set of the same unit.  The closure scan and the pointer graph
 * are unchanged (they read every word); with a unit above 4096 a scan asked
 * of kc_page_hash / kc_snapshot runs as its own pass over the ranges after
 * the hashing pass (same results).  *n_units (if non-NULL) receives the unit
 * count.  kc_rangeset_create is this call with unit = 4096. */
int kc_rangeset_create_unit(kc_ctx *ctx, const kc_range *ranges, uint32_t n,
                            uint64_t unit, kc_rangeset **out, uint64_t *n_units);
void kc_rangeset_destroy(kc_rangeset *rs);

/* ---- snapshot (Sec. 4.2.1: snapshot of all tracked memory) ------------- */

/* Hash every page: hash_d[g] = XXH64(page g, seed) (the public xxHash
 * definition over the page's 4096 bytes).  zero_bm_d bit g = page g is all
 * zero.  If prior_hash_d is non-NULL, changed_bm_d (then required) bit g =
 * hash_d[g] != prior_hash_d[g].  If scan is non-NULL the closure scan runs in
 * the same pass over the data (same results as kc_closure_scan).
 * Sizes: hash_d / prior_hash_d N u64, bitmaps ceil(N/64) u64. */
int kc_page_hash(kc_ctx *ctx, const kc_rangeset *rs, uint64_t seed,
                 const uint64_t *prior_hash_d, uint64_t *hash_d,
                 uint64_t *zero_bm_d, uint64_t *changed_bm_d,
                 const kc_scan_args *scan, void *stream);

/* Compact the kept pages in ascending g: keep = not zero (changed_bm_d NULL)
 * or changed and not zero (delta).  packed_d[s*4096 ...] receives the page of
 * slot s and page_va_d[s] its VA, for s < cap_pages; *n_kept_d (device u64)
 * receives the exact kept count even when it exceeds cap_pages. */
int kc_compact(kc_ctx *ctx, const kc_rangeset *rs, const uint64_t *zero_bm_d,
               const uint64_t *changed_bm_d, void *packed_d,
               uint64_t *page_va_d, uint64_t cap_pages, uint64_t *n_kept_d,
               void *stream);

/* kc_page_hash followed by kc_compact with identical outputs.  Without a
 * prior (full snapshot) the data is read once: a probe of each page's first
 * 16 bytes (the whole page only when those are zero) fixes the zero bitmap
 * and the slots, then one pass hashes, scans and writes the packed pages.
 * With a prior (delta snapshot) the kept set depends on the hashes, so the
 * changed pages are read a second time. */
int kc_snapshot(kc_ctx *ctx, const kc_rangeset *rs, uint64_t seed,
                const uint64_t *prior_hash_d, uint64_t *hash_d,
                uint64_t *zero_bm_d, uint64_t *changed_bm_d, void *packed_d,
                uint64_t *page_va_d, uint64_t cap_pages, uint64_t *n_kept_d,
                const kc_scan_args *scan, void *stream);

/* ---- restore (Sec. 4.5.1, replay stage 5: copy captured data into each
 *      region at its original VA) ----------------------------------------- */

/* 1) zero-fill every selected zero page (all pages for a full snapshot,
 *    changed_bm_d NULL; the changed ones for a delta); then
 * 2) copy packed_d page s to page_va_d[s] for s < min(*n_kept_d, cap_pages).
 * A page_va that is not a 4096-aligned address inside some range is skipped
 * and counted into *n_bad_d (device u64, set by the call; may be NULL). */
int kc_restore(kc_ctx *ctx, const kc_rangeset *rs, const uint64_t *zero_bm_d,
               const uint64_t *changed_bm_d, const void *packed_d,
               const uint64_t *page_va_d, const uint64_t *n_kept_d,
               uint64_t cap_pages, uint64_t *n_bad_d, void *stream);

/* ---- address space of a replay (Sec. 4.5.1, replay stages 3-4: reserve each
 *      captured region at its original VA before anything else allocates,
 *      abort on relocation) ------------------------------------------------- */

/* Map device memory of `hip_device` at exactly the VAs of the ranges: each
 * range is covered by a span aligned to the device's recommended
 * virtual-memory granularity (touching spans merge), every span is reserved at its own
 * address, backed by device memory and made readable and writable.  If any
 * span cannot be reserved at its address, everything reserved so far is
 * released and KC_ERELOC is returned (the replay must not run relocated).
 * Contents are undefined until restored (kc_snapshot_load + kc_restore).
 * Call it before other device allocations of the process.  *n_spans and
 * *mapped_bytes (either may be NULL) report the spans. */
int kc_vaspace_create(int hip_device, const kc_range *ranges, uint32_t n,
                      kc_vaspace **out, uint32_t *n_spans,
                      uint64_t *mapped_bytes);

/* Unmap and release everything kc_vaspace_create mapped (NULL is a no-op). */
void kc_vaspace_destroy(kc_vaspace *vs);

/* An address at which `size` bytes (rounded up to the virtual-memory
 * granularity) could be reserved a moment ago, chosen away from the blocks the
 * runtime takes for itself: a trial reservation shows where free reservations
 * land; addresses 64 GiB, 128 GiB, ... below that are tried and the first one
 * granted exactly is returned (every trial is released again).  A capture
 * that maps its tracked memory there with kc_vaspace_create lets a replay
 * process, which maps the same ranges before anything else allocates, get the
 * same addresses. */
int kc_vaspace_suggest(int hip_device, uint64_t size, uint64_t *base);

/* ---- validation ----------------------------------------------------------- */

/* Per-range byte difference between the live bytes of the ranges and a full
 * snapshot of them (kc_snapshot output, changed_bm NULL), hash first (Sec.
 * 4.5.2, byte-exact comparison reported per region):
 * 1) the live pages are hashed with `seed` against gold_hash_d (which must be
 *    the snapshot's hash table, made with the same seed): cand_hash_d,
 *    cand_zero_bm_d and changed_bm_d receive the live hash table, zero bitmap
 *    and changed-page bitmap (each fully written);
 * 2) only changed pages are compared byte by byte with the snapshot's copy:
 *    all zeros when the page's gold zero bit is set, else packed page s,
 *    s = number of non-zero pages before it, accepted iff
 *    s < min(*gold_n_kept_d, cap_pages) and gold_page_va_d[s] is the page's VA.
 *    Non-zero pages without an accepted copy are counted in n_bad_pages
 *    (changed or not) and not compared.
 * res_d: device, one kc_region_diff_result per range, fully written.  Equal to a full
 * byte compare unless two different pages share an XXH64 hash.  Allocates
 * nothing, asynchronous on `stream`. */
int kc_region_diff(kc_ctx *ctx, const kc_rangeset *rs, uint64_t seed,
                   const uint64_t *gold_hash_d, const uint64_t *gold_zero_bm_d,
                   const void *gold_packed_d, const uint64_t *gold_page_va_d,
                   const uint64_t *gold_n_kept_d, uint64_t cap_pages,
                   uint64_t *cand_hash_d, uint64_t *cand_zero_bm_d,
                   uint64_t *changed_bm_d, kc_region_diff_result *res_d,
                   void *stream);

/* Pointer graph between ranges (Sec. 4.2.1: the paper captures all tracked
 * memory rather than chasing pointers; this is the graph such a chase would
 * follow, so that callers can capture the reachable ranges only).
 * edge_bm_d: device, n_ranges rows of ceil(n_ranges / 64) u64 words, every
 * word written by the call.  Bit b of row a is set iff some 8-byte-aligned
 * word of range a is pointer-like (win_lo / win_hi as in kc_scan_args,
 * (0, 0) = default window) and lies in range b (half-open).  Self edges are
 * kept.  More than KC_GRAPH_MAX_RANGES ranges: KC_ELIMIT.  Asynchronous on
 * `stream`, allocates nothing. */
int kc_pointer_graph(kc_ctx *ctx, const kc_rangeset *rs, uint64_t win_lo,
                     uint64_t win_hi, uint64_t *edge_bm_d, void *stream);

/* Host-only: the ranges reachable from root_words (e.g. the words of a
 * kernel-argument block): the ranges the root words lie in, then, over the
 * edges of edge_bm (host copy of kc_pointer_graph's output for the same
 * ranges), everything reachable from them.  reach_bm: host, ceil(n / 64) u64
 * words, bit r set iff range r is reached (bits past n cleared).  Ranges are
 * checked as in kc_range_check. */
int kc_graph_reach(const kc_range *ranges, uint32_t n, const uint64_t *edge_bm,
                   const uint64_t *root_words, uint64_t n_root_words,
                   uint64_t *reach_bm);

/* Closure scan (Sec. 4.2.1, address-space closure and its bounds): every
 * 8-byte-aligned word of every range is tested against the window; a
 * pointer-like word is in range iff base_r <= w < base_r + size_r for some r
 * (half-open: one past the end is out of range). */
int kc_closure_scan(kc_ctx *ctx, const kc_rangeset *rs,
                    const kc_scan_args *scan, void *stream);

/* Compare each pair (Sec. 4.5.2: byte-exact comparison reports differing
 * bytes; tolerance comparison reports NaNs explicitly).  Per element, bitwise
 * equal -> distance 0; both NaN -> n_nan_both; one NaN -> n_nan_*_only;
 * otherwise the ULP distance |ord(c) - ord(g)| with ord = +-magnitude bits
 * goes to the histogram and the fp64 errors.  res_d: n_pairs device structs.
 * All pairs run in one persistent launch unless the tuning sets per_item.
 * Grows ctx scratch on demand and stages the pair list through pinned host
 * memory: not for graph capture.  Errors: KC_EDTYPE, KC_EALIGN, KC_EINVAL. */
int kc_compare(kc_ctx *ctx, const kc_pair *pairs, uint32_t n_pairs,
               kc_cmp_result *res_d, void *stream);

/* A resident pair list for repeated or graph-recorded compares: the pair and
 * tile tables (tile size taken from the context's compare tuning at creation)
 * and the accumulators live on the device.  Creation validates like
 * kc_compare, allocates and uploads synchronously; the buffers it names must
 * stay alive and in place while the set is used. */
int kc_pairset_create(kc_ctx *ctx, const kc_pair *pairs, uint32_t n_pairs,
                      kc_pairset **out);
void kc_pairset_destroy(kc_pairset *ps);

/* kc_compare over a resident pair set: no allocation, no host
 * synchronisation, so it can be recorded into a graph.  Results are identical
 * to kc_compare on the same pairs.  One stream at a time per set. */
int kc_compare_pairset(kc_ctx *ctx, const kc_pairset *ps, kc_cmp_result *res_d,
                       void *stream);

/* For callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  kc_compare with the same
 * arguments, checks, error codes and reports (bit-identical), but nothing is
 * allocated, on the device or on the host: the pair records travel in the
 * kernel arguments (48 pairs per launch) and the per-pair accumulators live
 * in a static device array of KC_NOALLOC_MAX_PAIRS x 512 bytes (2 MiB), one
 * copy per device, bound when the first context is created on that device and
 * held until the process ends.  More than KC_NOALLOC_MAX_PAIRS pairs:
 * KC_ELIMIT, nothing launched.  Every call on a device shares that device's
 * array, so calls that overlap on one device (two streams, or two threads)
 * race and their reports are undefined: serialize them.  Each call first
 * clears the accumulators it uses with a fill kernel (no memset node), so
 * whatever an earlier or failed call left there does not matter.  Launch
 * shape from the context's compare tuning (grid and tile size; per_item does
 * not apply).  Asynchronous on `stream`: res_d[0 .. n_pairs) is written by
 * the last kernels of the call. */
int kc_compare_noalloc(kc_ctx *ctx, const kc_pair *pairs, uint32_t n_pairs,
                       kc_cmp_result *res_d, void *stream);

/* ---- candidate materialisation for the validation server (a request names
 *      a golden buffer, a tolerance and a seed; the candidate is the golden
 *      moved by the seeded perturbation: Sec. 4.5.2's validation of a
 *      reproducer's outputs, reproducers feeding tuning agents, Sec. 1) ----- */

/* One buffer of a typed arena: element offset and length, and its seed (the
 * low 31 bits are used). */
typedef struct {
  uint64_t offset, length;
  uint32_t seed, reserved;
} kc_perturb_buf;

/* In place on arena_d (device, arena_elems elements of `dtype`, aligned to
 * the element size): in each buffer, block j < floor(length / block) moves
 * one element, offset + j*block + (h1 mod block), by 1 + (h2 mod kmax)
 * steps, towards -inf when bit 20 of h2 is set, with
 *   h1 = mix32(seed*0x9E37 + j*0x85EB + 1), h2 = mix32(h1 + seed + 0x27D4EB2F),
 *   mix32(x) = two rounds of x = ((x >> 16) ^ x) * 0x45D9F3B mod 2^32, then
 *              (x >> 16) ^ x.
 * A float steps in the sign-magnitude order of its bits (+0 and -0 both 0),
 * clamped at +-inf, or at the largest finite code where the format has no
 * inf; NaN codes stay.  Integers move by the step, clamped to their range.
 * Buffers may not overlap.  The caller owns arena_d; bufs (host) is read
 * during the call only.  Asynchronous on `stream`; the buffer list is
 * passed in kernel arguments (no allocation, no staging, no host sync).
 * Errors, all detected before any launch except the last: KC_EINVAL (no
 * context, a buffer past arena_elems, block or kmax 0), KC_EDTYPE (KC_U8),
 * KC_EALIGN (arena_d not aligned to the element size), KC_EHIP (a launch
 * failed; kc_last_error names it). */
int kc_perturb(kc_ctx *ctx, void *arena_d, uint64_t arena_elems, uint32_t dtype,
               const kc_perturb_buf *bufs, uint32_t n_bufs, uint64_t block,
               uint32_t kmax, void *stream);

/* One candidate to materialise: its golden (device, 16-byte aligned), its
 * place in the arena (element offset; arena_d + offset elements 16-byte
 * aligned), its length in elements and its seed (the low 31 bits are used). */
typedef struct {
  const void *src_d;
  uint64_t offset, length;
  uint32_t seed, reserved;
} kc_materialize_buf;

/* Copy and perturb in one pass: buffer b of arena_d becomes its golden moved
 * by exactly the perturbation kc_perturb applies (same block, kmax and seed
 * rules), so that the result equals a copy of each golden into the arena
 * followed by kc_perturb, at one read of the golden and one write of the
 * candidate.  Nothing outside [offset, offset + length) of each buffer is
 * written and nothing past each golden is read.  Buffers may not overlap each
 * other or their goldens.  The caller owns arena_d and every src_d; bufs
 * (host) is read during the call only.  Asynchronous on `stream`; the buffer
 * list goes in kernel arguments (no allocation, no host sync).  Errors, all
 * detected before any launch except the last: KC_EINVAL (no context, a
 * buffer past arena_elems, a null golden of nonzero length, block or kmax 0),
 * KC_EDTYPE (KC_U8), KC_EALIGN (a golden or a destination not 16-byte
 * aligned), KC_EHIP (a launch failed; kc_last_error names it). */
int kc_materialize(kc_ctx *ctx, void *arena_d, uint64_t arena_elems, uint32_t dtype,
                   const kc_materialize_buf *bufs, uint32_t n_bufs, uint64_t block,
                   uint32_t kmax, void *stream);

/* ---- snapshot files (Sec. 4.2.1: every region streamed to files in
 *      fixed-size chunks, metadata written before the data) ------------------ */

typedef struct {
  uint64_t bytes;     /* data bytes moved (metadata files not counted)       */
  double seconds;     /* wall time of the call                                 */
  double copy_wait_s; /* of which the host waited for device copies           */
  double file_s;      /* of which the host spent in file writes (reads)       */
} kc_io_stats;

/* Write a snapshot to directory `dir` (created if missing): manifest.json
 * (human-readable: seed, counts, every region's base and size, file list) and
 * header.bin + ranges.bin (the same metadata, binary) first, then hash.bin
 * (N u64), zero_bm.bin, changed_bm.bin (delta snapshots: changed_bm_d non-NULL),
 * page_va.bin (min(n_kept, cap_pages) u64) and packed.bin (that many pages).
 * Device-to-host copies go through four pinned buffers of chunk_bytes (0 = 64
 * MiB) on `stream`: while one chunk is written, the copies of the next three
 * are in flight.  *stats (may be NULL) receives the data bytes, the wall time,
 * and how much of it the host spent waiting for copies and inside file
 * writes (which of the two bounds the save).  Synchronous: returns when the
 * files are complete.  Allocates pinned memory for the call.  Errors:
 * KC_EINVAL (bad arguments, file system errors; see kc_last_error), KC_EHIP. */
int kc_snapshot_save(kc_ctx *ctx, const kc_rangeset *rs, const char *dir,
                     uint64_t seed, const uint64_t *hash_d,
                     const uint64_t *zero_bm_d, const uint64_t *changed_bm_d,
                     const void *packed_d, const uint64_t *page_va_d,
                     const uint64_t *n_kept_d, uint64_t cap_pages,
                     uint64_t chunk_bytes, void *stream, kc_io_stats *stats);

/* Load a saved snapshot into device buffers for kc_restore.  The snapshot's
 * ranges must equal the range set's (same VAs and sizes: the restore is
 * VA-faithful), else KC_EINVAL.  hash_d may be NULL (not loaded); a delta
 * snapshot needs changed_bm_d; more packed pages than cap_pages is
 * KC_ELIMIT.  A header whose kept count exceeds its page count, or whose
 * packed count exceeds its kept count, is KC_EINVAL.  A snapshot saved
 * truncated (cap_pages below its kept count at save time, so fewer packed
 * pages than kept pages) is refused with KC_ELIMIT: a restore from it would
 * leave the missing pages unwritten.  On success *n_kept_d equals the number
 * of packed pages loaded.  Host-to-device copies are chunked like the save
 * (a chunk is read while the copies of up to three earlier ones are in
 * flight), each chunk read by up to four host threads on slices of it;
 * *stats splits the time into copy waits and file reads.  Synchronous. */
int kc_snapshot_load(kc_ctx *ctx, const kc_rangeset *rs, const char *dir,
                     uint64_t *hash_d, uint64_t *zero_bm_d,
                     uint64_t *changed_bm_d, void *packed_d,
                     uint64_t *page_va_d, uint64_t *n_kept_d,
                     uint64_t cap_pages, uint64_t chunk_bytes, void *stream,
                     kc_io_stats *stats);

#ifdef __cplusplus
}
#endif
#endif

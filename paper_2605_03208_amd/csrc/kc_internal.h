// kc_internal.h -- shared definitions of the gfx950 kernels and the ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <vector>

#include "kc.h"

namespace kc {

constexpr uint32_t kPage = 4096;
constexpr uint32_t kWave = 64;
constexpr uint32_t kTilePages = 16;     // pages per wave tile (one lane quad per page)
constexpr uint32_t kChunk = 512;        // bytes of each page staged per step
constexpr uint32_t kStageStride = kChunk + 32;  // padded LDS row: quads land in distinct banks
constexpr uint32_t kFences = 256;       // range-table entries held in LDS by one-wave workgroups
constexpr uint32_t kWideFences = 4096;  // the same, shared by the waves of a multi-wave workgroup
constexpr uint32_t kBuckets = 1024;     // entries of the LDS bucket index over the ranges

// 16-byte global accesses.  Data that streams through once (pages, packed
// snapshot, compared buffers) uses non-temporal loads and stores, which on
// gfx950 measured 7.2 TB/s for a read-only stream against 6.35 TB/s for
// plain loads.
//
// The addresses are typed as global memory (address space 1).  A plain
// pointer made from an integer compiles to a flat access, which counts on the
// LDS counter as well, so the first LDS wait after it (the hash reads its
// stage from LDS while the next chunk is in flight) would wait for the
// global loads too.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
#define KC_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ uint4 ld16(uint64_t addr) {
  const v4u v = *(const KC_GLOBAL v4u*)addr;
  return make_uint4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st16(uint64_t addr, uint4 v) {
  const v4u x = {v.x, v.y, v.z, v.w};
  *(KC_GLOBAL v4u*)addr = x;
}
__device__ __forceinline__ uint4 ld16nt(uint64_t addr) {
  const v4u v = __builtin_nontemporal_load((const KC_GLOBAL v4u*)addr);
  return make_uint4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st16nt(uint64_t addr, uint4 v) {
  const v4u x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, (KC_GLOBAL v4u*)addr);
}
// An 8-byte global load through a plain pointer, kept a global access.
__device__ __forceinline__ uint64_t ld8g(const uint64_t* p) { return *(const KC_GLOBAL uint64_t*)p; }

// Hash units: a range is cut into units of 2^ushift bytes (4 KiB pages by
// default, up to 2 MiB for whole-allocation capture of large tensors); the
// hash table, bitmaps and packed slots count units.  The closure scan and the
// pointer graph always walk 4 KiB page tiles.
constexpr uint32_t kMinUnitShift = 12, kMaxUnitShift = 21;

// A tile: up to 16 consecutive units of one range.  Only a range's last unit
// can be partial (a range size that is not a multiple of the unit); last_len
// is the byte count of the tile's last unit.
struct Tile {
  uint64_t va;              // VA of the first unit
  uint32_t g;               // global index of the first unit
  uint32_t npages : 8;      // 1..16 units (1..64 in the tiles of the pipelined hashing pass)
  uint32_t last_len : 24;   // 1..unit bytes
};
static_assert(sizeof(Tile) == 16, "tile layout");

// Bytes of page j of a 4 KiB page tile.
__device__ __forceinline__ uint32_t page_bytes(const Tile& t, uint32_t j) {
  return j + 1u == t.npages ? (uint32_t)t.last_len : kPage;
}
// Bytes of unit j of a tile of units of `unit` bytes.
__device__ __forceinline__ uint32_t unit_bytes(const Tile& t, uint32_t j, uint32_t unit) {
  return j + 1u == t.npages ? (uint32_t)t.last_len : unit;
}

// The 16 bytes at offset off of a page of len bytes, bytes at or past len
// cleared.
__device__ __forceinline__ uint4 clip16(uint4 v, uint32_t off, uint32_t len) {
  if (off + 16u <= len) return v;
  if (off >= len) return make_uint4(0, 0, 0, 0);
  const uint32_t keep = len - off;  // 1..15 bytes
  const auto cut = [&](uint32_t w, uint32_t i) -> uint32_t {
    const uint32_t lo = i * 4u;
    if (keep >= lo + 4u) return w;
    if (keep <= lo) return 0u;
    return w & ((1u << (8u * (keep - lo))) - 1u);
  };
  return make_uint4(cut(v.x, 0), cut(v.y, 1), cut(v.z, 2), cut(v.w, 3));
}

// The two 8-byte words of the 16 bytes at offset off of a page of len bytes,
// each cleared unless it lies wholly inside the page (a cleared word is never
// pointer-like: windows start at 1 or above).
__device__ __forceinline__ uint4 words_inside(uint4 v, uint32_t off, uint32_t len) {
  if (off + 16u <= len) return v;
  if (off + 8u <= len) return make_uint4(v.x, v.y, 0u, 0u);
  return make_uint4(0, 0, 0, 0);
}

// 16 bytes at tile segment s (1 KiB each, four per page) for this lane, with
// the words that are not wholly inside the range cleared.
__device__ __forceinline__ uint4 seg_words(const Tile& t, uint32_t s, uint32_t lane, uint4 v) {
  const uint32_t pg = s >> 2, off = (s & 3u) * 1024u + lane * 16u;
  return pg + 1u == t.npages ? words_inside(v, off, t.last_len) : v;
}

// Store only the first n (0..16) bytes of v at addr.
__device__ __forceinline__ void st_bytes(uint64_t addr, uint4 v, uint32_t n) {
  if (n >= 16u) {
    st16nt(addr, v);
    return;
  }
#pragma unroll
  for (uint32_t i = 0; i < 16u; ++i) {
    if (i < n) {
      const uint32_t w = i < 4u ? v.x : (i < 8u ? v.y : (i < 12u ? v.z : v.w));
      *(KC_GLOBAL uint8_t*)(addr + i) = (uint8_t)(w >> (8u * (i & 3u)));
    }
  }
}

// Sorted range table on the device (bases and one-past-end addresses), with
// a bucket index over [lo, lo + span) = [lowest base, highest end): bucket b
// covers addresses lo + [b << shift, (b + 1) << shift) and holds the last
// fence whose base is at or below the bucket's first address.
struct RangeTable {
  const uint64_t* base;
  const uint64_t* end;
  const uint16_t* bucket;  // kBuckets entries
  uint64_t lo, span;
  uint32_t n;
  uint32_t stride;   // LDS fence stride: fence i = range i * stride
  uint32_t n_fence;  // ceil(n / stride) <= kFences
  uint32_t shift;
  // The wide table (up to kWideFences fences, in dynamic LDS shared by the
  // waves of a workgroup): its stride, fence count and bucket index.
  const uint16_t* bucket_w;
  uint32_t stride_w, n_fence_w;
};

// The closure-scan totals are accumulated in kScanSlots slot pairs, each on
// its own 256-byte line: every wave adds its counts once at its end, and
// waves that finish together would otherwise queue on one address.
constexpr uint32_t kScanSlots = 64;
constexpr uint32_t kScanSlotStride = 32;  // u64 words between slots
constexpr uint32_t kScanCountWords = kScanSlots * kScanSlotStride;

struct ScanDev {
  uint64_t lo, span;                 // pointer-like iff (w - lo) < span
  RangeTable rt;
  uint32_t* tile_oob;                // per-tile out-of-range count
  unsigned long long* counts;        // slot s: [s * kScanSlotStride] n_ptr_like, [+1] n_in_range (accumulated)
};

struct HashParams {
  const Tile* tiles;
  uint32_t n_tiles;
  uint32_t tile0;          // index of tiles[0] in the rangeset's tile list
  const uint32_t* ragged;  // indices (in the rangeset's list) of tiles with a partial last page
  uint32_t n_ragged;
  uint64_t seed;
  const uint64_t* prior;   // nullable
  uint64_t* hash;
  uint64_t* zero_bm;       // output, or input when gathering
  uint64_t* changed_bm;
  const uint64_t* word_prefix;  // keep prefix per bitmap word (gathering)
  uint8_t* packed;
  uint64_t* page_va;
  uint64_t cap_pages;
  uint32_t ushift;         // log2 of the hash unit (12: 4 KiB pages)
  ScanDev scan;
};

// Exclusive-scan sources.
enum ScanSrcKind : uint32_t { kSrcKeepBits = 0, kSrcCounts = 1 };
struct ScanSrc {
  uint32_t kind;
  const uint64_t* zero_bm;     // keep bits: ~zero (& changed)
  const uint64_t* changed_bm;  // nullable
  uint64_t n_pages;
  const uint32_t* counts;      // per-item counts
  uint64_t n_items;            // words or counts
};

struct CmpPairDev {
  const uint8_t* cand;
  const uint8_t* gold;
  uint64_t n_elems;
  uint32_t dtype, tol;
  uint32_t n_tiles, esize;
  double atol, rtol;
};
static_assert(sizeof(CmpPairDev) == 56, "pair layout");

struct CmpTileDev {
  uint32_t pair, idx;
};

// Pairs carried in the kernel arguments of one compare launch (the variant
// that allocates nothing): pair records and the inclusive prefix of their
// tile counts, under the 4 KiB kernel-argument limit.
constexpr uint32_t kArgPairs = 48;
struct CmpArgPairs {
  CmpPairDev pair[kArgPairs];
  uint32_t tile_end[kArgPairs];
  uint32_t n;        // pairs in this launch
  uint32_t n_tiles;  // = tile_end[n - 1]
};
static_assert(sizeof(CmpArgPairs) <= 3072, "kernel arguments");

constexpr uint32_t kAccWords = 64;  // per-pair accumulator words
// accumulator word map
enum : uint32_t {
  kAccMisElems = 0, kAccMisBytes, kAccNanBoth, kAccNanCand, kAccNanGold, kAccOverTol,
  kAccMaxAbs, kAccMaxRel, kAccFirstInv, kAccNotClose, kAccHist = 16  // 48 bins: words 16..63
};

// ---- launchers (kc_kernels.hip) ------------------------------------------
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_zero3(uint64_t* a, uint64_t na, uint64_t* b, uint64_t nb, uint64_t* c, uint64_t nc,
                        hipStream_t s);
// depth 2 to 4: the pipelined pass of large units with that many chunks in flight per wave (few tiles, about one
// wave per SIMD); not with scan.  0 or 1: the pass with one chunk in flight.
hipError_t launch_page_hash(const HashParams& p, bool gather, bool prior, bool scan, uint32_t depth,
                            uint32_t grid, uint32_t n_cu, hipStream_t s);
// The pipelined pass of units above 4 KiB (kc_units.hip), depth 2 to 4, on a launch shape already chosen.
hipError_t launch_page_hash_deep(const HashParams& p, bool gather, bool prior, uint32_t depth, uint32_t blocks,
                                 uint32_t waves_per_block, hipStream_t s);
hipError_t launch_probe_zero(const Tile* tiles, uint32_t n_tiles, uint64_t* zero_bm, uint32_t ushift,
                             uint32_t grid, hipStream_t s);
hipError_t launch_scan(const ScanSrc& src, uint64_t* out, uint64_t* block_sums,
                       uint64_t* total_out, hipStream_t s);
hipError_t launch_gather(const Tile* tiles, uint32_t n_tiles, const uint64_t* zero_bm,
                         const uint64_t* changed_bm, const uint64_t* word_prefix,
                         uint8_t* packed, uint64_t* page_va, uint64_t cap_pages, uint32_t ushift,
                         uint32_t grid, hipStream_t s);
hipError_t launch_restore_zero(const Tile* tiles, uint32_t n_tiles, const uint64_t* zero_bm,
                               const uint64_t* changed_bm, unsigned long long* n_bad, uint32_t ushift,
                               uint32_t grid, hipStream_t s);
hipError_t launch_restore_scatter(const RangeTable& rt, const uint8_t* packed,
                                  const uint64_t* page_va, const uint64_t* n_kept,
                                  uint64_t cap_pages, unsigned long long* n_bad,
                                  bool ragged, bool delta, uint32_t ushift, uint32_t grid, hipStream_t s);
hipError_t launch_closure(const Tile* tiles, uint32_t n_tiles, uint32_t tile0,
                          const ScanDev& sd, uint32_t grid, uint32_t n_cu, hipStream_t s);
hipError_t launch_pointer_graph(const Tile* tiles, uint32_t n_tiles, uint64_t lo, uint64_t span,
                                const RangeTable& rt, uint64_t* edge_bm, uint32_t row_words, uint32_t grid,
                                uint32_t n_cu, hipStream_t s);
hipError_t launch_region_init(kc_region_diff_result* res, uint32_t n, uint64_t* bm_a, uint64_t* bm_b, uint64_t n_words,
                              hipStream_t s);
hipError_t launch_region_diff(const Tile* tiles, uint32_t n_tiles, const RangeTable& rt, const uint64_t* changed_bm,
                              const uint64_t* gold_zero_bm, const uint64_t* rank_prefix, const uint64_t* gold_page_va,
                              const uint64_t* gold_n_kept, uint64_t cap, const uint8_t* gold_packed,
                              kc_region_diff_result* res, uint32_t ushift, uint32_t grid, hipStream_t s);
hipError_t launch_oob_emit(const Tile* tiles, uint32_t n_tiles, const ScanDev& sd,
                           const uint64_t* tile_prefix, const uint64_t* n_oob, kc_oob* oob,
                           uint64_t cap, kc_scan_result* res, uint64_t n_words, hipStream_t s);
hipError_t launch_compare(const CmpPairDev* pairs, const CmpTileDev* tiles, uint32_t n_tiles,
                          uint32_t tile_bytes, unsigned long long* acc, uint32_t grid, hipStream_t s);
hipError_t launch_compare_finalize(const CmpPairDev* pairs, uint32_t n_pairs, unsigned long long* acc,
                                   kc_cmp_result* res, hipStream_t s);
// The pass and the reports of the pairs in `a` (accumulators acc[pair * kAccWords ...], zero on entry and
// zeroed again; reports res[0 .. a.n)).
hipError_t launch_compare_args(const CmpArgPairs& a, uint32_t tile_bytes, unsigned long long* acc,
                               kc_cmp_result* res, uint32_t grid, hipStream_t s);

// ---- shared host helpers (kc_api.hip) ----------------------------------------
uint32_t grid_for(const kc_ctx* c, uint32_t op, uint32_t fallback_per_cu);  // persistent grid of an op
uint32_t elem_size(uint32_t dtype);                                         // bytes of one element
uint32_t compare_tile_bytes(const kc_ctx* c, const kc_pair* pairs, uint32_t n_pairs);

// ---- the compare that allocates nothing (kc_noalloc.hip) ---------------------
// Looks up, once per device, the device address of the static scratch array
// (the device must be current); KC_EHIP if the lookup fails.
int noalloc_bind(int device);

// ---- errors and device selection (kc_api.hip) ------------------------------
void set_error_text(const char* text);
void set_error(const char* what, hipError_t e);

#define KC_HIP(call)                          \
  do {                                        \
    hipError_t kc_e_ = (call);                \
    if (kc_e_ != hipSuccess) {                \
      ::kc::set_error(#call, kc_e_);          \
      return KC_EHIP;                         \
    }                                         \
  } while (0)

// Makes `dev` current for the scope of a call and restores the caller's device.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();  // do not leave the failure for the caller's next HIP call
      char msg[64];
      std::snprintf(msg, sizeof(msg), "hipSetDevice(%d) failed", dev);
      set_error_text(msg);
    }
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace kc

// ---- library objects --------------------------------------------------------
struct kc_ctx {
  int device = 0;
  uint32_t n_cu = 256;
  kc_tuning tune[KC_OP_COUNT];
  uint8_t* cmp_dev = nullptr;  // pairs | tiles
  size_t cmp_dev_cap = 0;
  unsigned long long* cmp_acc = nullptr;  // accumulators: zero between calls (finalize resets them)
  size_t cmp_acc_cap = 0;
  bool cmp_acc_dirty = false;
  uint8_t* cmp_host = nullptr;  // pinned staging of pairs | tiles
  size_t cmp_host_cap = 0;
  hipEvent_t staged = nullptr;  // completion of the last staging copy
  bool staged_pending = false;
  bool timing = false;  // record events around the main kernel of each op
  hipEvent_t t_start[KC_OP_COUNT] = {};
  hipEvent_t t_stop[KC_OP_COUNT] = {};
  bool t_valid[KC_OP_COUNT] = {};
};

struct kc_rangeset {
  kc_ctx* ctx = nullptr;
  int device = 0;  // recorded at creation: destroy never touches the context
  uint32_t n_ranges = 0, n_tiles = 0;
  uint32_t ushift = 12;              // log2 of the hash unit; n_pages, n_words and the tiles count units
  uint64_t n_pages = 0, n_words = 0;
  uint64_t n_scan_words = 0;         // 8-byte words wholly inside the ranges
  uint32_t n_ragged = 0;             // tiles with a partial last page (at most one per range)
  uint32_t* ragged = nullptr;        // their indices, ascending (device)
  std::vector<uint32_t> ragged_of;   // per range: its entry in ragged, or UINT32_MAX
  std::vector<uint32_t> range_tile;  // first tile of each range (n + 1)
  uint64_t win_lo = 0, win_hi = 0;   // default pointer window
  std::vector<kc_range> host_ranges;
  // 4 KiB page tiles walked by the closure scan, its list emission and the
  // pointer graph (the same list as `tiles` when the unit is the page)
  uint32_t n_scan_tiles = 0;
  std::vector<uint32_t> scan_range_tile;
  kc::Tile* scan_tiles = nullptr;
  // tiles of the pipelined hashing pass of large units: up to 32 units of one
  // range, each lane quad hashing up to two of them in turn (the same list as
  // `tiles` when a quad takes one unit)
  uint32_t n_deep_tiles = 0;
  std::vector<uint32_t> deep_range_tile;
  kc::Tile* deep_tiles = nullptr;
  void* dev = nullptr;
  kc::Tile* tiles = nullptr;
  uint64_t* bases = nullptr;
  uint64_t* ends = nullptr;
  uint32_t* tile_oob = nullptr;
  uint64_t* tile_prefix = nullptr;
  uint64_t* word_prefix = nullptr;
  uint64_t* block_sums = nullptr;
  unsigned long long* counts = nullptr;  // closure-scan slots (kScanCountWords)
  unsigned long long* n_bad = nullptr;   // rejected page VAs of a restore given no counter
  uint64_t* n_oob = nullptr;
  kc::RangeTable rt{};
};

struct kc_pairset {
  kc_ctx* ctx = nullptr;
  int device = 0;  // recorded at creation: destroy never touches the context
  uint32_t n_pairs = 0, tile_bytes = 0;
  uint64_t n_tiles = 0;
  std::vector<uint64_t> tile_off;
  void* dev = nullptr;
  kc::CmpPairDev* pairs = nullptr;
  kc::CmpTileDev* tiles = nullptr;
  unsigned long long* acc = nullptr;
  mutable bool acc_dirty = false;  // a failed compare left accumulators set
};


// kc_api.hip -- the extern "C" entry points of libkc.so: argument checks,
// range-set upload, scratch ownership and the launch sequence of each op.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "kc_internal.h"

using namespace kc;

namespace {
thread_local char g_last_error[256] = "";
}  // namespace

namespace kc {
void set_error_text(const char* text) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", text); }
void set_error(const char* what, hipError_t e) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%s)", what, hipGetErrorName(e),
                hipGetErrorString(e));
}
}  // namespace kc

namespace {



constexpr uint64_t kMaxPages = (1ull << 32) - 1;
constexpr uint32_t kMaxRanges = 1u << 31;

int range_check(const kc_range* r, uint32_t n, uint64_t* n_pages) {
  if (n > 0 && r == nullptr) return KC_EINVAL;
  if (n >= kMaxRanges) return KC_ELIMIT;
  uint64_t pages = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const uint64_t base = r[i].base, size = r[i].size;
    if (base == 0 || size == 0) return KC_EINVAL;
    if (base & (KC_PAGE_SIZE - 1)) return KC_EALIGN;
    if (base + size < base) return KC_EINVAL;
    if (i > 0 && base < r[i - 1].base + r[i - 1].size) return KC_EORDER;
    pages += (size + KC_PAGE_SIZE - 1) / KC_PAGE_SIZE;  // a partial last page counts
    if (pages > kMaxPages) return KC_ELIMIT;
  }
  if (n_pages) *n_pages = pages;
  return KC_OK;
}

void default_window(const kc_range* r, uint32_t n, uint64_t* lo, uint64_t* hi) {
  const uint64_t margin = 1ull << 32;
  if (n == 0) {
    *lo = *hi = 0;
    return;
  }
  const uint64_t min_base = r[0].base, max_end = r[n - 1].base + r[n - 1].size;
  *lo = min_base > margin + KC_PAGE_SIZE ? min_base - margin : KC_PAGE_SIZE;
  *hi = max_end <= UINT64_MAX - margin ? max_end + margin : UINT64_MAX;
}

}  // namespace

namespace kc {
uint32_t grid_for(const kc_ctx* c, uint32_t op, uint32_t fallback_per_cu) {
  const uint32_t per = c->tune[op].grid_per_cu ? c->tune[op].grid_per_cu : fallback_per_cu;
  return std::max(1u, c->n_cu * per);
}
}  // namespace kc

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Brackets the main-kernel launches of one op with timing events when enabled.
struct KernelTimer {
  kc_ctx* c;
  uint32_t op;
  hipStream_t s;
  KernelTimer(kc_ctx* c_, uint32_t op_, hipStream_t s_) : c(c_), op(op_), s(s_) {
    if (c->timing) (void)hipEventRecord(c->t_start[op], s);
  }
  ~KernelTimer() {
    if (c->timing && hipEventRecord(c->t_stop[op], s) == hipSuccess) c->t_valid[op] = true;
  }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Resolve a closure-scan request into the device-side description.
int make_scan(const kc_rangeset* rs, const kc_scan_args* sa, ScanDev* sd) {
  if (sa->res_d == nullptr || (sa->oob_cap > 0 && sa->oob_d == nullptr)) return KC_EINVAL;
  uint64_t lo = sa->win_lo, hi = sa->win_hi;
  if (lo == 0 && hi == 0) {
    lo = rs->win_lo;
    hi = rs->win_hi;
  } else if (lo == 0 || lo >= hi) {
    return KC_EINVAL;
  }
  sd->lo = lo;
  sd->span = hi - lo;
  if (rs->n_ranges == 0) sd->span = 0;
  sd->rt = rs->rt;
  sd->tile_oob = rs->tile_oob;
  sd->counts = rs->counts;
  return KC_OK;
}

// Count-scan the per-tile out-of-range totals, emit the ordered list, write
// the result struct.
int finish_scan(kc_rangeset* rs, const kc_scan_args* sa, const ScanDev& sd, hipStream_t s) {
  ScanSrc src{};
  src.kind = kSrcCounts;
  src.counts = rs->tile_oob;
  src.n_items = rs->n_scan_tiles;
  KC_HIP(launch_scan(src, rs->tile_prefix, rs->block_sums, rs->n_oob, s));
  KC_HIP(launch_oob_emit(rs->scan_tiles, rs->n_scan_tiles, sd, rs->tile_prefix, rs->n_oob, sa->oob_d, sa->oob_cap,
                         sa->res_d, rs->n_scan_words, s));
  return KC_OK;
}

}  // namespace

extern "C" {

const char* kc_strerror(int code) {
  switch (code) {
    case KC_OK: return "ok";
    case KC_EINVAL: return "invalid argument";
    case KC_EALIGN: return "misaligned range or buffer";
    case KC_EORDER: return "ranges unsorted or overlapping";
    case KC_ENOMEM: return "out of memory";
    case KC_EHIP: return "HIP runtime error";
    case KC_EDTYPE: return "unknown element type";
    case KC_ELIMIT: return "size limit exceeded";
    case KC_ERELOC: return "address range not available at its original VA";
    default: return "unknown status";
  }
}

const char* kc_last_error(void) { return g_last_error; }

int kc_abi_version(void) { return KC_ABI_VERSION; }

int kc_range_check(const kc_range* ranges, uint32_t n, uint64_t* n_pages) { return range_check(ranges, n, n_pages); }

int kc_default_window(const kc_range* ranges, uint32_t n, uint64_t* win_lo, uint64_t* win_hi) {
  if (win_lo == nullptr || win_hi == nullptr) return KC_EINVAL;
  const int st = range_check(ranges, n, nullptr);
  if (st != KC_OK) return st;
  default_window(ranges, n, win_lo, win_hi);
  return KC_OK;
}

int kc_ctx_create(kc_ctx** out, int hip_device) {
  if (out == nullptr) return KC_EINVAL;
  *out = nullptr;
  DeviceGuard g(hip_device);
  if (!g.ok) {
    std::snprintf(g_last_error, sizeof(g_last_error), "hipSetDevice(%d) failed", hip_device);
    return KC_EHIP;
  }
  int cu = 0;
  KC_HIP(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, hip_device));
  kc_ctx* c = new (std::nothrow) kc_ctx();
  if (c == nullptr) return KC_ENOMEM;
  c->device = hip_device;
  c->n_cu = cu > 0 ? (uint32_t)cu : 256u;
  std::memset(c->tune, 0, sizeof(c->tune));
  hipError_t e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming);
  if (e != hipSuccess) {
    set_error("hipEventCreateWithFlags", e);
    delete c;
    return KC_EHIP;
  }
  const int bound = noalloc_bind(hip_device);  // device address of the static compare scratch, once per device
  if (bound != KC_OK) {
    (void)hipEventDestroy(c->staged);
    delete c;
    return bound;
  }
  *out = c;
  return KC_OK;
}

void kc_ctx_destroy(kc_ctx* c) {
  if (c == nullptr) return;
  DeviceGuard g(c->device);
  if (c->staged) {
    (void)hipEventSynchronize(c->staged);
    (void)hipEventDestroy(c->staged);
  }
  if (c->cmp_dev) (void)hipFree(c->cmp_dev);
  if (c->cmp_acc) (void)hipFree(c->cmp_acc);
  if (c->cmp_host) (void)hipHostFree(c->cmp_host);
  for (uint32_t op = 0; op < KC_OP_COUNT; ++op) {
    if (c->t_start[op]) (void)hipEventDestroy(c->t_start[op]);
    if (c->t_stop[op]) (void)hipEventDestroy(c->t_stop[op]);
  }
  delete c;
}

int kc_ctx_enable_timing(kc_ctx* c, int on) {
  if (c == nullptr) return KC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  if (on) {
    for (uint32_t op = 0; op < KC_OP_COUNT; ++op) {
      if (!c->t_start[op]) KC_HIP(hipEventCreate(&c->t_start[op]));
      if (!c->t_stop[op]) KC_HIP(hipEventCreate(&c->t_stop[op]));
    }
  }
  c->timing = on != 0;
  return KC_OK;
}

int kc_ctx_kernel_ms(kc_ctx* c, uint32_t op, float* ms) {
  if (c == nullptr || ms == nullptr || op >= KC_OP_COUNT || !c->t_valid[op]) return KC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  KC_HIP(hipEventSynchronize(c->t_stop[op]));
  KC_HIP(hipEventElapsedTime(ms, c->t_start[op], c->t_stop[op]));
  return KC_OK;
}

int kc_ctx_set_tuning(kc_ctx* c, uint32_t op, const kc_tuning* t) {
  if (c == nullptr || t == nullptr || op >= KC_OP_COUNT) return KC_EINVAL;
  if (t->grid_per_cu > 1024u || t->depth > 4u) return KC_EINVAL;
  if (t->tile_bytes != 0 && (t->tile_bytes % 16u != 0 || t->tile_bytes < 4096u || t->tile_bytes > (64u << 20)))
    return KC_EINVAL;
  c->tune[op] = *t;
  return KC_OK;
}

int kc_ctx_get_tuning(const kc_ctx* c, uint32_t op, kc_tuning* t) {
  if (c == nullptr || t == nullptr || op >= KC_OP_COUNT) return KC_EINVAL;
  *t = c->tune[op];
  return KC_OK;
}

int kc_rangeset_create(kc_ctx* c, const kc_range* ranges, uint32_t n, kc_rangeset** out, uint64_t* n_pages_out) {
  return kc_rangeset_create_unit(c, ranges, n, KC_PAGE_SIZE, out, n_pages_out);
}

int kc_rangeset_create_unit(kc_ctx* c, const kc_range* ranges, uint32_t n, uint64_t unit, kc_rangeset** out,
                            uint64_t* n_units_out) {
  if (c == nullptr || out == nullptr) return KC_EINVAL;
  *out = nullptr;
  uint32_t ushift = kMinUnitShift;
  while (ushift < kMaxUnitShift && (1ull << ushift) < unit) ++ushift;
  if ((1ull << ushift) != unit) return KC_EINVAL;  // a power of two from 4 KiB to 2 MiB
  uint64_t n_pages = 0;
  int st = range_check(ranges, n, &n_pages);
  if (st != KC_OK) return st;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  kc_rangeset* rs = new (std::nothrow) kc_rangeset();
  if (rs == nullptr) return KC_ENOMEM;
  rs->ctx = c;
  rs->device = c->device;
  rs->n_ranges = n;
  rs->ushift = ushift;
  rs->host_ranges.assign(ranges, ranges + n);
  default_window(ranges, n, &rs->win_lo, &rs->win_hi);

  // Tiles of up to per_tile units of one range; a range's last unit holds
  // what is left of its size.  Returns the number of units.
  auto build_tiles = [&](uint32_t shift, uint32_t per_tile, std::vector<Tile>& tiles,
                         std::vector<uint32_t>& range_tile, std::vector<uint32_t>* ragged,
                         std::vector<uint32_t>* ragged_of) {
    const uint64_t u = 1ull << shift;
    range_tile.assign(n + 1, 0);
    if (ragged_of) ragged_of->assign(n, UINT32_MAX);
    uint64_t g0 = 0;
    for (uint32_t i = 0; i < n; ++i) {
      range_tile[i] = (uint32_t)tiles.size();
      const uint64_t units = (ranges[i].size + u - 1) / u;
      const uint32_t tail = (uint32_t)(ranges[i].size - (units - 1) * u);  // bytes of the last unit
      for (uint64_t p = 0; p < units; p += per_tile) {
        Tile t;
        t.va = ranges[i].base + (p << shift);
        t.g = (uint32_t)(g0 + p);
        t.npages = (uint32_t)std::min<uint64_t>(per_tile, units - p);
        t.last_len = p + t.npages == units ? tail : (uint32_t)u;
        tiles.push_back(t);
      }
      g0 += units;
      if (ragged && tail != u) {  // the range's last tile holds a partial unit
        (*ragged_of)[i] = (uint32_t)ragged->size();
        ragged->push_back((uint32_t)tiles.size() - 1u);
      }
    }
    range_tile[n] = (uint32_t)tiles.size();
    return g0;
  };
  std::vector<Tile> tiles, scan_tiles;
  std::vector<uint32_t> ragged;
  // Units above 4 KiB: when 16-unit tiles would leave fewer than two waves per SIMD for the pipelined hashing
  // pass, tiles of 8 units give twice the waves (each with half its quads busy), and two waves per SIMD cover
  // each other's instruction latencies (2 MiB units of a 30 GiB pool: 11.4-12.6 ms against 16.5-17.2 ms).
  // That pass takes tiles of 32 units up to 256 KiB units (each lane quad hashes two units in turn) when those
  // still give two waves per SIMD: the skew of its quads then idles them for a smaller share of its rounds.
  // Measured at 64 KiB units on the 30 GiB pool, averages of three rounds in one process: 11.95 ms against
  // 12.68 at one unit per quad and 12.53 at four (128 KiB: 12.35 / 12.47 / 12.38).
  uint32_t per_tile = kTilePages, deep_per_tile = kTilePages;
  if (ushift > kMinUnitShift) {
    auto n_tiles_of = [&](uint64_t per) {
      uint64_t t = 0;
      for (uint32_t i = 0; i < n; ++i) t += (((ranges[i].size + (1ull << ushift) - 1) >> ushift) + per - 1) / per;
      return t;
    };
    const uint64_t want = 8ull * c->n_cu;
    if (n_tiles_of(kTilePages) < want) per_tile = kTilePages / 2;
    deep_per_tile = per_tile;
    for (uint32_t u = ushift <= 18 ? 2u : 1u; u > 1u; u /= 2u)
      if (n_tiles_of(kTilePages * u) >= want) {
        deep_per_tile = kTilePages * u;
        break;
      }
  }
  const uint64_t n_units = build_tiles(ushift, per_tile, tiles, rs->range_tile, &ragged, &rs->ragged_of);
  std::vector<Tile> deep_tiles;
  if (deep_per_tile != per_tile) build_tiles(ushift, deep_per_tile, deep_tiles, rs->deep_range_tile, nullptr, nullptr);
  else rs->deep_range_tile = rs->range_tile;
  if (ushift != kMinUnitShift)
    build_tiles(kMinUnitShift, kTilePages, scan_tiles, rs->scan_range_tile, nullptr, nullptr);
  else rs->scan_range_tile = rs->range_tile;
  std::vector<uint64_t> bases(n), ends(n);
  for (uint32_t i = 0; i < n; ++i) {
    rs->n_scan_words += ranges[i].size / 8;
    bases[i] = ranges[i].base;
    ends[i] = ranges[i].base + ranges[i].size;
  }
  rs->n_pages = n_units;
  rs->n_words = (n_units + 63) / 64;
  rs->n_tiles = (uint32_t)tiles.size();
  rs->n_scan_tiles = ushift != kMinUnitShift ? (uint32_t)scan_tiles.size() : rs->n_tiles;
  rs->n_deep_tiles = deep_per_tile != per_tile ? (uint32_t)deep_tiles.size() : rs->n_tiles;

  const uint64_t nb_words = (rs->n_words + 2047) / 2048, nb_tiles = ((uint64_t)rs->n_scan_tiles + 2047) / 2048;
  const size_t sz_tiles = align_up(sizeof(Tile) * std::max<size_t>(1, tiles.size()), 256);
  const size_t sz_st = align_up(sizeof(Tile) * scan_tiles.size(), 256);  // 4 KiB page tiles of the scans
  const size_t sz_dt = align_up(sizeof(Tile) * deep_tiles.size(), 256);  // tiles of the pipelined pass
  const size_t sz_r = align_up(8 * std::max<size_t>(1, n), 256);
  const size_t sz_oob = align_up(4 * std::max<size_t>(1, rs->n_scan_tiles), 256);
  const size_t sz_tp = align_up(8 * std::max<size_t>(1, rs->n_scan_tiles), 256);
  const size_t sz_wp = align_up(8 * std::max<uint64_t>(1, rs->n_words), 256);
  const size_t sz_bs = align_up(8 * std::max<uint64_t>(1, std::max(nb_words, nb_tiles)), 256);
  const size_t sz_misc = 256 + align_up(8 * kScanCountWords, 256);
  const size_t sz_bk = 2 * align_up(sizeof(uint16_t) * kBuckets, 256);  // bucket index of each fence table
  const size_t sz_rg = align_up(4 * std::max<size_t>(1, ragged.size()), 256);
  const size_t total = sz_tiles + sz_st + sz_dt + 2 * sz_r + sz_oob + sz_tp + sz_wp + sz_bs + sz_misc + sz_bk + sz_rg;
  hipError_t e = hipMalloc(&rs->dev, total);
  if (e != hipSuccess) {
    set_error("hipMalloc(rangeset)", e);
    delete rs;
    return e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
  }
  uint8_t* p = static_cast<uint8_t*>(rs->dev);
  rs->tiles = reinterpret_cast<Tile*>(p); p += sz_tiles;
  rs->scan_tiles = ushift != kMinUnitShift ? reinterpret_cast<Tile*>(p) : rs->tiles; p += sz_st;
  rs->deep_tiles = deep_tiles.empty() ? rs->tiles : reinterpret_cast<Tile*>(p); p += sz_dt;
  rs->bases = reinterpret_cast<uint64_t*>(p); p += sz_r;
  rs->ends = reinterpret_cast<uint64_t*>(p); p += sz_r;
  rs->tile_oob = reinterpret_cast<uint32_t*>(p); p += sz_oob;
  rs->tile_prefix = reinterpret_cast<uint64_t*>(p); p += sz_tp;
  rs->word_prefix = reinterpret_cast<uint64_t*>(p); p += sz_wp;
  rs->block_sums = reinterpret_cast<uint64_t*>(p); p += sz_bs;
  rs->n_bad = reinterpret_cast<unsigned long long*>(p);
  rs->n_oob = reinterpret_cast<uint64_t*>(p + 64);
  rs->counts = reinterpret_cast<unsigned long long*>(p + 256);
  p += sz_misc;
  uint16_t* bucket_d = reinterpret_cast<uint16_t*>(p);
  uint16_t* bucket_w_d = reinterpret_cast<uint16_t*>(p + sz_bk / 2);
  p += sz_bk;
  rs->ragged = reinterpret_cast<uint32_t*>(p);
  rs->n_ragged = (uint32_t)ragged.size();
  // Bucket index over [lowest base, highest end): the last fence at or below
  // each bucket's first address, for a table of every stride-th range.
  const uint64_t lo = n ? ranges[0].base : 0, span = n ? ranges[n - 1].base + ranges[n - 1].size - lo : 0;
  uint32_t shift = 12;
  while (span > 0 && ((span - 1) >> shift) >= kBuckets) ++shift;
  auto fence_stride = [&](uint32_t cap) { return n <= cap ? 1u : (n + cap - 1) / cap; };
  auto bucket_index = [&](uint32_t stride, uint32_t n_fence) {
    std::vector<uint16_t> bucket(kBuckets, 0);
    for (uint32_t b = 0, i = 0; b < kBuckets && n > 0; ++b) {
      const uint64_t start = (uint64_t)b << shift;  // offset from lo
      while (i + 1 < n_fence && ranges[(uint64_t)(i + 1) * stride].base - lo <= start) ++i;
      bucket[b] = (uint16_t)i;
    }
    return bucket;
  };
  const uint32_t stride = fence_stride(kFences), stride_w = fence_stride(kWideFences);
  const uint32_t n_fence = n == 0 ? 0u : (n + stride - 1) / stride;
  const uint32_t n_fence_w = n == 0 ? 0u : (n + stride_w - 1) / stride_w;
  const std::vector<uint16_t> bucket = bucket_index(stride, n_fence), bucket_w = bucket_index(stride_w, n_fence_w);

  auto fail = [&](const char* what, hipError_t err) {
    set_error(what, err);
    (void)hipFree(rs->dev);
    delete rs;
    return KC_EHIP;
  };
  if (!tiles.empty() && (e = hipMemcpy(rs->tiles, tiles.data(), sizeof(Tile) * tiles.size(),
                                       hipMemcpyHostToDevice)) != hipSuccess)
    return fail("hipMemcpy(tiles)", e);
  if (!scan_tiles.empty() && (e = hipMemcpy(rs->scan_tiles, scan_tiles.data(), sizeof(Tile) * scan_tiles.size(),
                                            hipMemcpyHostToDevice)) != hipSuccess)
    return fail("hipMemcpy(scan tiles)", e);
  if (!deep_tiles.empty() && (e = hipMemcpy(rs->deep_tiles, deep_tiles.data(), sizeof(Tile) * deep_tiles.size(),
                                            hipMemcpyHostToDevice)) != hipSuccess)
    return fail("hipMemcpy(pipelined pass tiles)", e);
  if (n > 0) {
    if ((e = hipMemcpy(rs->bases, bases.data(), 8 * n, hipMemcpyHostToDevice)) != hipSuccess)
      return fail("hipMemcpy(bases)", e);
    if ((e = hipMemcpy(rs->ends, ends.data(), 8 * n, hipMemcpyHostToDevice)) != hipSuccess)
      return fail("hipMemcpy(ends)", e);
  }
  if ((e = hipMemset(rs->n_bad, 0, sz_misc)) != hipSuccess) return fail("hipMemset(counts)", e);
  if ((e = hipMemcpy(bucket_d, bucket.data(), sizeof(uint16_t) * kBuckets, hipMemcpyHostToDevice)) != hipSuccess)
    return fail("hipMemcpy(bucket index)", e);
  if ((e = hipMemcpy(bucket_w_d, bucket_w.data(), sizeof(uint16_t) * kBuckets, hipMemcpyHostToDevice)) !=
      hipSuccess)
    return fail("hipMemcpy(bucket index)", e);
  if (!ragged.empty() &&
      (e = hipMemcpy(rs->ragged, ragged.data(), 4 * ragged.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return fail("hipMemcpy(ragged tiles)", e);
  rs->rt.base = rs->bases;
  rs->rt.end = rs->ends;
  rs->rt.bucket = bucket_d;
  rs->rt.lo = lo;
  rs->rt.span = span;
  rs->rt.n = n;
  rs->rt.stride = stride;
  rs->rt.n_fence = n_fence;
  rs->rt.shift = shift;
  rs->rt.bucket_w = bucket_w_d;
  rs->rt.stride_w = stride_w;
  rs->rt.n_fence_w = n_fence_w;
  *out = rs;
  if (n_units_out) *n_units_out = n_units;
  return KC_OK;
}

void kc_rangeset_destroy(kc_rangeset* rs) {
  if (rs == nullptr) return;
  DeviceGuard g(rs->device);
  (void)hipFree(rs->dev);
  delete rs;
}

// The standalone closure scan over the 4 KiB page tiles (one launch, or one
// per range); the caller has cleared the scan totals.
static int run_closure(kc_rangeset* rs, const ScanDev& sd, hipStream_t s) {
  kc_ctx* c = rs->ctx;
  const uint32_t grid = grid_for(c, KC_OP_CLOSURE, 8);
  KernelTimer timer(c, KC_OP_CLOSURE, s);
  if (!c->tune[KC_OP_CLOSURE].per_item) {
    KC_HIP(launch_closure(rs->scan_tiles, rs->n_scan_tiles, 0, sd, grid, c->n_cu, s));
  } else {
    for (uint32_t r = 0; r < rs->n_ranges; ++r) {
      const uint32_t t0 = rs->scan_range_tile[r];
      KC_HIP(launch_closure(rs->scan_tiles + t0, rs->scan_range_tile[r + 1] - t0, t0, sd, grid, c->n_cu, s));
    }
  }
  return KC_OK;
}

// Launch the page-hash kernel over all tiles, or once per range.
static int run_hash(kc_rangeset* rs, HashParams hp, bool gather, bool prior, bool scan, uint32_t op,
                    hipStream_t s) {
  kc_ctx* c = rs->ctx;
  KernelTimer timer(c, op, s);
  // read-only hashing runs best with twice the waves of the fused snapshot (which also writes and scans)
  uint32_t grid = grid_for(c, op, op == KC_OP_PAGE_HASH ? 8 : 4);
  uint32_t depth = c->tune[op].depth;
  if (depth == 0u && rs->ushift > kMinUnitShift) depth = 2u;
  if (scan) depth = 1u;
  // the pipelined pass walks its own tiles
  const bool deep = depth > 1u;
  Tile* const tiles = deep ? rs->deep_tiles : rs->tiles;
  const std::vector<uint32_t>& range_tile = deep ? rs->deep_range_tile : rs->range_tile;
  // large units give few tiles, each a long serial chain: one wave per tile rather than two tiles on some
  // waves, each wave keeping two chunks in flight in the skewed pass (three or four measured no faster)
  if (rs->ushift > kMinUnitShift) grid = std::max(grid, std::min(deep ? rs->n_deep_tiles : rs->n_tiles, 16u * c->n_cu));
  hp.ushift = rs->ushift;
  if (!c->tune[op].per_item) {
    hp.tiles = tiles;
    hp.n_tiles = deep ? rs->n_deep_tiles : rs->n_tiles;
    hp.tile0 = 0;
    hp.ragged = rs->ragged;
    hp.n_ragged = rs->n_ragged;
    KC_HIP(launch_page_hash(hp, gather, prior, scan, depth, grid, c->n_cu, s));
    return KC_OK;
  }
  for (uint32_t r = 0; r < rs->n_ranges; ++r) {
    hp.tile0 = range_tile[r];
    hp.tiles = tiles + hp.tile0;
    hp.n_tiles = range_tile[r + 1] - hp.tile0;
    const bool rg = rs->ragged_of[r] != UINT32_MAX;
    hp.ragged = rg ? rs->ragged + rs->ragged_of[r] : nullptr;
    hp.n_ragged = rg ? 1u : 0u;
    KC_HIP(launch_page_hash(hp, gather, prior, scan, depth, grid, c->n_cu, s));
  }
  return KC_OK;
}

int kc_page_hash(kc_ctx* c, const kc_rangeset* crs, uint64_t seed, const uint64_t* prior_hash_d, uint64_t* hash_d,
                 uint64_t* zero_bm_d, uint64_t* changed_bm_d, const kc_scan_args* scan, void* stream) {
  kc_rangeset* rs = const_cast<kc_rangeset*>(crs);
  if (c == nullptr || rs == nullptr || rs->ctx != c) return KC_EINVAL;
  if (rs->n_pages > 0 && (hash_d == nullptr || zero_bm_d == nullptr)) return KC_EINVAL;
  if (prior_hash_d != nullptr && changed_bm_d == nullptr) return KC_EINVAL;
  ScanDev sd{};
  if (scan) {
    const int st = make_scan(rs, scan, &sd);
    if (st != KC_OK) return st;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = as_stream(stream);
  KC_HIP(launch_zero3(zero_bm_d, rs->n_words, changed_bm_d, prior_hash_d ? rs->n_words : 0,
                      reinterpret_cast<uint64_t*>(rs->counts), scan ? kScanCountWords : 0, s));
  HashParams hp{};
  hp.seed = seed;
  hp.prior = prior_hash_d;
  hp.hash = hash_d;
  hp.zero_bm = zero_bm_d;
  hp.changed_bm = changed_bm_d;
  hp.scan = sd;
  const bool fused = scan != nullptr && rs->ushift == kMinUnitShift;  // the scan rides on 4 KiB page tiles
  int st = run_hash(rs, hp, false, prior_hash_d != nullptr, fused, KC_OP_PAGE_HASH, s);
  if (st != KC_OK) return st;
  if (scan && !fused && (st = run_closure(rs, sd, s)) != KC_OK) return st;
  if (scan) return finish_scan(rs, scan, sd, s);
  return KC_OK;
}

int kc_compact(kc_ctx* c, const kc_rangeset* crs, const uint64_t* zero_bm_d, const uint64_t* changed_bm_d,
               void* packed_d, uint64_t* page_va_d, uint64_t cap_pages, uint64_t* n_kept_d, void* stream) {
  kc_rangeset* rs = const_cast<kc_rangeset*>(crs);
  if (c == nullptr || rs == nullptr || rs->ctx != c || n_kept_d == nullptr) return KC_EINVAL;
  if (rs->n_pages > 0 && zero_bm_d == nullptr) return KC_EINVAL;
  if (cap_pages > 0 && (packed_d == nullptr || page_va_d == nullptr)) return KC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = as_stream(stream);
  ScanSrc src{};
  src.kind = kSrcKeepBits;
  src.zero_bm = zero_bm_d;
  src.changed_bm = changed_bm_d;
  src.n_pages = rs->n_pages;
  src.n_items = rs->n_words;
  KC_HIP(launch_scan(src, rs->word_prefix, rs->block_sums, n_kept_d, s));
  const uint32_t grid = grid_for(c, KC_OP_COMPACT, 8);
  KernelTimer timer(c, KC_OP_COMPACT, s);
  if (!c->tune[KC_OP_COMPACT].per_item) {
    KC_HIP(launch_gather(rs->tiles, rs->n_tiles, zero_bm_d, changed_bm_d, rs->word_prefix,
                         static_cast<uint8_t*>(packed_d), page_va_d, cap_pages, rs->ushift, grid, s));
  } else {
    for (uint32_t r = 0; r < rs->n_ranges; ++r) {
      const uint32_t t0 = rs->range_tile[r];
      KC_HIP(launch_gather(rs->tiles + t0, rs->range_tile[r + 1] - t0, zero_bm_d, changed_bm_d,
                           rs->word_prefix, static_cast<uint8_t*>(packed_d), page_va_d, cap_pages, rs->ushift,
                           grid, s));
    }
  }
  return KC_OK;
}

int kc_snapshot(kc_ctx* c, const kc_rangeset* crs, uint64_t seed, const uint64_t* prior_hash_d, uint64_t* hash_d,
                uint64_t* zero_bm_d, uint64_t* changed_bm_d, void* packed_d, uint64_t* page_va_d,
                uint64_t cap_pages, uint64_t* n_kept_d, const kc_scan_args* scan, void* stream) {
  kc_rangeset* rs = const_cast<kc_rangeset*>(crs);
  if (c == nullptr || rs == nullptr || rs->ctx != c || n_kept_d == nullptr) return KC_EINVAL;
  if (rs->n_pages > 0 && (hash_d == nullptr || zero_bm_d == nullptr)) return KC_EINVAL;
  if (cap_pages > 0 && (packed_d == nullptr || page_va_d == nullptr)) return KC_EINVAL;
  if (prior_hash_d != nullptr) {
    const int st = kc_page_hash(c, rs, seed, prior_hash_d, hash_d, zero_bm_d, changed_bm_d, scan, stream);
    if (st != KC_OK) return st;
    return kc_compact(c, rs, zero_bm_d, changed_bm_d, packed_d, page_va_d, cap_pages, n_kept_d, stream);
  }
  ScanDev sd{};
  if (scan) {
    const int st = make_scan(rs, scan, &sd);
    if (st != KC_OK) return st;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = as_stream(stream);
  KC_HIP(launch_zero3(zero_bm_d, rs->n_words, nullptr, 0, reinterpret_cast<uint64_t*>(rs->counts),
                      scan ? kScanCountWords : 0, s));
  KC_HIP(launch_probe_zero(rs->tiles, rs->n_tiles, zero_bm_d, rs->ushift, grid_for(c, KC_OP_SNAPSHOT, 8), s));
  ScanSrc src{};
  src.kind = kSrcKeepBits;
  src.zero_bm = zero_bm_d;
  src.n_pages = rs->n_pages;
  src.n_items = rs->n_words;
  KC_HIP(launch_scan(src, rs->word_prefix, rs->block_sums, n_kept_d, s));
  HashParams hp{};
  hp.seed = seed;
  hp.hash = hash_d;
  hp.zero_bm = zero_bm_d;
  hp.word_prefix = rs->word_prefix;
  hp.packed = static_cast<uint8_t*>(packed_d);
  hp.page_va = page_va_d;
  hp.cap_pages = cap_pages;
  hp.scan = sd;
  const bool fused = scan != nullptr && rs->ushift == kMinUnitShift;  // the scan rides on 4 KiB page tiles
  int st = run_hash(rs, hp, true, false, fused, KC_OP_SNAPSHOT, s);
  if (st != KC_OK) return st;
  if (scan && !fused && (st = run_closure(rs, sd, s)) != KC_OK) return st;
  if (scan) return finish_scan(rs, scan, sd, s);
  return KC_OK;
}

int kc_restore(kc_ctx* c, const kc_rangeset* crs, const uint64_t* zero_bm_d, const uint64_t* changed_bm_d,
               const void* packed_d, const uint64_t* page_va_d, const uint64_t* n_kept_d, uint64_t cap_pages,
               uint64_t* n_bad_d, void* stream) {
  kc_rangeset* rs = const_cast<kc_rangeset*>(crs);
  if (c == nullptr || rs == nullptr || rs->ctx != c || n_kept_d == nullptr) return KC_EINVAL;
  if (rs->n_pages > 0 && zero_bm_d == nullptr) return KC_EINVAL;
  if (cap_pages > 0 && (packed_d == nullptr || page_va_d == nullptr)) return KC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = as_stream(stream);
  unsigned long long* bad = n_bad_d ? reinterpret_cast<unsigned long long*>(n_bad_d) : rs->n_bad;
  const uint32_t grid = grid_for(c, KC_OP_RESTORE, 16);
  KC_HIP(launch_restore_zero(rs->tiles, rs->n_tiles, zero_bm_d, changed_bm_d, bad, rs->ushift, grid, s));
  KernelTimer timer(c, KC_OP_RESTORE, s);
  KC_HIP(launch_restore_scatter(rs->rt, static_cast<const uint8_t*>(packed_d), page_va_d, n_kept_d, cap_pages,
                                bad, rs->n_ragged > 0, changed_bm_d != nullptr, rs->ushift, grid, s));
  return KC_OK;
}

int kc_region_diff(kc_ctx* c, const kc_rangeset* crs, uint64_t seed, const uint64_t* gold_hash_d,
                   const uint64_t* gold_zero_bm_d, const void* gold_packed_d, const uint64_t* gold_page_va_d,
                   const uint64_t* gold_n_kept_d, uint64_t cap_pages, uint64_t* cand_hash_d, uint64_t* cand_zero_bm_d,
                   uint64_t* changed_bm_d, kc_region_diff_result* res_d, void* stream) {
  kc_rangeset* rs = const_cast<kc_rangeset*>(crs);
  if (c == nullptr || rs == nullptr || rs->ctx != c) return KC_EINVAL;
  if (rs->n_ranges == 0) return KC_OK;
  if (res_d == nullptr || gold_n_kept_d == nullptr) return KC_EINVAL;
  if (rs->n_pages > 0 && (gold_hash_d == nullptr || gold_zero_bm_d == nullptr || cand_hash_d == nullptr ||
                          cand_zero_bm_d == nullptr || changed_bm_d == nullptr))
    return KC_EINVAL;
  if (cap_pages > 0 && (gold_packed_d == nullptr || gold_page_va_d == nullptr)) return KC_EINVAL;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = as_stream(stream);
  KC_HIP(launch_region_init(res_d, rs->n_ranges, cand_zero_bm_d, changed_bm_d, rs->n_words, s));
  HashParams hp{};
  hp.seed = seed;
  hp.prior = gold_hash_d;
  hp.hash = cand_hash_d;
  hp.zero_bm = cand_zero_bm_d;
  hp.changed_bm = changed_bm_d;
  int st = run_hash(rs, hp, false, true, false, KC_OP_PAGE_HASH, s);
  if (st != KC_OK) return st;
  ScanSrc src{};  // rank of each non-zero snapshot page: keep prefix of the gold zero bitmap
  src.kind = kSrcKeepBits;
  src.zero_bm = gold_zero_bm_d;
  src.n_pages = rs->n_pages;
  src.n_items = rs->n_words;
  KC_HIP(launch_scan(src, rs->word_prefix, rs->block_sums, rs->n_oob, s));
  KernelTimer timer(c, KC_OP_REGION_DIFF, s);
  KC_HIP(launch_region_diff(rs->tiles, rs->n_tiles, rs->rt, changed_bm_d, gold_zero_bm_d, rs->word_prefix,
                            gold_page_va_d, gold_n_kept_d, cap_pages, static_cast<const uint8_t*>(gold_packed_d),
                            res_d, rs->ushift, grid_for(c, KC_OP_REGION_DIFF, 8), s));
  return KC_OK;
}

int kc_pointer_graph(kc_ctx* c, const kc_rangeset* rs, uint64_t win_lo, uint64_t win_hi, uint64_t* edge_bm_d,
                     void* stream) {
  if (c == nullptr || rs == nullptr || rs->ctx != c) return KC_EINVAL;
  if (rs->n_ranges > KC_GRAPH_MAX_RANGES) return KC_ELIMIT;
  if (rs->n_ranges == 0) return KC_OK;
  if (edge_bm_d == nullptr) return KC_EINVAL;
  uint64_t lo = win_lo, hi = win_hi;
  if (lo == 0 && hi == 0) {
    lo = rs->win_lo;
    hi = rs->win_hi;
  } else if (lo == 0 || lo >= hi) {
    return KC_EINVAL;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = as_stream(stream);
  const uint32_t row_words = (rs->n_ranges + 63u) / 64u;
  KC_HIP(launch_fill_u64(edge_bm_d, (uint64_t)rs->n_ranges * row_words, 0, s));
  KernelTimer timer(c, KC_OP_GRAPH, s);
  KC_HIP(launch_pointer_graph(rs->scan_tiles, rs->n_scan_tiles, lo, hi - lo, rs->rt, edge_bm_d, row_words,
                              grid_for(c, KC_OP_GRAPH, 8), c->n_cu, s));
  return KC_OK;
}

int kc_graph_reach(const kc_range* ranges, uint32_t n, const uint64_t* edge_bm, const uint64_t* root_words,
                   uint64_t n_root_words, uint64_t* reach_bm) {
  const int st = range_check(ranges, n, nullptr);
  if (st != KC_OK) return st;
  if (n > KC_GRAPH_MAX_RANGES) return KC_ELIMIT;
  if ((n > 0 && (edge_bm == nullptr || reach_bm == nullptr)) || (n_root_words > 0 && root_words == nullptr))
    return KC_EINVAL;
  if (n == 0) return KC_OK;
  const uint32_t rw = (n + 63u) / 64u;
  std::fill(reach_bm, reach_bm + rw, 0ull);
  std::vector<uint32_t> stack;
  stack.reserve(n);
  auto visit = [&](uint32_t r) {
    if (!((reach_bm[r >> 6] >> (r & 63u)) & 1ull)) {
      reach_bm[r >> 6] |= 1ull << (r & 63u);
      stack.push_back(r);
    }
  };
  for (uint64_t i = 0; i < n_root_words; ++i) {  // the range each root word lies in
    const uint64_t w = root_words[i];
    const kc_range* it = std::upper_bound(ranges, ranges + n, w,
                                          [](uint64_t v, const kc_range& r) { return v < r.base; });
    if (it != ranges && w - (it - 1)->base < (it - 1)->size) visit((uint32_t)(it - 1 - ranges));
  }
  while (!stack.empty()) {  // depth-first over the rows, a word of targets at a time
    const uint32_t a = stack.back();
    stack.pop_back();
    const uint64_t* row = edge_bm + (uint64_t)a * rw;
    for (uint32_t k = 0; k < rw; ++k) {
      uint64_t fresh = row[k] & ~reach_bm[k];
      if (k == rw - 1u && (n & 63u)) fresh &= (1ull << (n & 63u)) - 1ull;  // bits past the last range
      while (fresh) {
        visit(k * 64u + (uint32_t)__builtin_ctzll(fresh));
        fresh &= fresh - 1ull;
      }
    }
  }
  return KC_OK;
}

int kc_closure_scan(kc_ctx* c, const kc_rangeset* crs, const kc_scan_args* scan, void* stream) {
  kc_rangeset* rs = const_cast<kc_rangeset*>(crs);
  if (c == nullptr || rs == nullptr || rs->ctx != c || scan == nullptr) return KC_EINVAL;
  ScanDev sd{};
  const int st = make_scan(rs, scan, &sd);
  if (st != KC_OK) return st;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = as_stream(stream);
  KC_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(rs->counts), kScanCountWords, 0, s));
  const int rc = run_closure(rs, sd, s);
  if (rc != KC_OK) return rc;
  return finish_scan(rs, scan, sd, s);
}

}  // extern "C"


namespace kc {

uint32_t elem_size(uint32_t dtype) {
  switch (dtype) {
    case KC_F64: case KC_I64: return 8u;
    case KC_F32: case KC_I32: return 4u;
    case KC_BF16: case KC_F16: case KC_I16: return 2u;
    default: return 1u;
  }
}

// Tuned tile size, else 64 KiB halved (down to 16 KiB) while the pairs would
// give fewer than eight tiles per compute unit: small batches still spread
// over the whole chip.
uint32_t compare_tile_bytes(const kc_ctx* c, const kc_pair* pairs, uint32_t n_pairs) {
  if (c->tune[KC_OP_COMPARE].tile_bytes) return c->tune[KC_OP_COMPARE].tile_bytes;
  uint64_t total = 0;
  for (uint32_t i = 0; i < n_pairs; ++i)
    if (pairs[i].dtype <= KC_I64 && pairs[i].n_elems <= (1ull << 60)) total += pairs[i].n_elems * elem_size(pairs[i].dtype);
  uint32_t tb = 64u << 10;
  while (tb > (16u << 10) && total / tb < 8ull * c->n_cu) tb >>= 1;
  return tb;
}

}  // namespace kc

namespace {

// Validate a pair list and count its tiles.
int plan_pairs(const kc_pair* pairs, uint32_t n_pairs, uint32_t tile_bytes, std::vector<uint64_t>& tile_off) {
  tile_off.assign(n_pairs + 1, 0);
  for (uint32_t i = 0; i < n_pairs; ++i) {
    const kc_pair& pr = pairs[i];
    if (pr.dtype > KC_I64) return KC_EDTYPE;
    if (pr.n_elems > (1ull << 60)) return KC_ELIMIT;
    if (!(pr.atol >= 0.0) || !(pr.rtol >= 0.0)) return KC_EINVAL;  // negative or NaN tolerances
    if (pr.n_elems > 0) {
      if (pr.cand_d == nullptr || pr.gold_d == nullptr) return KC_EINVAL;
      // element-aligned buffers; those not 16-byte aligned take the element-wise path
      if ((reinterpret_cast<uintptr_t>(pr.cand_d) | reinterpret_cast<uintptr_t>(pr.gold_d)) & (elem_size(pr.dtype) - 1u))
        return KC_EALIGN;
    }
    const uint64_t nb = pr.n_elems * elem_size(pr.dtype);
    const uint64_t nt = nb == 0 ? 1 : (nb + tile_bytes - 1) / tile_bytes;
    tile_off[i + 1] = tile_off[i] + nt;
  }
  if (tile_off[n_pairs] > 0xFFFFFFFFull) return KC_ELIMIT;
  return KC_OK;
}

// Fill the device-layout pair and tile tables (host memory).
void fill_pair_tables(const kc_pair* pairs, uint32_t n_pairs, const std::vector<uint64_t>& tile_off,
                      CmpPairDev* hp, CmpTileDev* ht) {
  for (uint32_t i = 0; i < n_pairs; ++i) {
    const kc_pair& pr = pairs[i];
    CmpPairDev d;
    d.cand = static_cast<const uint8_t*>(pr.cand_d);
    d.gold = static_cast<const uint8_t*>(pr.gold_d);
    d.n_elems = pr.n_elems;
    d.dtype = pr.dtype;
    d.tol = pr.ulp_tol;
    d.n_tiles = (uint32_t)(tile_off[i + 1] - tile_off[i]);
    d.esize = elem_size(pr.dtype);
    d.atol = pr.atol;
    d.rtol = pr.rtol;
    hp[i] = d;
    for (uint64_t t = tile_off[i]; t < tile_off[i + 1]; ++t) {
      ht[t].pair = i;
      ht[t].idx = (uint32_t)(t - tile_off[i]);
    }
  }
}

// Run the pass (one launch, or one per pair), write the reports.  The
// accumulators are zero on entry and the finalize kernel zeroes them again.
// A call that failed between the pass and the finalize leaves *acc_dirty set;
// the next call clears the whole accumulator area first (fill kernel, so the
// call stays capturable).
int run_compare(kc_ctx* c, const CmpPairDev* dpairs, const CmpTileDev* dtiles, const std::vector<uint64_t>& tile_off,
                uint32_t n_pairs, uint32_t tile_bytes, unsigned long long* dacc, uint64_t acc_words, bool* acc_dirty,
                kc_cmp_result* res_d, hipStream_t s) {
  // built-in shape: 2 workgroups per CU, 4 when there are few tiles to share (a persistent grid reads the c4 pairs
  // 4 % faster than one workgroup per tile)
  const uint32_t grid = grid_for(c, KC_OP_COMPARE, tile_off[n_pairs] < 16ull * c->n_cu ? 4 : 2);
  if (*acc_dirty) KC_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(dacc), acc_words, 0, s));
  *acc_dirty = true;
  {
    KernelTimer timer(c, KC_OP_COMPARE, s);
    if (!c->tune[KC_OP_COMPARE].per_item) {
      KC_HIP(launch_compare(dpairs, dtiles, (uint32_t)tile_off[n_pairs], tile_bytes, dacc, grid, s));
    } else {
      for (uint32_t i = 0; i < n_pairs; ++i)
        KC_HIP(launch_compare(dpairs, dtiles + tile_off[i], (uint32_t)(tile_off[i + 1] - tile_off[i]), tile_bytes,
                              dacc, grid, s));
    }
  }
  KC_HIP(launch_compare_finalize(dpairs, n_pairs, dacc, res_d, s));
  *acc_dirty = false;
  return KC_OK;
}

}  // namespace

extern "C" {

int kc_compare(kc_ctx* c, const kc_pair* pairs, uint32_t n_pairs, kc_cmp_result* res_d, void* stream) {
  if (c == nullptr || (n_pairs > 0 && (pairs == nullptr || res_d == nullptr))) return KC_EINVAL;
  if (n_pairs == 0) return KC_OK;
  const uint32_t tile_bytes = compare_tile_bytes(c, pairs, n_pairs);
  std::vector<uint64_t> tile_off;
  int st = plan_pairs(pairs, n_pairs, tile_bytes, tile_off);
  if (st != KC_OK) return st;
  const uint64_t n_tiles = tile_off[n_pairs];
  const size_t sz_pairs = align_up(sizeof(CmpPairDev) * n_pairs, 256);
  const size_t sz_tiles = align_up(sizeof(CmpTileDev) * n_tiles, 256);
  const size_t sz_acc = (size_t)n_pairs * kAccWords * 8;
  const size_t need_dev = sz_pairs + sz_tiles, need_host = sz_pairs + sz_tiles;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  const hipStream_t s = as_stream(stream);
  if (c->staged_pending) {
    KC_HIP(hipEventSynchronize(c->staged));  // the staging buffer is free again
    c->staged_pending = false;
  }
  if (need_dev > c->cmp_dev_cap) {
    KC_HIP(hipStreamSynchronize(s));
    const size_t cap = std::max(need_dev, c->cmp_dev_cap * 2);
    if (c->cmp_dev) KC_HIP(hipFree(c->cmp_dev));
    c->cmp_dev = nullptr;
    c->cmp_dev_cap = 0;
    hipError_t e = hipMalloc(&c->cmp_dev, cap);
    if (e != hipSuccess) {
      set_error("hipMalloc(compare scratch)", e);
      return e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
    }
    c->cmp_dev_cap = cap;
  }
  if (sz_acc > c->cmp_acc_cap) {
    KC_HIP(hipStreamSynchronize(s));
    const size_t cap = std::max(sz_acc, c->cmp_acc_cap * 2);
    if (c->cmp_acc) KC_HIP(hipFree(c->cmp_acc));
    c->cmp_acc = nullptr;
    c->cmp_acc_cap = 0;
    hipError_t e = hipMalloc(&c->cmp_acc, cap);
    if (e != hipSuccess) {
      set_error("hipMalloc(compare accumulators)", e);
      return e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
    }
    KC_HIP(hipMemset(c->cmp_acc, 0, cap));
    c->cmp_acc_cap = cap;
    c->cmp_acc_dirty = false;
  }
  if (need_host > c->cmp_host_cap) {
    if (c->cmp_host) KC_HIP(hipHostFree(c->cmp_host));
    c->cmp_host = nullptr;
    c->cmp_host_cap = 0;
    const size_t cap = std::max(need_host, (size_t)1 << 20);
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->cmp_host), cap, hipHostMallocDefault);
    if (e != hipSuccess) {
      set_error("hipHostMalloc(compare staging)", e);
      return KC_ENOMEM;
    }
    c->cmp_host_cap = cap;
  }
  fill_pair_tables(pairs, n_pairs, tile_off, reinterpret_cast<CmpPairDev*>(c->cmp_host),
                   reinterpret_cast<CmpTileDev*>(c->cmp_host + sz_pairs));
  CmpPairDev* dpairs = reinterpret_cast<CmpPairDev*>(c->cmp_dev);
  CmpTileDev* dtiles = reinterpret_cast<CmpTileDev*>(c->cmp_dev + sz_pairs);
  unsigned long long* dacc = c->cmp_acc;
  KC_HIP(hipMemcpyAsync(c->cmp_dev, c->cmp_host, need_host, hipMemcpyHostToDevice, s));
  KC_HIP(hipEventRecord(c->staged, s));
  c->staged_pending = true;
  return run_compare(c, dpairs, dtiles, tile_off, n_pairs, tile_bytes, dacc, c->cmp_acc_cap / 8, &c->cmp_acc_dirty,
                     res_d, s);
}

int kc_pairset_create(kc_ctx* c, const kc_pair* pairs, uint32_t n_pairs, kc_pairset** out) {
  if (c == nullptr || out == nullptr || (n_pairs > 0 && pairs == nullptr)) return KC_EINVAL;
  *out = nullptr;
  const uint32_t tile_bytes = compare_tile_bytes(c, pairs, n_pairs);
  std::vector<uint64_t> tile_off;
  int st = plan_pairs(pairs, n_pairs, tile_bytes, tile_off);
  if (st != KC_OK) return st;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  kc_pairset* ps = new (std::nothrow) kc_pairset();
  if (ps == nullptr) return KC_ENOMEM;
  ps->ctx = c;
  ps->device = c->device;
  ps->n_pairs = n_pairs;
  ps->tile_bytes = tile_bytes;
  ps->n_tiles = tile_off[n_pairs];
  ps->tile_off = std::move(tile_off);
  const size_t sz_pairs = align_up(sizeof(CmpPairDev) * std::max<uint32_t>(1, n_pairs), 256);
  const size_t sz_tiles = align_up(sizeof(CmpTileDev) * std::max<uint64_t>(1, ps->n_tiles), 256);
  const size_t sz_acc = (size_t)std::max<uint32_t>(1, n_pairs) * kAccWords * 8;
  hipError_t e = hipMalloc(&ps->dev, sz_pairs + sz_tiles + sz_acc);
  if (e != hipSuccess) {
    set_error("hipMalloc(pairset)", e);
    delete ps;
    return e == hipErrorOutOfMemory ? KC_ENOMEM : KC_EHIP;
  }
  uint8_t* base = static_cast<uint8_t*>(ps->dev);
  ps->pairs = reinterpret_cast<CmpPairDev*>(base);
  ps->tiles = reinterpret_cast<CmpTileDev*>(base + sz_pairs);
  ps->acc = reinterpret_cast<unsigned long long*>(base + sz_pairs + sz_tiles);
  std::vector<uint8_t> host(sz_pairs + sz_tiles);
  fill_pair_tables(pairs, n_pairs, ps->tile_off, reinterpret_cast<CmpPairDev*>(host.data()),
                   reinterpret_cast<CmpTileDev*>(host.data() + sz_pairs));
  if ((e = hipMemcpy(ps->dev, host.data(), host.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(ps->acc, 0, sz_acc)) != hipSuccess) {
    set_error("hipMemcpy(pairset)", e);
    (void)hipFree(ps->dev);
    delete ps;
    return KC_EHIP;
  }
  *out = ps;
  return KC_OK;
}

void kc_pairset_destroy(kc_pairset* ps) {
  if (ps == nullptr) return;
  DeviceGuard g(ps->device);
  (void)hipFree(ps->dev);
  delete ps;
}

int kc_compare_pairset(kc_ctx* c, const kc_pairset* ps, kc_cmp_result* res_d, void* stream) {
  if (c == nullptr || ps == nullptr || ps->ctx != c || (ps->n_pairs > 0 && res_d == nullptr)) return KC_EINVAL;
  if (ps->n_pairs == 0) return KC_OK;
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  return run_compare(c, ps->pairs, ps->tiles, ps->tile_off, ps->n_pairs, ps->tile_bytes, ps->acc,
                     (uint64_t)ps->n_pairs * kAccWords, &ps->acc_dirty, res_d, as_stream(stream));
}

}  // extern "C"

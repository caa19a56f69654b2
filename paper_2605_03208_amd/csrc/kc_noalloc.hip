// kc_noalloc.hip -- the compare for callers that cannot allocate (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// kc_compare keeps its pair table, tile list and per-pair accumulators in
// context memory that it grows with hipMalloc and stages through pinned host
// memory.  kc_compare_noalloc computes the same reports with neither: the pair
// records travel in kernel arguments (kArgPairs per launch, the tile of a
// workgroup found by a search over their tile prefix), and the accumulators
// live in `scratch`, a static device array of a fixed size.  Its device
// address is looked up once per device when a context is created on it; host
// code only ever passes that address, never the array's own name.
#include <algorithm>
#include <atomic>
#include <mutex>

#include "kc_internal.h"

// Per-pair accumulators of kc_compare_noalloc: KC_NOALLOC_MAX_PAIRS pairs of
// kc::kAccWords u64 words (2 MiB), one copy per device, zero at load.
static __device__ __align__(256) unsigned long long scratch[(uint64_t)KC_NOALLOC_MAX_PAIRS * kc::kAccWords];

namespace kc {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_bind_mu;
std::atomic<unsigned long long*> g_scratch[kMaxDevices];

}  // namespace

int noalloc_bind(int device) {
  if (device < 0 || device >= kMaxDevices) {
    set_error_text("device index beyond the table of static compare scratch addresses");
    return KC_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_bind_mu);
  if (g_scratch[device].load() != nullptr) return KC_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    set_error("hipGetSymbolAddress(scratch)", e);
    return KC_EHIP;
  }
  g_scratch[device].store(static_cast<unsigned long long*>(p));
  return KC_OK;
}

}  // namespace kc

using namespace kc;

extern "C" {

int kc_compare_noalloc(kc_ctx* c, const kc_pair* pairs, uint32_t n_pairs, kc_cmp_result* res_d, void* stream) {
  if (c == nullptr || (n_pairs > 0 && (pairs == nullptr || res_d == nullptr))) return KC_EINVAL;
  if (n_pairs == 0) return KC_OK;
  if (n_pairs > KC_NOALLOC_MAX_PAIRS) {
    set_error_text("kc_compare_noalloc: more pairs than KC_NOALLOC_MAX_PAIRS (the static scratch holds 4096)");
    return KC_ELIMIT;
  }
  const uint32_t tile_bytes = compare_tile_bytes(c, pairs, n_pairs);
  // the checks of kc_compare, pair by pair, before anything is launched
  uint64_t chunk_tiles = 0;
  for (uint32_t i = 0; i < n_pairs; ++i) {
    const kc_pair& pr = pairs[i];
    if (pr.dtype > KC_I64) return KC_EDTYPE;
    if (pr.n_elems > (1ull << 60)) return KC_ELIMIT;
    if (!(pr.atol >= 0.0) || !(pr.rtol >= 0.0)) return KC_EINVAL;
    if (pr.n_elems > 0) {
      if (pr.cand_d == nullptr || pr.gold_d == nullptr) return KC_EINVAL;
      // element-aligned buffers; those not 16-byte aligned take the element-wise path
      if ((reinterpret_cast<uintptr_t>(pr.cand_d) | reinterpret_cast<uintptr_t>(pr.gold_d)) & (elem_size(pr.dtype) - 1u))
        return KC_EALIGN;
    }
    if (i % kArgPairs == 0) chunk_tiles = 0;
    const uint64_t nb = pr.n_elems * elem_size(pr.dtype);
    chunk_tiles += nb == 0 ? 1 : (nb + tile_bytes - 1) / tile_bytes;
    if (chunk_tiles > 0xFFFFFFFFull) return KC_ELIMIT;
  }
  DeviceGuard g(c->device);
  if (!g.ok) return KC_EHIP;
  unsigned long long* const acc = c->device >= 0 && c->device < kMaxDevices ? g_scratch[c->device].load() : nullptr;
  if (acc == nullptr) {
    set_error_text("the static compare scratch of this device was never bound");
    return KC_EHIP;
  }
  const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the accumulators this call uses start at zero whatever an earlier call left (fill kernel: capturable)
  KC_HIP(launch_fill_u64(reinterpret_cast<uint64_t*>(acc), (uint64_t)n_pairs * kAccWords, 0, s));
  for (uint32_t b0 = 0; b0 < n_pairs; b0 += kArgPairs) {
    CmpArgPairs a{};
    a.n = std::min(kArgPairs, n_pairs - b0);
    uint64_t t = 0;
    for (uint32_t j = 0; j < a.n; ++j) {
      const kc_pair& pr = pairs[b0 + j];
      const uint64_t nb = pr.n_elems * elem_size(pr.dtype);
      const uint64_t nt = nb == 0 ? 1 : (nb + tile_bytes - 1) / tile_bytes;
      CmpPairDev& d = a.pair[j];
      d.cand = static_cast<const uint8_t*>(pr.cand_d);
      d.gold = static_cast<const uint8_t*>(pr.gold_d);
      d.n_elems = pr.n_elems;
      d.dtype = pr.dtype;
      d.tol = pr.ulp_tol;
      d.n_tiles = (uint32_t)nt;
      d.esize = elem_size(pr.dtype);
      d.atol = pr.atol;
      d.rtol = pr.rtol;
      t += nt;
      a.tile_end[j] = (uint32_t)t;
    }
    a.n_tiles = (uint32_t)t;
    const uint32_t grid = grid_for(c, KC_OP_COMPARE, t < 16ull * c->n_cu ? 4 : 2);
    KC_HIP(launch_compare_args(a, tile_bytes, acc + (uint64_t)b0 * kAccWords, res_d + b0, grid, s));
  }
  return KC_OK;
}

}  // extern "C"

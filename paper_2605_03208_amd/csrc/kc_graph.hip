// kc_graph.hip -- gfx950 kernels over the ranges beyond the snapshot itself:
// the pointer graph between ranges and the per-range byte difference against
// a snapshot.  Same execution model as the snapshot kernels: persistent grids
// of 64-lane waves over the 16-page tile list, range fences in LDS (the graph:
// up to eight waves per workgroup sharing the wide table; the region diff:
// one wave per workgroup).
#include <algorithm>

#include "kc_device.h"
#include "kc_internal.h"

namespace kc {
namespace {

inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

// Pointer graph: for every pointer-like word, set bit (source range, target
// range).  Lanes of a wave that hit the same target share one atomicOr, and a
// wave skips the target it set last.
__device__ __forceinline__ void graph_emit(int32_t t, uint32_t lane, uint64_t* row, int32_t& last) {
  uint64_t pending = __ballot(t >= 0);
  while (pending) {
    const int32_t leader = __ffsll((long long)pending) - 1;
    const int32_t tb = __shfl(t, leader, 64);
    pending &= ~__ballot(t == tb);
    if (tb != last && (int32_t)lane == leader) atomicOr((unsigned long long*)&row[tb >> 6], 1ull << (tb & 63));
    last = tb;
  }
}

// Workgroups of kWideWaves independent waves share the wide range table.
__global__ __launch_bounds__(kWideWaves * kWave) __attribute__((amdgpu_waves_per_eu(4))) void k_pointer_graph(
    const Tile* tiles, uint32_t n_tiles, uint64_t lo, uint64_t span, RangeTable rt, uint64_t* edge_bm,
    uint32_t row_words) {
  const uint32_t lane = threadIdx.x % kWave, wpb = blockDim.x / kWave;
  const uint32_t wave = blockIdx.x * wpb + threadIdx.x / kWave, n_waves = gridDim.x * wpb;
  load_wide_fences(rt, threadIdx.x, blockDim.x);
  __syncthreads();
  for (uint32_t t = wave; t < n_tiles; t += n_waves) {
    const Tile tile = tiles[t];
    const int32_t src = wide_range_index(tile.va, rt);  // the tile's own range (always found)
    uint64_t* row = edge_bm + (uint64_t)(src < 0 ? 0 : src) * row_words;
    int32_t last = -1;
    const uint32_t nseg = tile.npages * 4u;
    for (uint32_t s0 = 0; s0 < nseg; s0 += 8) {
      uint4 x[8];
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i)
        x[i] = (s0 + i < nseg) ? ld16nt(tile.va + (uint64_t)(s0 + i) * 1024u + lane * 16u) : make_uint4(0, 0, 0, 0);
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i) {
        const uint4 v = seg_words(tile, s0 + i, lane, x[i]);  // words wholly inside the range only
        const uint64_t w0 = ((uint64_t)v.y << 32) | v.x;
        const uint64_t w1 = ((uint64_t)v.w << 32) | v.z;
        const bool p0 = (w0 - lo) < span, p1 = (w1 - lo) < span;
        if (__ballot(p0 || p1) == 0ull || src < 0) continue;  // no pointer-like word here
        graph_emit(p0 ? wide_range_index(w0, rt) : -1, lane, row, last);
        graph_emit(p1 ? wide_range_index(w1, rt) : -1, lane, row, last);
      }
    }
  }
}

// Per-range byte difference against a full snapshot.  Pages are visited in
// order inside a tile; the snapshot slot of a non-zero page is its rank among
// the non-zero pages (prefix per bitmap word + popcount below its bit).
__global__ void k_region_init(kc_region_diff_result* res, uint32_t n, uint64_t* bm_a, uint64_t* bm_b, uint64_t n_words) {
  const uint64_t m = n > n_words ? n : n_words;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x) {
    if (i < n) {
      res[i].n_diff_bytes = 0;
      res[i].n_diff_pages = 0;
      res[i].first_diff_va = ~0ull;
      res[i].n_bad_pages = 0;
    }
    if (i < n_words) {
      bm_a[i] = 0;
      bm_b[i] = 0;
    }
  }
}

__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t x) {
  return (uint32_t)((x & 0xFFu) != 0u) + (uint32_t)((x & 0xFF00u) != 0u) + (uint32_t)((x & 0xFF0000u) != 0u) +
         (uint32_t)((x & 0xFF000000u) != 0u);
}

__device__ __forceinline__ void flush_region(kc_region_diff_result* res, int32_t a, uint64_t dbytes, uint64_t dpages,
                                             uint64_t first) {
  if (a < 0 || dbytes == 0) return;
  kc_region_diff_result* r = res + a;
  atomicAdd((unsigned long long*)&r->n_diff_bytes, (unsigned long long)dbytes);
  atomicAdd((unsigned long long*)&r->n_diff_pages, (unsigned long long)dpages);
  atomicMin((unsigned long long*)&r->first_diff_va, (unsigned long long)first);
}

// A wave takes four consecutive tiles at a time, one lane per page: each lane
// resolves its page's snapshot copy and changed bit, then the whole wave
// compares the changed pages one after another (ascending).  Each wave owns a
// contiguous run of tile groups and folds its pages per range, touching a
// range's counters only when it moves to the next range or ends: waves that
// all add into one range's counters as they go queue on those addresses.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_region_diff(
    const Tile* tiles, uint32_t n_tiles, RangeTable rt, const uint64_t* changed_bm, const uint64_t* gold_zero_bm,
    const uint64_t* rank_prefix, const uint64_t* gold_page_va, const uint64_t* gold_n_kept, uint64_t cap,
    const uint8_t* gold_packed, kc_region_diff_result* res, uint32_t ushift) {
  __shared__ FenceLds fences;
  const uint32_t lane = threadIdx.x, sub = lane >> 4, j = lane & 15u;
  const uint32_t unit = 1u << ushift;
  load_fences(fences, rt, lane, kWave);
  __syncthreads();
  const uint64_t kept = *gold_n_kept;
  const uint64_t n_valid = kept < cap ? kept : cap;
  const uint32_t n_groups = (n_tiles + 3u) / 4u;
  const uint32_t per_wave = (n_groups + gridDim.x - 1u) / gridDim.x;
  const uint32_t gbeg = min(blockIdx.x * per_wave, n_groups), gend = min(gbeg + per_wave, n_groups);
  int32_t cur = -1;  // the range being folded, and its totals so far
  uint64_t dbytes = 0, dpages = 0, first = ~0ull;
  for (uint32_t gi = gbeg; gi < gend; ++gi) {
    const uint32_t t = gi * 4u + sub;
    Tile tile{0, 0, 0};
    if (t < n_tiles) tile = tiles[t];
    const bool live = j < tile.npages;
    const uint64_t g = (uint64_t)tile.g + j, va = tile.va + ((uint64_t)j << ushift);
    bool zero = false, bad = false, need = false;
    uint64_t gp = 0;
    int32_t a = -1;
    const uint32_t len = live ? unit_bytes(tile, j, unit) : 0u;
    if (live) {
      a = range_index(va, fences, rt);
      const uint64_t zw = gold_zero_bm[g >> 6];
      zero = (zw >> (g & 63u)) & 1ull;
      if (!zero) {
        const uint64_t slot = rank_prefix[g >> 6] + (uint64_t)__popcll(~zw & ((1ull << (g & 63u)) - 1ull));
        bad = slot >= n_valid || gold_page_va[slot] != va;
        gp = (uint64_t)gold_packed + (slot << ushift);
      }
      need = !bad && ((changed_bm[g >> 6] >> (g & 63u)) & 1ull);
    }
    const uint64_t bad_mask = __ballot(bad);
    if (j == 0u && live && a >= 0) {  // the 16 lanes of a tile share its range
      const uint32_t nb = (uint32_t)__popcll((bad_mask >> (16u * sub)) & 0xFFFFull);
      if (nb) atomicAdd((unsigned long long*)&res[a].n_bad_pages, (unsigned long long)nb);
    }
    uint64_t need_mask = __ballot(need);
    while (need_mask) {
      const int32_t L = __ffsll((long long)need_mask) - 1;
      need_mask &= need_mask - 1ull;
      const uint64_t pva = __shfl((unsigned long long)va, L, 64);
      const uint64_t pgp = __shfl((unsigned long long)gp, L, 64);
      const int32_t pz = __shfl((int)zero, L, 64);
      const int32_t pa = __shfl(a, L, 64);
      const uint32_t plen = __shfl(len, L, 64);  // bytes of the unit (a range's last unit may be partial)
      uint32_t nd = 0, fo = ~0u;
      for (uint32_t o0 = 0; o0 < plen; o0 += kPage) {  // 4 KiB of the unit per round, in address order
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) {
          const uint32_t off = o0 + k * 1024u + lane * 16u;
          const uint4 c = off < plen ? clip16(ld16nt(pva + off), off, plen) : make_uint4(0, 0, 0, 0);
          const uint4 d = pz || off >= plen ? make_uint4(0, 0, 0, 0) : clip16(ld16nt(pgp + off), off, plen);
          const uint32_t x[4] = {c.x ^ d.x, c.y ^ d.y, c.z ^ d.z, c.w ^ d.w};
#pragma unroll
          for (uint32_t i = 0; i < 4; ++i) {
            nd += nonzero_bytes(x[i]);
            if (x[i] != 0u && fo == ~0u) fo = off + 4u * i + ((uint32_t)__builtin_ctz(x[i]) >> 3);
          }
        }
      }
      nd = wave_sum_u32(nd);
#pragma unroll
      for (int dd = 32; dd >= 1; dd >>= 1) {
        const uint32_t y = __shfl_xor(fo, dd, 64);
        fo = y < fo ? y : fo;
      }
      if (pa != cur) {
        if (lane == 0) flush_region(res, cur, dbytes, dpages, first);
        cur = pa;
        dbytes = dpages = 0;
        first = ~0ull;
      }
      if (nd) {
        dbytes += nd;
        ++dpages;
        if (first == ~0ull) first = pva + fo;  // pages ascend within a range
      }
    }
  }
  if (lane == 0) flush_region(res, cur, dbytes, dpages, first);
}

}  // namespace

hipError_t launch_pointer_graph(const Tile* tiles, uint32_t n_tiles, uint64_t lo, uint64_t span,
                                const RangeTable& rt, uint64_t* edge_bm, uint32_t row_words, uint32_t grid,
                                uint32_t n_cu, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  uint32_t blocks = 1, wpb = 1;
  wide_shape(std::min(grid, n_tiles), n_cu, &blocks, &wpb);  // grid counts waves
  hipLaunchKernelGGL(k_pointer_graph, dim3(blocks), dim3(wpb * kWave), wide_lds_bytes(rt), s, tiles, n_tiles, lo,
                     span, rt, edge_bm, row_words);
  return hipGetLastError();
}

hipError_t launch_region_init(kc_region_diff_result* res, uint32_t n, uint64_t* bm_a, uint64_t* bm_b, uint64_t n_words,
                              hipStream_t s) {
  const uint64_t m = std::max<uint64_t>(n, n_words);
  if (m == 0) return hipSuccess;
  const uint64_t nbk = blocks_for(m, 256);
  hipLaunchKernelGGL(k_region_init, dim3((uint32_t)(nbk < 4096 ? nbk : 4096)), dim3(256), 0, s, res, n, bm_a, bm_b,
                     n_words);
  return hipGetLastError();
}

hipError_t launch_region_diff(const Tile* tiles, uint32_t n_tiles, const RangeTable& rt, const uint64_t* changed_bm,
                              const uint64_t* gold_zero_bm, const uint64_t* rank_prefix, const uint64_t* gold_page_va,
                              const uint64_t* gold_n_kept, uint64_t cap, const uint8_t* gold_packed,
                              kc_region_diff_result* res, uint32_t ushift, uint32_t grid, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  grid = std::max(1u, std::min(grid, n_tiles));
  hipLaunchKernelGGL(k_region_diff, dim3(grid), dim3(64), 0, s, tiles, n_tiles, rt, changed_bm, gold_zero_bm,
                     rank_prefix, gold_page_va, gold_n_kept, cap, gold_packed, res, ushift);
  return hipGetLastError();
}

}  // namespace kc

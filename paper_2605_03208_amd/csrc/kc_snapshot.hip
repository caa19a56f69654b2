// kc_snapshot.hip -- gfx950 kernels of the snapshot, restore and closure scan.
//
// Memory-bound streaming kernels: persistent grids of 64-lane waves striding
// over a tile list (16 pages of one range per tile).  Most workgroups are one
// wave; the hash pass and the standalone scan put several independent waves in
// a workgroup to share one range table, and the out-of-range emission uses one
// wave per page of a tile.  Global traffic is 16-byte loads / stores that
// cover whole 512-byte or 1-KiB runs; the XXH64 lanes read their words from a
// padded LDS stage.
#include <algorithm>

#include "kc_device.h"
#include "kc_internal.h"
#include "kc_xxh64.h"

namespace kc {
namespace {

// --------------------------------------------------------------- fill -----
__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Zero up to three arrays in one launch (index space = their concatenation).
__global__ void k_zero3(uint64_t* a, uint64_t na, uint64_t* b, uint64_t nb, uint64_t* c, uint64_t nc) {
  const uint64_t n = na + nb + nc;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (i < na) a[i] = 0;
    else if (i < na + nb) b[i - na] = 0;
    else c[i - na - nb] = 0;
  }
}

// ---------------------------------------------------------- page hash -----
// One wave hashes a tile of up to 16 pages: lane quad q owns page q, lane k of
// the quad runs XXH64 accumulator k over the words 8k + 32s of each stripe s.
// The wave streams the tile in 8 chunks of 512 bytes per page: 8 loads of
// 16 bytes per lane (instruction j covers pages 2j and 2j+1 with 32 lanes
// each), the chunk goes to a padded LDS stage, and the quad lanes read their
// 16 words of the chunk from there.  While chunk c is hashed, the loads of
// chunk c+1 are in flight.
//
// GATHER: zero bits come from the probe, zero pages are not read (their hash
// is computed from zeros), kept pages are also stored to their packed slot.
// RAGGED = false: every tile whose pages are all whole (the hot path); RAGGED =
// true: only the tiles listed in p.ragged, whose last page is partial (at most
// one per range), with the bytes past the range's end masked out.
//
// A workgroup holds up to kHashWaves independent waves, each with its own
// stage; with the closure scan they share one wide range table in dynamic LDS.
template <bool GATHER, bool PRIOR, bool SCAN, bool RAGGED>
__global__ __launch_bounds__(kHashWaves * kWave) __attribute__((amdgpu_waves_per_eu(RAGGED ? 1 : (SCAN ? 3 : 4)))) void k_page_hash(
    HashParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t stage_all[kHashWaves][kTilePages * kStageStride];
  __shared__ uint64_t tail_all[kHashWaves][kTilePages][4];  // a partial page's bytes past its last whole stripe
  const uint32_t lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, wpb = blockDim.x / kWave;
  uint8_t* const stage = stage_all[wv];
  uint64_t(*const tail_lds)[4] = tail_all[wv];
  const uint32_t q = lane >> 2, k = lane & 3u;
  const uint32_t half = lane >> 5, off16 = (lane & 31u) * 16u;
  const uint64_t scan_lo = p.scan.lo, scan_span = p.scan.span;
  const uint32_t ushift = p.ushift, unit = 1u << ushift;  // hash unit: 4 KiB .. 2 MiB
  const uint32_t n_chunks = unit / kChunk;
  if (SCAN) {
    load_wide_fences(p.scan.rt, threadIdx.x, blockDim.x);
    __syncthreads();  // the only workgroup barrier: the waves share nothing else
  }
  uint32_t n_ptr = 0, n_in = 0;

  const uint32_t wave = blockIdx.x * wpb + wv, n_waves = gridDim.x * wpb;
  const uint32_t n_items = RAGGED ? p.n_ragged : p.n_tiles;
  for (uint32_t it = wave; it < n_items; it += n_waves) {
    const uint32_t t = RAGGED ? p.ragged[it] - p.tile0 : it;
    const Tile tile = p.tiles[t];
    if (!RAGGED && tile.last_len != unit) continue;  // left to the ragged launch
    const uint32_t np = tile.npages;
    const uint64_t va = tile.va;
    const uint32_t last_pg = np - 1u, last_len = RAGGED ? (uint32_t)tile.last_len : unit;  // only the last unit can be partial
    uint32_t keep = (1u << np) - 1u;
    uint64_t slot_j[8];
    if (GATHER) {
      uint64_t slot = 0;
      bool kept = false;
      if (lane < np) {
        const uint64_t g = (uint64_t)tile.g + lane;
        const uint64_t zw = p.zero_bm[g >> 6];
        kept = ((zw >> (g & 63u)) & 1ull) == 0ull;
        slot = p.word_prefix[g >> 6] + (uint64_t)__popcll(~zw & ((1ull << (g & 63u)) - 1ull));
      }
      keep = (uint32_t)__ballot(kept);
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) slot_j[j] = __shfl(slot, 2 * j + half, 64);
      if (kept && slot < p.cap_pages) p.page_va[slot] = va + ((uint64_t)lane << ushift);
    }
    uint32_t nonzero = 0, oob = 0;
    uint64_t acc = acc_init(p.seed, k);

    uint4 cur[8];
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) {
      const uint32_t pg = 2 * j + half;
      if (RAGGED) {
        const uint32_t len = pg == last_pg ? last_len : unit;
        cur[j] = ((keep >> pg) & 1u) && off16 < len
                     ? clip16(ld16nt(va + ((uint64_t)pg << ushift) + off16), off16, len)
                     : make_uint4(0, 0, 0, 0);
      } else {
        cur[j] = ((keep >> pg) & 1u) ? ld16nt(va + ((uint64_t)pg << ushift) + off16) : make_uint4(0, 0, 0, 0);
      }
    }
    // this lane's quad: stripes of its unit, and the bytes past the last stripe
    const uint32_t qlen = RAGGED && q == last_pg ? last_len : unit;
    const uint32_t lim = qlen / 32u, rem = qlen & 31u;
#pragma unroll 1
    for (uint32_t c = 0; c < n_chunks; ++c) {
      uint32_t ptr_mask = 0;  // bit 2j+h: word h of this lane's 16 bytes of load j is pointer-like
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        const uint32_t pg = 2 * j + half;
        const uint4 v = cur[j];
        if (!GATHER) {
          const uint64_t b = __ballot(nz16(v));
          nonzero |= ((uint32_t)((uint32_t)b != 0u) << (2 * j)) | ((uint32_t)((b >> 32) != 0ull) << (2 * j + 1));
        }
        if (SCAN) {  // pointer-like words are only marked here; the range search runs once per chunk
          const uint64_t w0 = ((uint64_t)v.y << 32) | v.x;
          const uint64_t w1 = ((uint64_t)v.w << 32) | v.z;
          uint32_t p0 = (w0 - scan_lo) < scan_span ? 1u : 0u;
          uint32_t p1 = (w1 - scan_lo) < scan_span ? 1u : 0u;
          if (RAGGED) {  // words wholly inside the range only
            const uint32_t o = c * kChunk + off16, len = pg == last_pg ? last_len : unit;
            p0 = o + 8u <= len ? p0 : 0u;
            p1 = o + 16u <= len ? p1 : 0u;
          }
          ptr_mask |= (p0 << (2 * j)) | (p1 << (2 * j + 1));
        }
        if (GATHER) {
          if (((keep >> pg) & 1u) && slot_j[j] < p.cap_pages)
            st16nt((uint64_t)p.packed + (slot_j[j] << ushift) + c * kChunk + off16, v);
        }
        *reinterpret_cast<uint4*>(stage + pg * kStageStride + off16) = v;
      }
      wave_lds_order();
      // loads of the next chunk overlap the hashing of this one
      const uint32_t cn = c + 1 < n_chunks ? c + 1 : c;
      const uint32_t more = c + 1 < n_chunks ? keep : 0u;
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        const uint32_t pg = 2 * j + half, o = cn * kChunk + off16;
        if (RAGGED) {
          const uint32_t len = pg == last_pg ? last_len : unit;
          cur[j] = ((more >> pg) & 1u) && o < len ? clip16(ld16nt(va + ((uint64_t)pg << ushift) + o), o, len)
                                                  : make_uint4(0, 0, 0, 0);
        } else {
          cur[j] = ((more >> pg) & 1u) ? ld16nt(va + ((uint64_t)pg << ushift) + o) : make_uint4(0, 0, 0, 0);
        }
      }
      if (SCAN && __ballot(ptr_mask != 0u)) {
        // the marked words, read back from the stage: one search chain per lane per chunk
        n_ptr += (uint32_t)__popc(ptr_mask);
        for (uint32_t m = ptr_mask; m != 0u; m &= m - 1u) {
          const uint32_t bit = (uint32_t)__builtin_ctz(m);
          const uint64_t w = *reinterpret_cast<const uint64_t*>(stage + (2u * (bit >> 1) + half) * kStageStride +
                                                                 off16 + (bit & 1u) * 8u);
          if (wide_range_index(w, p.scan.rt) >= 0) ++n_in; else ++oob;
        }
      }
      const uint8_t* row = stage + q * kStageStride + k * 8u;
#pragma unroll
      for (uint32_t s = 0; s < kChunk / 32; ++s)
        if (!RAGGED || c * (kChunk / 32) + s < lim) acc = xround(acc, *reinterpret_cast<const uint64_t*>(row + s * 32u));
      if (RAGGED && rem != 0u && c == lim / (kChunk / 32))  // the partial page's last bytes are in this chunk
        tail_lds[q][k] = *reinterpret_cast<const uint64_t*>(stage + q * kStageStride + (lim * 32u - c * kChunk) + 8u * k);
      wave_lds_order();
    }

    const uint64_t merged = xxh64_merge4(acc, k);  // every lane of the quad takes part
    uint64_t h = (lim > 0u ? merged : p.seed + kP5) + qlen;
    if (RAGGED && rem != 0u) {
      const uint64_t tail[4] = {tail_lds[q][0], tail_lds[q][1], tail_lds[q][2], tail_lds[q][3]};
      h = xxh64_tail(h, tail, rem);
    }
    h = xxh64_avalanche(h);
    const bool mine = (k == 0u) && (q < np);
    if (mine) p.hash[tile.g + q] = h;
    const uint32_t valid = (1u << np) - 1u;
    if (!GATHER) {
      const uint32_t zero = ~nonzero & valid;
      if (lane == 0) or_page_bits(p.zero_bm, tile.g, np, zero);
    }
    if (PRIOR) {
      const bool ch = mine && (h != p.prior[tile.g + q]);
      const uint32_t cb = quad_bits(__ballot(ch));
      if (lane == 0) or_page_bits(p.changed_bm, tile.g, np, cb);
    }
    if (SCAN) {
      const uint32_t o = wave_sum_u32(oob);
      if (lane == 0) p.scan.tile_oob[p.tile0 + t] = o;
    }
  }
  if (SCAN) {
    const uint32_t a = wave_sum_u32(n_ptr), b = wave_sum_u32(n_in);
    if (lane == 0) {
      add_scan_counts(p.scan.counts, wave, a, b);
    }
  }
}

// ------------------------------------------------------------ zero probe --
// Exact zero bitmap.  A wave takes four tiles at a time, one lane per unit:
// each lane reads the first 16 bytes of its unit; a unit whose first 16 bytes
// are zero is then read by the whole wave (four such units at a time, 4 KiB of
// each per round) until a non-zero byte shows or the unit ends.
__global__ __launch_bounds__(64) void k_probe_zero(const Tile* tiles, uint32_t n_tiles,
                                                   uint64_t* zero_bm, uint32_t ushift) {
  const uint32_t lane = threadIdx.x, sub = lane >> 4, pl = lane & 15u;
  const uint32_t unit = 1u << ushift, nsub = unit / kPage;
  for (uint32_t t0 = blockIdx.x * 4u; t0 < n_tiles; t0 += gridDim.x * 4u) {
    const uint32_t t = t0 + sub;
    Tile tile{0, 0, 0};
    if (t < n_tiles) tile = tiles[t];
    const bool valid = pl < tile.npages;
    const uint32_t len = valid ? unit_bytes(tile, pl, unit) : 0u;  // a partial unit is tested over its bytes only
    const uint64_t unit_va = tile.va + ((uint64_t)pl << ushift);
    const uint4 v = valid ? clip16(ld16(unit_va), 0u, len) : make_uint4(0, 0, 0, 0);
    const bool cand = valid && !nz16(v);
    uint64_t maybe = __ballot(cand && len == unit);
    uint64_t maybe_part = __ballot(cand && len != unit);
    uint64_t zero = 0;
    while (maybe) {  // whole units, four at a time
      uint32_t ln[4];
      uint64_t pva[4];
      uint32_t cnt = 0;
#pragma unroll
      for (uint32_t i = 0; i < 4; ++i) {
        ln[i] = maybe ? (uint32_t)__builtin_ctzll(maybe) : 0u;
        pva[i] = __shfl(unit_va, ln[i], 64);
        if (maybe) {
          maybe &= maybe - 1ull;
          ++cnt;
        }
      }
      uint32_t alive = (1u << cnt) - 1u;  // units with no non-zero byte seen yet
      for (uint32_t b = 0; b < nsub && alive != 0u; ++b) {
        uint4 x[16];
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i)
#pragma unroll
          for (uint32_t j = 0; j < 4; ++j)
            x[i * 4 + j] = ((alive >> i) & 1u) ? ld16nt(pva[i] + (uint64_t)b * kPage + j * 1024u + lane * 16u)
                                               : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
          const bool nzl = nz16(x[i * 4]) || nz16(x[i * 4 + 1]) || nz16(x[i * 4 + 2]) || nz16(x[i * 4 + 3]);
          if (__ballot(nzl) != 0ull) alive &= ~(1u << i);
        }
      }
#pragma unroll
      for (uint32_t i = 0; i < 4; ++i)
        if ((alive >> i) & 1u) zero |= 1ull << ln[i];
    }
    while (maybe_part) {  // partial last units (one per range at most), one at a time over their bytes
      const uint32_t L = (uint32_t)__builtin_ctzll(maybe_part);
      maybe_part &= maybe_part - 1ull;
      const uint64_t pva = __shfl(unit_va, L, 64);
      const uint32_t plen = __shfl(len, L, 64);
      bool nzw = false;
      for (uint32_t o0 = 0; o0 < plen && !nzw; o0 += kPage) {
        bool nzl = false;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
          const uint32_t o = o0 + j * 1024u + lane * 16u;
          if (o < plen) nzl = nzl || nz16(clip16(ld16nt(pva + o), o, plen));
        }
        nzw = __ballot(nzl) != 0ull;
      }
      if (!nzw) zero |= 1ull << L;
    }
    if (pl == 0 && t < n_tiles) or_page_bits(zero_bm, tile.g, tile.npages, (uint32_t)((zero >> (16u * sub)) & 0xFFFFull));
  }
}

// ------------------------------------------------ reduce-then-scan (u64) --
constexpr uint32_t kScanThreads = 256, kScanPerThread = 8;
constexpr uint32_t kScanBlock = kScanThreads * kScanPerThread;

__device__ __forceinline__ uint32_t scan_item(const ScanSrc& s, uint64_t i) {
  if (i >= s.n_items) return 0u;
  if (s.kind == kSrcCounts) return s.counts[i];
  uint64_t keep = ~s.zero_bm[i];
  if (s.changed_bm) keep &= s.changed_bm[i];
  if (i == s.n_items - 1 && (s.n_pages & 63u)) keep &= (1ull << (s.n_pages & 63u)) - 1ull;
  return (uint32_t)__popcll(keep);
}

// Exclusive scan of one value per thread across a 256-thread block.
__device__ __forceinline__ uint64_t block_exclusive(uint64_t x, uint64_t* lds4, uint64_t* total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint64_t inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(inc, d, 64);
    if (lane >= (uint32_t)d) inc += y;
  }
  if (lane == 63) lds4[wave] = inc;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
#pragma unroll
  for (uint32_t w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) pre += lds4[w];
    tot += lds4[w];
  }
  __syncthreads();
  if (total) *total = tot;
  return pre + inc - x;
}

__global__ __launch_bounds__(256) void k_scan_reduce(ScanSrc src, uint64_t* block_sums) {
  __shared__ uint64_t lds4[4];
  const uint64_t i0 = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPerThread;
  uint64_t s = 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanPerThread; ++i) s += scan_item(src, i0 + i);
  uint64_t tot = 0;
  block_exclusive(s, lds4, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_top(uint64_t* block_sums, uint32_t nb, uint64_t* total_out) {
  __shared__ uint64_t lds[16];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  uint64_t carry = 0;
  for (uint32_t base = 0; base < nb; base += 1024) {
    const uint32_t i = base + tid;
    const uint64_t x = i < nb ? block_sums[i] : 0ull;
    uint64_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(inc, d, 64);
      if (lane >= (uint32_t)d) inc += y;
    }
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
    for (uint32_t w = 0; w < 16; ++w) {
      if (w < wave) pre += lds[w];
      tot += lds[w];
    }
    if (i < nb) block_sums[i] = carry + pre + inc - x;
    carry += tot;
    __syncthreads();
  }
  if (tid == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(256) void k_scan_down(ScanSrc src, const uint64_t* block_sums, uint64_t* out) {
  __shared__ uint64_t lds4[4];
  const uint64_t i0 = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPerThread;
  uint32_t v[kScanPerThread];
  uint64_t s = 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanPerThread; ++i) {
    v[i] = scan_item(src, i0 + i);
    s += v[i];
  }
  uint64_t run = block_exclusive(s, lds4, nullptr) + block_sums[blockIdx.x];
#pragma unroll
  for (uint32_t i = 0; i < kScanPerThread; ++i) {
    if (i0 + i < src.n_items) out[i0 + i] = run;
    run += v[i];
  }
}

// Whole scan in one block when the items fit in it (small inputs: one launch
// instead of three).
__global__ __launch_bounds__(256) void k_scan_small(ScanSrc src, uint64_t* out, uint64_t* total_out) {
  __shared__ uint64_t lds4[4];
  const uint64_t i0 = (uint64_t)threadIdx.x * kScanPerThread;
  uint32_t v[kScanPerThread];
  uint64_t s = 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanPerThread; ++i) {
    v[i] = scan_item(src, i0 + i);
    s += v[i];
  }
  uint64_t tot = 0;
  uint64_t run = block_exclusive(s, lds4, &tot);
#pragma unroll
  for (uint32_t i = 0; i < kScanPerThread; ++i) {
    if (i0 + i < src.n_items) out[i0 + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0 && total_out) *total_out = tot;
}

// ------------------------------------------------------ slots of a tile ---
// Lane i < np: keep bit and packed slot of page i of the tile.
__device__ __forceinline__ void tile_slots(const Tile& tile, const uint64_t* zero_bm,
                                           const uint64_t* changed_bm, const uint64_t* word_prefix,
                                           uint32_t lane, bool& kept, uint64_t& slot) {
  kept = false;
  slot = 0;
  if (lane < tile.npages) {
    const uint64_t g = (uint64_t)tile.g + lane;
    uint64_t kw = ~zero_bm[g >> 6];
    if (changed_bm) kw &= changed_bm[g >> 6];
    kept = ((kw >> (g & 63u)) & 1ull) != 0ull;
    slot = word_prefix[g >> 6] + (uint64_t)__popcll(kw & ((1ull << (g & 63u)) - 1ull));
  }
}

// --------------------------------------------------------------- gather ---
// Kept units of a tile, four at a time, copied to their packed slots 4 KiB of
// each per round; a partial unit's slot is filled up with zeros.
__global__ __launch_bounds__(64) void k_gather(const Tile* tiles, uint32_t n_tiles, const uint64_t* zero_bm,
                                               const uint64_t* changed_bm, const uint64_t* word_prefix,
                                               uint8_t* packed, uint64_t* page_va, uint64_t cap, uint32_t ushift) {
  const uint32_t lane = threadIdx.x;
  const uint32_t unit = 1u << ushift, nsub = unit / kPage;
  for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const Tile tile = tiles[t];
    bool kept;
    uint64_t slot;
    tile_slots(tile, zero_bm, changed_bm, word_prefix, lane, kept, slot);
    const bool go = kept && slot < cap;
    if (go) page_va[slot] = tile.va + ((uint64_t)lane << ushift);
    uint32_t mask = (uint32_t)__ballot(go);
    while (mask) {
      uint32_t pg[4];
      uint64_t dst[4];
      uint32_t cnt = 0;
#pragma unroll
      for (uint32_t i = 0; i < 4; ++i) {
        pg[i] = mask ? (uint32_t)__builtin_ctz(mask) : 0u;
        dst[i] = __shfl(slot, pg[i], 64);
        if (mask) {
          mask &= mask - 1u;
          ++cnt;
        }
      }
      for (uint32_t b = 0; b < nsub; ++b) {
        uint4 x[16];
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i)
#pragma unroll
          for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t o = b * kPage + j * 1024u + lane * 16u, len = unit_bytes(tile, pg[i], unit);
            if (i < cnt)
              x[i * 4 + j] = o < len ? clip16(ld16nt(tile.va + ((uint64_t)pg[i] << ushift) + o), o, len)
                                     : make_uint4(0, 0, 0, 0);  // a partial unit: zeros after its bytes
          }
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i)
#pragma unroll
          for (uint32_t j = 0; j < 4; ++j)
            if (i < cnt)
              st16nt((uint64_t)packed + (dst[i] << ushift) + b * kPage + j * 1024u + lane * 16u, x[i * 4 + j]);
      }
    }
  }
}

// -------------------------------------------------------------- restore ---
__global__ __launch_bounds__(64) void k_restore_zero(const Tile* tiles, uint32_t n_tiles,
                                                     const uint64_t* zero_bm, const uint64_t* changed_bm,
                                                     unsigned long long* n_bad, uint32_t ushift) {
  const uint32_t lane = threadIdx.x, unit = 1u << ushift;
  if (blockIdx.x == 0 && lane == 0) *n_bad = 0ull;  // the scatter that follows counts into it
  for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const Tile tile = tiles[t];
    bool sel = false;
    if (lane < tile.npages) {
      const uint64_t g = (uint64_t)tile.g + lane;
      uint64_t w = zero_bm[g >> 6];
      if (changed_bm) w &= changed_bm[g >> 6];
      sel = ((w >> (g & 63u)) & 1ull) != 0ull;
    }
    uint32_t mask = (uint32_t)__ballot(sel);
    const uint4 z = make_uint4(0, 0, 0, 0);
    while (mask) {
      const uint32_t pg = (uint32_t)__builtin_ctz(mask);
      mask &= mask - 1u;
      const uint32_t len = unit_bytes(tile, pg, unit);  // never past the range's end
      const uint64_t uva = tile.va + ((uint64_t)pg << ushift);
      for (uint32_t o0 = 0; o0 < len; o0 += kPage) {
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
          const uint32_t o = o0 + j * 1024u + lane * 16u;
          if (o + 16u <= len) st16nt(uva + o, z);
          else if (o < len) st_bytes(uva + o, z, len - o);
        }
      }
    }
  }
}

// Packed units back to their VAs, one 4 KiB block per wave and WAVES waves
// (that many consecutive blocks) per workgroup, the grid covering every block
// of the capacity (no persistent stride).  Block b of the packed snapshot
// belongs to slot b >> (ushift - 12); the wave reads that slot's page-VA entry
// (one scalar load for the whole wave), validates it (4 KiB aligned, inside a
// range, the start of a unit of that range) with a scalar search of the range
// set's arrays, and copies the block, if it lies wholly inside the range, with
// four 16-byte loads and stores per lane.  Workgroups are dispatched in block order, so the waves in flight cover
// one compact, advancing window of both buffers: against a persistent grid
// striding four-block groups over the snapshot (with a range table loaded into
// LDS per workgroup) the one-wave form runs at the speed of a plain copy
// kernel between the same buffers.  Four-wave workgroups copy a full snapshot
// about 5 % slower (a workgroup's slot is freed only when its last wave ends)
// but dispatch a quarter of the workgroups, which is what a delta restore pays
// for when its kept count is far below the capacity the grid covers.
template <uint32_t WAVES>
__global__ __launch_bounds__(WAVES * kWave) void k_restore_scatter(RangeTable rt, const uint8_t* packed,
                                                                   const uint64_t* page_va, const uint64_t* n_kept,
                                                                   uint64_t cap, unsigned long long* n_bad,
                                                                   uint32_t ushift) {
  const uint32_t lane = threadIdx.x % kWave;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // so the block index is scalar
  const uint32_t bshift = ushift - 12u;  // 4 KiB blocks per unit: 1 << bshift
  const uint64_t unit = 1ull << ushift;
  const uint64_t nblk = min(*n_kept, cap) << bshift;
  for (uint64_t blk = (uint64_t)blockIdx.x * WAVES + wave; blk < nblk; blk += (uint64_t)gridDim.x * WAVES) {
    const uint64_t sub = blk & ((1ull << bshift) - 1ull);
    const uint64_t va = ((const KC_CONST uint64_t*)page_va)[blk >> bshift];  // one scalar load for the wave
    bool good = false, ok = false;
    if ((va & (kPage - 1)) == 0) {
      const RangeHit r = range_find_uniform(va, rt);
      if (r.a >= 0) {  // of a range's partial last unit, the bytes past its last whole block go to k_restore_tail
        good = ((va - r.base) & (unit - 1ull)) == 0ull;
        ok = good && va + (sub << 12) + kPage <= r.end;
      }
    }
    if (!good && sub == 0 && lane == 0) atomicAdd(n_bad, 1ull);  // counted once per slot
    if (!ok) continue;
    const uint64_t src = (uint64_t)packed + blk * kPage + lane * 16u, dst = va + (sub << 12) + lane * 16u;
    uint4 x[4];
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) x[j] = ld16nt(src + j * 1024u);
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) st16nt(dst + j * 1024u, x[j]);
  }
}

// Packed units bound for a range's partial last unit: the restore scatter
// copies its whole 4 KiB blocks; here only its last bytes past them are
// written, never past the range's end.  One lane per slot finds such units;
// the wave copies each one's remainder (under 4 KiB).
__global__ __launch_bounds__(64) void k_restore_tail(RangeTable rt, const uint8_t* packed, const uint64_t* page_va,
                                                     const uint64_t* n_kept, uint64_t cap, uint32_t ushift) {
  __shared__ FenceLds fences;
  const uint32_t lane = threadIdx.x;
  const uint64_t unit = 1ull << ushift;
  load_fences(fences, rt, lane, kWave);
  __syncthreads();
  const uint64_t n = min(*n_kept, cap);
  for (uint64_t s0 = (uint64_t)blockIdx.x * 64u; s0 < n; s0 += (uint64_t)gridDim.x * 64u) {
    uint64_t va = 0;
    uint32_t len = 0;
    if (s0 + lane < n) {
      va = page_va[s0 + lane];
      const int32_t a = (va & (kPage - 1)) == 0 ? range_index(va, fences, rt) : -1;
      if (a >= 0) {
        const uint64_t base = rt.stride == 1u ? fences.base[a] : ld8g(rt.base + a);
        const uint64_t end = rt.stride == 1u ? fences.end[a] : ld8g(rt.end + a);
        if (((va - base) & (unit - 1ull)) == 0ull && va + unit > end && ((end - va) & (kPage - 1)) != 0ull)
          len = (uint32_t)(end - va);
      }
    }
    for (uint64_t m = __ballot(len != 0u); m != 0ull; m &= m - 1ull) {
      const int32_t L = __ffsll((long long)m) - 1;
      const uint64_t dva = __shfl((unsigned long long)va, L, 64);
      const uint32_t dlen = __shfl(len, L, 64);
      const uint64_t src = (uint64_t)packed + ((s0 + (uint64_t)L) << ushift);
      const uint32_t o0 = dlen & ~(kPage - 1u);  // the bytes before it went with the scatter's whole blocks
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t o = o0 + j * 1024u + lane * 16u;
        if (o < dlen) st_bytes(dva + o, ld16nt(src + o), dlen - o);  // never past the range's end
      }
    }
  }
}

// --------------------------------------------------------- closure scan ---
__device__ __forceinline__ void closure_words(uint4 v, uint64_t lo, uint64_t span, const RangeTable& rt,
                                              uint32_t& n_ptr, uint32_t& n_in, uint32_t& oob) {
  const uint64_t w0 = ((uint64_t)v.y << 32) | v.x;
  const uint64_t w1 = ((uint64_t)v.w << 32) | v.z;
  const bool p0 = (w0 - lo) < span, p1 = (w1 - lo) < span;
  if (__ballot(p0 || p1)) {
    if (p0) {
      ++n_ptr;
      if (wide_range_index(w0, rt) >= 0) ++n_in; else ++oob;
    }
    if (p1) {
      ++n_ptr;
      if (wide_range_index(w1, rt) >= 0) ++n_in; else ++oob;
    }
  }
}

// Standalone scan: a tile's 16 pages are read as 64 contiguous 1-KiB runs.
// Workgroups of kWideWaves independent waves share the wide range table.
__global__ __launch_bounds__(kWideWaves * kWave) __attribute__((amdgpu_waves_per_eu(4))) void k_closure(
    const Tile* tiles, uint32_t n_tiles, uint32_t tile0, ScanDev sd) {
  const uint32_t lane = threadIdx.x % kWave, wpb = blockDim.x / kWave;
  const uint32_t wave = blockIdx.x * wpb + threadIdx.x / kWave, n_waves = gridDim.x * wpb;
  load_wide_fences(sd.rt, threadIdx.x, blockDim.x);
  __syncthreads();
  uint32_t n_ptr = 0, n_in = 0;
  for (uint32_t t = wave; t < n_tiles; t += n_waves) {
    const Tile tile = tiles[t];
    const uint32_t nseg = tile.npages * 4u;
    uint32_t oob = 0;
    for (uint32_t s0 = 0; s0 < nseg; s0 += 8) {
      uint4 x[8];
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i)
        x[i] = (s0 + i < nseg) ? ld16nt(tile.va + (uint64_t)(s0 + i) * 1024u + lane * 16u) : make_uint4(0, 0, 0, 0);
#pragma unroll
      for (uint32_t i = 0; i < 8; ++i)
        closure_words(seg_words(tile, s0 + i, lane, x[i]), sd.lo, sd.span, sd.rt, n_ptr, n_in, oob);
    }
    const uint32_t o = wave_sum_u32(oob);
    if (lane == 0) sd.tile_oob[tile0 + t] = o;
  }
  const uint32_t a = wave_sum_u32(n_ptr), b = wave_sum_u32(n_in);
  if (lane == 0) {
    add_scan_counts(sd.counts, wave, a, b);
  }
}

// Writes the out-of-range words of each tile at its prefix position, in
// ascending address order, up to the list capacity.  A block owns a slice of
// consecutive tiles: one parallel read of their counts lists the tiles with
// entries below the capacity, then each listed tile is read again with one
// wave per page (its four 1-KiB segments in one round trip), the waves'
// entries placed by a prefix over their counts.
constexpr uint32_t kEmitThreads = kTilePages * kWave;  // one wave per page of a tile
constexpr uint32_t kEmitMaxSlice = kEmitThreads;       // tiles a block lists at once
constexpr uint32_t kEmitMaxBlocks = 128;

__global__ __launch_bounds__(kEmitThreads) void k_oob_emit(const Tile* tiles, uint32_t n_tiles, uint32_t slice,
                                                           ScanDev sd, const uint64_t* tile_prefix,
                                                           const uint64_t* n_oob, kc_oob* oob, uint64_t cap,
                                                           kc_scan_result* res, uint64_t n_words) {
  __shared__ FenceLds fences;
  __shared__ uint32_t listed[kEmitMaxSlice];
  __shared__ uint32_t n_listed;
  __shared__ uint32_t wave_cnt[kTilePages];
  const uint32_t tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
  const uint64_t total = *n_oob;
  if (blockIdx.x == 0 && wv == 0) {  // the result struct, from the slot totals
    static_assert(kScanSlots == kWave, "one slot per lane");
    const unsigned long long* c = sd.counts + (size_t)lane * kScanSlotStride;
    const unsigned long long a = wave_sum_u64(c[0]), b = wave_sum_u64(c[1]);
    if (lane == 0) {
      res->n_words = n_words;
      res->n_ptr_like = a;
      res->n_in_range = b;
      res->n_oob = total;
      res->n_written = (uint32_t)(total < cap ? total : cap);
      res->truncated = total > cap ? 1u : 0u;
    }
  }
  if (total == 0 || cap == 0) return;  // nothing to list: no tile to revisit
  const uint64_t below = (1ull << lane) - 1ull;
  bool fenced = false;
  for (uint64_t t0 = (uint64_t)blockIdx.x * slice; t0 < n_tiles; t0 += (uint64_t)gridDim.x * slice) {
    if (tid == 0) n_listed = 0u;
    __syncthreads();
    const uint64_t t = t0 + tid;
    if (tid < slice && t < n_tiles && sd.tile_oob[t] != 0u && tile_prefix[t] < cap)
      listed[atomicAdd(&n_listed, 1u)] = (uint32_t)t;
    __syncthreads();
    const uint32_t n = n_listed;  // the same in every thread
    if (n != 0u && !fenced) {     // the range table, only for blocks with a tile to revisit
      load_fences(fences, sd.rt, tid, kEmitThreads);
      __syncthreads();
      fenced = true;
    }
    for (uint32_t i = 0; i < n; ++i) {
      const uint32_t tt = listed[i];
      const Tile tile = tiles[tt];
      const bool mine = wv < tile.npages;
      uint4 x[4];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j)
        x[j] = mine ? ld16(tile.va + (uint64_t)(wv * 4u + j) * 1024u + lane * 16u) : make_uint4(0, 0, 0, 0);
      uint64_t b0[4], b1[4];
      uint32_t cnt = 0;
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {  // zero words (and pages past the tile) are never pointer-like
        const uint4 v = seg_words(tile, wv * 4u + j, lane, x[j]);  // same words as the counting pass
        const uint64_t w0 = ((uint64_t)v.y << 32) | v.x;
        const uint64_t w1 = ((uint64_t)v.w << 32) | v.z;
        b0[j] = __ballot((w0 - sd.lo) < sd.span && !in_ranges(w0, fences, sd.rt));
        b1[j] = __ballot((w1 - sd.lo) < sd.span && !in_ranges(w1, fences, sd.rt));
        cnt += (uint32_t)(__popcll(b0[j]) + __popcll(b1[j]));
        x[j] = v;
      }
      if (lane == 0) wave_cnt[wv] = cnt;
      __syncthreads();
      uint64_t done = tile_prefix[tt];
      for (uint32_t w = 0; w < wv; ++w) done += wave_cnt[w];
#pragma unroll
      for (uint32_t j = 0; j < 4; ++j) {  // segments in order, lanes in order, word 0 before word 1
        const uint64_t a = tile.va + (uint64_t)(wv * 4u + j) * 1024u + lane * 16u;
        const bool o0 = ((b0[j] >> lane) & 1ull) != 0ull, o1 = ((b1[j] >> lane) & 1ull) != 0ull;
        const uint64_t r0 = done + (uint64_t)__popcll(b0[j] & below) + (uint64_t)__popcll(b1[j] & below);
        const uint64_t r1 = r0 + (o0 ? 1u : 0u);
        if (o0 && r0 < cap) {
          oob[r0].word_va = a;
          oob[r0].value = ((uint64_t)x[j].y << 32) | x[j].x;
        }
        if (o1 && r1 < cap) {
          oob[r1].word_va = a + 8u;
          oob[r1].value = ((uint64_t)x[j].w << 32) | x[j].z;
        }
        done += (uint64_t)__popcll(b0[j]) + (uint64_t)__popcll(b1[j]);
      }
      __syncthreads();  // wave_cnt is reused by the next listed tile
    }
    __syncthreads();  // every thread has read n_listed before it is cleared again
  }
}

inline uint32_t blocks_for(uint64_t n, uint32_t per) { return (uint32_t)((n + per - 1) / per); }

}  // namespace

// ------------------------------------------------------------- launchers --
hipError_t launch_zero3(uint64_t* a, uint64_t na, uint64_t* b, uint64_t nb, uint64_t* c, uint64_t nc,
                        hipStream_t s) {
  const uint64_t n = na + nb + nc;
  if (n == 0) return hipSuccess;
  const uint64_t nbk = blocks_for(n, 256);
  hipLaunchKernelGGL(k_zero3, dim3((uint32_t)(nbk < 4096 ? nbk : 4096)), dim3(256), 0, s, a, na, b, nb, c, nc);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t nb = blocks_for(n, 256);
  const uint32_t grid = (uint32_t)(nb < 4096 ? nb : 4096);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_page_hash(const HashParams& p, bool gather, bool prior, bool scan, uint32_t depth, uint32_t grid,
                            uint32_t n_cu, hipStream_t s) {
  if (p.n_tiles == 0) return hipSuccess;
  uint32_t blocks = 1, wpb = 1, blocks_r = 1, wpb_r = 1;  // grid counts waves
  wide_shape(std::min(grid, p.n_tiles), n_cu, &blocks, &wpb, kHashWaves);
  wide_shape(std::min(grid, std::max(1u, p.n_ragged)), n_cu, &blocks_r, &wpb_r, kHashWaves);
  const size_t lds = scan ? wide_lds_bytes(p.scan.rt) : 0;
  if (depth > 1u && !scan)  // every tile, partial last units included, through the pipelined pass
    return launch_page_hash_deep(p, gather, prior, depth, blocks, wpb, s);
#define KC_HASH_CASE(G, P, S)                                                                              \
  if (gather == G && prior == P && scan == S) {                                                           \
    hipLaunchKernelGGL((k_page_hash<G, P, S, false>), dim3(blocks), dim3(wpb * kWave), lds, s, p);        \
    hipError_t e = hipGetLastError();                                                                     \
    if (e != hipSuccess || p.n_ragged == 0) return e;                                                     \
    hipLaunchKernelGGL((k_page_hash<G, P, S, true>), dim3(blocks_r), dim3(wpb_r * kWave), lds, s, p);     \
    return hipGetLastError();                                                                             \
  }
  KC_HASH_CASE(false, false, false)
  KC_HASH_CASE(false, false, true)
  KC_HASH_CASE(false, true, false)
  KC_HASH_CASE(false, true, true)
  KC_HASH_CASE(true, false, false)
  KC_HASH_CASE(true, false, true)
#undef KC_HASH_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_probe_zero(const Tile* tiles, uint32_t n_tiles, uint64_t* zero_bm, uint32_t ushift, uint32_t grid,
                             hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  grid = std::max(1u, std::min(grid, n_tiles));
  hipLaunchKernelGGL(k_probe_zero, dim3(grid), dim3(64), 0, s, tiles, n_tiles, zero_bm, ushift);
  return hipGetLastError();
}

hipError_t launch_scan(const ScanSrc& src, uint64_t* out, uint64_t* block_sums, uint64_t* total_out,
                       hipStream_t s) {
  const uint32_t nb = blocks_for(src.n_items, kScanBlock);
  if (nb <= 1) {
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kScanThreads), 0, s, src, out, total_out);
    return hipGetLastError();
  }
  if (nb > 0) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, src, block_sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, block_sums, nb, total_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nb == 0) return e;
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanThreads), 0, s, src, (const uint64_t*)block_sums, out);
  return hipGetLastError();
}

hipError_t launch_gather(const Tile* tiles, uint32_t n_tiles, const uint64_t* zero_bm,
                         const uint64_t* changed_bm, const uint64_t* word_prefix, uint8_t* packed,
                         uint64_t* page_va, uint64_t cap_pages, uint32_t ushift, uint32_t grid, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  grid = std::max(1u, std::min(grid, n_tiles));
  hipLaunchKernelGGL(k_gather, dim3(grid), dim3(64), 0, s, tiles, n_tiles, zero_bm, changed_bm, word_prefix,
                     packed, page_va, cap_pages, ushift);
  return hipGetLastError();
}

hipError_t launch_restore_zero(const Tile* tiles, uint32_t n_tiles, const uint64_t* zero_bm,
                               const uint64_t* changed_bm, unsigned long long* n_bad, uint32_t ushift, uint32_t grid,
                               hipStream_t s) {
  grid = std::max(1u, std::min(grid, std::max(1u, n_tiles)));
  hipLaunchKernelGGL(k_restore_zero, dim3(grid), dim3(64), 0, s, tiles, n_tiles, zero_bm, changed_bm, n_bad,
                     ushift);
  return hipGetLastError();
}

template <uint32_t WAVES>
void launch_scatter_waves(const RangeTable& rt, const uint8_t* packed, const uint64_t* page_va,
                          const uint64_t* n_kept, uint64_t cap_pages, unsigned long long* n_bad, uint32_t ushift,
                          hipStream_t s) {
  // WAVES blocks per workgroup over every 4 KiB block of the capacity (blocks past the kept count exit at once);
  // the kernel strides only if a capacity ever exceeded the grid limit
  const uint32_t bshift = ushift - 12u;
  const uint64_t kMaxGrid = 0x7FFFFFFFull;
  const uint64_t wgs = cap_pages > ((kMaxGrid * WAVES) >> bshift) ? kMaxGrid
                                                                   : ((cap_pages << bshift) + WAVES - 1) / WAVES;
  hipLaunchKernelGGL(k_restore_scatter<WAVES>, dim3((uint32_t)wgs), dim3(WAVES * kWave), 0, s, rt, packed, page_va,
                     n_kept, cap_pages, n_bad, ushift);
}

hipError_t launch_restore_scatter(const RangeTable& rt, const uint8_t* packed, const uint64_t* page_va,
                                  const uint64_t* n_kept, uint64_t cap_pages, unsigned long long* n_bad,
                                  bool ragged, bool delta, uint32_t ushift, uint32_t grid, hipStream_t s) {
  if (cap_pages == 0) return hipSuccess;
  if (delta)
    launch_scatter_waves<4>(rt, packed, page_va, n_kept, cap_pages, n_bad, ushift, s);
  else
    launch_scatter_waves<1>(rt, packed, page_va, n_kept, cap_pages, n_bad, ushift, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !ragged) return e;
  const uint64_t groups64 = (cap_pages + 63) / 64;
  const uint32_t grid_t = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(groups64, 1024));
  hipLaunchKernelGGL(k_restore_tail, dim3(grid_t), dim3(64), 0, s, rt, packed, page_va, n_kept, cap_pages, ushift);
  return hipGetLastError();
}

hipError_t launch_closure(const Tile* tiles, uint32_t n_tiles, uint32_t tile0, const ScanDev& sd,
                          uint32_t grid, uint32_t n_cu, hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  uint32_t blocks = 1, wpb = 1;
  wide_shape(std::min(grid, n_tiles), n_cu, &blocks, &wpb);  // grid counts waves
  hipLaunchKernelGGL(k_closure, dim3(blocks), dim3(wpb * kWave), wide_lds_bytes(sd.rt), s, tiles, n_tiles, tile0,
                     sd);
  return hipGetLastError();
}

hipError_t launch_oob_emit(const Tile* tiles, uint32_t n_tiles, const ScanDev& sd, const uint64_t* tile_prefix,
                           const uint64_t* n_oob, kc_oob* oob, uint64_t cap, kc_scan_result* res, uint64_t n_words,
                           hipStream_t s) {
  // slices of up to 1024 tiles, at most 128 blocks unless the slices are full: few tiles per block on small sets,
  // so that listed tiles are revisited in parallel
  const uint32_t slice = std::max(1u, std::min(kEmitMaxSlice, blocks_for(n_tiles, kEmitMaxBlocks)));
  const uint32_t blocks = std::max(1u, blocks_for(n_tiles, slice));
  hipLaunchKernelGGL(k_oob_emit, dim3(blocks), dim3(kEmitThreads), 0, s, tiles, n_tiles, slice, sd, tile_prefix,
                     n_oob, oob, cap, res, n_words);
  return hipGetLastError();
}


}  // namespace kc

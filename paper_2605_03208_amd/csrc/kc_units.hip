// kc_units.hip -- the hashing pass of hash units above 4 KiB (8 KiB to 2 MiB):
// a lane quad per unit as in the 4 KiB pass, with several chunks in flight per
// wave and the quads skewed over the unit's chunks.
#include <algorithm>

#include "kc_device.h"
#include "kc_internal.h"
#include "kc_xxh64.h"

namespace kc {
namespace {

// Buffer resource over [base, base + bytes) (gfx9 raw buffer, no stride):
// loads outside it return zeros and stores outside it are dropped.  base and
// bytes must be the same in every lane of the wave.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(uint64_t base, uint32_t bytes) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), (short)0,
                                           (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
constexpr uint32_t kOutside = 0x80000000u;  // an offset beyond any resource made here (tiles are below 64 MiB)
constexpr int kNt = 2;                      // cache policy: non-temporal

// The hashing pass with DEPTH (2 to 4) chunks in flight per wave, for units
// above 4 KiB.  Large units give few tiles, about one wave per SIMD for 2 MiB
// units: with no other wave to switch to, a wave must cover the memory latency
// itself.  DEPTH register sets take turns: while round c is staged, stored and
// hashed, rounds c+1 .. c+DEPTH-1 are already loading, and the loads of round
// c+DEPTH are issued after round c's stores, so waiting for round c+1 never
// waits for those stores.
//
// The quads run skewed: in round c, quad q works on chunk c - q*skew of its
// unit, skew = n_chunks / 32 clamped to 1..8.  The units of a tile start
// 2^ushift bytes apart, so without the skew one load instruction's pieces
// (equal offsets in up to 16 units) would all sit at addresses congruent
// modulo the unit size; with it they are skew*512 bytes apart in that
// congruence.  A tile of np units takes (np-1)*skew rounds more than it has
// chunks (a quad idles before its first and after its last chunk).  Measured
// on the 30 GiB pool: 64 KiB units fastest at skew 4, 2 MiB units at skew 8
// (15 % faster than skew 1, and than skew 16).  Tiles hold 16 units, or 8
// when 16 would leave fewer than two waves per SIMD (the range set decides).
//
// The loads and stores go through buffer resources bounded to the tile's
// bytes and to its kept units' packed slots, so no lane branches around a
// memory access (a branch that may skip one leaves the compiler unsure how
// many are in flight, and it then waits for all of them): skipped units (zero
// units of a full snapshot, lanes past the tile) and chunks outside a unit use
// an offset outside the resource.  Every tile goes through it, a tile's
// partial last unit included; no closure scan (it runs as its own pass at
// units above 4 KiB).
template <bool GATHER, bool PRIOR, uint32_t DEPTH>
__global__ __launch_bounds__(kHashWaves * kWave) __attribute__((amdgpu_waves_per_eu(2))) void k_page_hash_deep(
    HashParams p) {
  __shared__ __attribute__((aligned(16))) uint8_t stage_all[kHashWaves][kTilePages * kStageStride];
  __shared__ uint64_t tail_all[kHashWaves][kTilePages][4];  // a partial unit's bytes past its last whole stripe
  const uint32_t lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, wpb = blockDim.x / kWave;
  uint8_t* const stage = stage_all[wv];
  uint64_t(*const tail_lds)[4] = tail_all[wv];
  const uint32_t q = lane >> 2, k = lane & 3u;
  const uint32_t half = lane >> 5, off16 = (lane & 31u) * 16u;
  const uint32_t ushift = p.ushift, unit = 1u << ushift;
  const uint32_t n_chunks = unit / kChunk;
  // chunks each quad starts after the one before it: 2 KiB apart at 64 KiB units, 4 KiB from 128 KiB up
  const uint32_t skew = min(8u, max(1u, n_chunks / 32u));
  const uint32_t wave = blockIdx.x * wpb + wv, n_waves = gridDim.x * wpb;
  for (uint32_t t = wave; t < p.n_tiles; t += n_waves) {
    const Tile tile = p.tiles[t];
    const uint32_t np = tile.npages;
    const uint64_t va = tile.va;
    const uint32_t last_pg = np - 1u, last_len = tile.last_len;  // only the last unit can be partial
    const uint32_t n_rounds = (n_chunks + last_pg * skew + DEPTH - 1u) / DEPTH * DEPTH;  // the last quad ends last
    uint32_t keep = (1u << np) - 1u;
    uint32_t st_base[8];  // each load's unit in the packed slots resource
    __amdgpu_buffer_rsrc_t dst = raw_rsrc((uint64_t)p.packed, 0u);  // no slots: every store dropped
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
      if (kept && slot < p.cap_pages) p.page_va[slot] = va + ((uint64_t)lane << ushift);
      // the tile's kept units have consecutive slots from the first one's; those below the capacity are written
      const uint64_t slot0 = __shfl(slot, keep ? __builtin_ctz(keep) : 0, 64);
      const uint64_t n_kept = (uint64_t)__popc(keep);
      const uint64_t room = slot0 < p.cap_pages ? min(n_kept, p.cap_pages - slot0) : 0ull;
      dst = raw_rsrc((uint64_t)p.packed + (slot0 << ushift), (uint32_t)(room << ushift));
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        const uint64_t sj = __shfl(slot, 2 * j + half, 64);
        st_base[j] = ((keep >> (2 * j + half)) & 1u) ? (uint32_t)((sj - slot0) << ushift) : kOutside;
      }
    }
    // the tile's bytes, the last 16-byte block of a partial unit included (its bytes past the end are cleared
    // when staged); loads of skipped units read nothing
    const __amdgpu_buffer_rsrc_t src = raw_rsrc(va, ((last_pg << ushift) + last_len + 15u) & ~15u);
    uint32_t ld_base[8];
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) {
      const uint32_t pg = 2 * j + half;
      ld_base[j] = ((keep >> pg) & 1u) ? (pg << ushift) + off16 : kOutside;
    }
    uint32_t nonzero = 0;
    uint64_t acc = acc_init(p.seed, k);
    // this lane's quad: stripes of its unit, and the bytes past the last stripe
    const uint32_t qlen = q == last_pg ? last_len : unit;
    const uint32_t lim = qlen / 32u, rem = qlen & 31u;
    // offset of page pg's chunk in round c within a resource, or kOutside when that chunk is not in the unit
    auto at = [&](uint32_t base, uint32_t pg, uint32_t c) -> uint32_t {
      const uint32_t cp = c - pg * skew;  // wraps past n_chunks before the quad's first chunk
      return base != kOutside && cp < n_chunks ? base + cp * kChunk : kOutside;
    };
    auto load = [&](uint4 (&r)[8], uint32_t c) {
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        const v4u x = __builtin_amdgcn_raw_buffer_load_b128(src, at(ld_base[j], 2 * j + half, c), 0, kNt);
        r[j] = make_uint4(x[0], x[1], x[2], x[3]);
      }
    };
    // round c in r: stage (and store to the packed slots), reload r with round c + DEPTH, hash this quad's chunk
    auto step = [&](uint4 (&r)[8], uint32_t c) {
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        const uint32_t pg = 2 * j + half, cp = c - pg * skew;
        // outside the unit the load returned zeros; inside, a partial unit's bytes past its end are cleared
        const uint4 v = cp < n_chunks ? clip16(r[j], cp * kChunk + off16, pg == last_pg ? last_len : unit) : r[j];
        if (!GATHER) {
          const uint64_t b = __ballot(nz16(v));
          nonzero |= ((uint32_t)((uint32_t)b != 0u) << (2 * j)) | ((uint32_t)((b >> 32) != 0ull) << (2 * j + 1));
        }
        if (GATHER) {  // a partial unit's slot: zeros after its bytes
          const v4u x = {v.x, v.y, v.z, v.w};
          __builtin_amdgcn_raw_buffer_store_b128(x, dst, at(st_base[j], pg, c) + off16, 0, kNt);
        }
        *reinterpret_cast<uint4*>(stage + pg * kStageStride + off16) = v;
      }
      wave_lds_order();
      load(r, c + DEPTH);
      // the chunk's 16 words of this lane, read from the stage before the serial chain starts (one LDS wait)
      const uint32_t cq = c - q * skew;  // this quad's chunk; wraps past n_chunks while the quad idles
      const uint8_t* row = stage + q * kStageStride + k * 8u;
      uint64_t w[kChunk / 32];
#pragma unroll
      for (uint32_t s = 0; s < kChunk / 32; ++s) w[s] = *reinterpret_cast<const uint64_t*>(row + s * 32u);
      if (rem != 0u && cq == lim / (kChunk / 32))  // a partial unit's last bytes are in this chunk
        tail_lds[q][k] = *reinterpret_cast<const uint64_t*>(stage + q * kStageStride + (lim * 32u - cq * kChunk) + 8u * k);
      wave_lds_order();
      const uint32_t s_end = cq < n_chunks && lim > cq * (kChunk / 32) ? min(lim - cq * (kChunk / 32), kChunk / 32) : 0u;
#pragma unroll
      for (uint32_t s = 0; s < kChunk / 32; ++s)
        if (s < s_end) acc = xround(acc, w[s]);
    };
    uint4 r[DEPTH][8];
#pragma unroll
    for (uint32_t d = 0; d < DEPTH; ++d) {
      load(r[d], d);
      __builtin_amdgcn_sched_barrier(0);  // all of round d's loads before round d + 1's
    }
#pragma unroll 1
    for (uint32_t c = 0; c < n_rounds; c += DEPTH) {
#pragma unroll
      for (uint32_t d = 0; d < DEPTH; ++d) {
        step(r[d], c + d);
        __builtin_amdgcn_sched_barrier(0);  // the steps in program order: each round's loads behind the last's
      }
    }
    const uint64_t merged = xxh64_merge4(acc, k);  // every lane of the quad takes part
    uint64_t h = (lim > 0u ? merged : p.seed + kP5) + qlen;
    if (rem != 0u) {
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
  }
}

}  // namespace

hipError_t launch_page_hash_deep(const HashParams& p, bool gather, bool prior, uint32_t depth, uint32_t blocks,
                                 uint32_t waves_per_block, hipStream_t s) {
#define KC_DEEP_CASE(G, P, D)                                                                                 \
  if (gather == G && prior == P && depth == D) {                                                              \
    hipLaunchKernelGGL((k_page_hash_deep<G, P, D>), dim3(blocks), dim3(waves_per_block * kWave), 0, s, p);  \
    return hipGetLastError();                                                                                \
  }
  KC_DEEP_CASE(false, false, 2u)
  KC_DEEP_CASE(false, true, 2u)
  KC_DEEP_CASE(true, false, 2u)
  KC_DEEP_CASE(false, false, 3u)
  KC_DEEP_CASE(false, true, 3u)
  KC_DEEP_CASE(true, false, 3u)
  KC_DEEP_CASE(false, false, 4u)
  KC_DEEP_CASE(false, true, 4u)
  KC_DEEP_CASE(true, false, 4u)
#undef KC_DEEP_CASE
  return hipErrorInvalidValue;
}

}  // namespace kc

// kc_units.hip -- the hashing pass of hash units above 4 KiB (8 KiB to 2 MiB):
// a lane quad per unit at a time as in the 4 KiB pass, each quad hashing a run
// of one or more units in turn, with several chunks in flight per wave and the
// quads skewed over their runs' chunks.
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

// Bits of up to 64 consecutive units (bit i = unit g0 + i) OR-ed into a unit
// bitmap; one lane calls this.
__device__ __forceinline__ void or_unit_bits64(uint64_t* bm, uint32_t g0, uint32_t np, uint64_t bits) {
  if (bits == 0ull) return;
  const uint32_t w = g0 >> 6, s = g0 & 63u;
  if ((bits << s) != 0ull) atomicOr(reinterpret_cast<unsigned long long*>(bm + w), (unsigned long long)(bits << s));
  if (s != 0u && s + np > 64u && (bits >> (64u - s)) != 0ull)
    atomicOr(reinterpret_cast<unsigned long long*>(bm + w + 1), (unsigned long long)(bits >> (64u - s)));
}

// The hashing pass with DEPTH (2 to 4) chunks in flight per wave, for units
// above 4 KiB.  Large units give few tiles, about one wave per SIMD for 2 MiB
// units: with no other wave to switch to, a wave must cover the memory latency
// itself.  DEPTH register sets take turns: while round c is staged, stored and
// hashed, rounds c+1 .. c+DEPTH-1 are already loading, and the loads of round
// c+DEPTH are issued after round c's stores, so waiting for round c+1 never
// waits for those stores.
//
// A tile holds np <= 64 units of one range.  Its lane quads split them into
// runs of U = ceil(np / 16): quad q hashes units qU .. qU+U-1 one after the
// other, a stream of U * n_chunks chunks through contiguous bytes, and page row
// q of the stage always holds quad q's current chunk.  The quads run skewed:
// in round c, quad q works on chunk c - q*skew of its stream, skew = n_chunks /
// 32 clamped to 1..8.  The streams start U * 2^ushift bytes apart, so without
// the skew one load instruction's pieces (equal offsets in up to 16 streams)
// would all sit at addresses congruent modulo that; with it they are skew*512
// bytes apart in that congruence.  A tile takes, over its quads, at most
// (units of the quad) * n_chunks + q*skew rounds: a quad idles before its
// stream starts and after it ends, which with one unit per quad costs 60 of
// 188 rounds at 64 KiB units and with two 60 of 316.  Measured on the 30 GiB
// pool: 64 KiB units fastest at skew 4, 2 MiB units at skew 8 (15 % faster
// than skew 1, and than skew 16).  The range set decides the tiles: 32 units
// up to 256 KiB units when that still gives two waves per SIMD, else 16, or 8
// when 16 would give fewer than that; the kernel takes up to 64.
//
// The loads and stores go through buffer resources bounded to the tile's
// bytes and to its kept units' packed slots, so no lane branches around a
// memory access (a branch that may skip one leaves the compiler unsure how
// many are in flight, and it then waits for all of them): skipped units (zero
// units of a full snapshot, quads outside their stream) use an offset outside
// the resource.  When every unit of the tile is kept, a unit's packed slot
// offset equals its offset in the tile, so a store reuses its load's offset.
// A unit's hash is handed to the lane of its index when its quad finishes it
// and stored with the tile's bits at the tile's end, so no memory access waits
// inside the rounds either.  Every tile goes through it, a tile's partial last
// unit included; no closure scan (it runs as its own pass at units above
// 4 KiB).
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
  const uint32_t cshift = ushift - 9u, n_chunks = 1u << cshift;  // chunks of kChunk = 512 bytes per unit
  // chunks each quad starts after the one before it: 2 KiB apart at 64 KiB units, 4 KiB from 128 KiB up
  const uint32_t skew = min(8u, max(1u, n_chunks / 32u));
  const uint32_t hskew = half * skew;  // row 2j + half of load j starts 2j*skew + hskew rounds late
  const uint32_t wave = blockIdx.x * wpb + wv, n_waves = gridDim.x * wpb;
  for (uint32_t t = wave; t < p.n_tiles; t += n_waves) {
    const Tile tile = p.tiles[t];
    const uint32_t np = tile.npages;  // 1 .. 64 units
    const uint64_t va = tile.va;
    const uint32_t last = np - 1u, last_len = tile.last_len;  // only the last unit can be partial
    const uint32_t U = (np + kTilePages - 1u) / kTilePages;  // units per quad
    // chunks of quad row pg's stream (zero past the tile's units)
    auto stream_len = [&](uint32_t pg) -> uint32_t { return pg * U < np ? min(U, np - pg * U) << cshift : 0u; };
    uint32_t n_rounds = 0;  // the quad whose stream ends last
    for (uint32_t qq = 0; qq < kTilePages; ++qq)
      if (qq * U < np) n_rounds = max(n_rounds, stream_len(qq) + qq * skew);
    n_rounds = (n_rounds + DEPTH - 1u) / DEPTH * DEPTH;
    const uint64_t valid = np >= 64u ? ~0ull : (1ull << np) - 1ull;
    uint64_t keep = valid;
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
      keep = __ballot(kept);
      if (kept && slot < p.cap_pages) p.page_va[slot] = va + ((uint64_t)lane << ushift);
      // the tile's kept units have consecutive slots from the first one's; those below the capacity are written
      const uint64_t slot0 = __shfl(slot, keep ? (int)__builtin_ctzll(keep) : 0, 64);
      const uint64_t n_kept = (uint64_t)__popcll(keep);
      const uint64_t room = slot0 < p.cap_pages ? min(n_kept, p.cap_pages - slot0) : 0ull;
      dst = raw_rsrc((uint64_t)p.packed + (slot0 << ushift), (uint32_t)(room << ushift));
    }
    const bool all_kept = keep == valid;  // then a unit's slot offset is its offset in the tile
    uint64_t prior_l = 0;  // lane i < np: unit i's prior hash
    if (PRIOR && lane < np) prior_l = p.prior[tile.g + lane];
    // the tile's bytes, the last 16-byte block of a partial unit included (its bytes past the end are cleared
    // when staged); loads of skipped units read nothing
    const __amdgpu_buffer_rsrc_t src = raw_rsrc(va, ((last << ushift) + last_len + 15u) & ~15u);
    const bool partial = last_len != unit;
    // this lane's row of each load j (2j + half): its stream's length and first byte (+ the lane's 16 bytes)
    uint32_t len_j[8], base_j[8];
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) {
      const uint32_t pg = 2u * j + half;
      len_j[j] = stream_len(pg);
      base_j[j] = ((pg * U) << ushift) + off16;
    }
    // this lane's quad: its stream's length and first unit
    const uint32_t len_q = stream_len(q), unit0_q = q * U;
    const int from = (int)((min(lane, last) / U) * 4u);  // first lane of the quad holding unit `lane`
    uint64_t nonzero = 0;  // bit i: unit i holds a non-zero byte
    uint64_t hash_l = 0;   // lane i < np: unit i's hash, once its quad has finished it
    uint64_t acc = acc_init(p.seed, k);
    // round c into one register set: this lane's 16 bytes of each load j, and the offsets in the packed slots
    // the same bytes are stored to when the set is staged
    auto load = [&](uint4 (&rr)[8], uint32_t (&so)[8], uint32_t c) {
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        const uint32_t P = (c - 2u * j * skew) - hskew;  // stream position; wraps below zero before the start
        bool in = P < len_j[j];
        uint32_t ui = 0;
        if (!all_kept) {  // skipped units are not read
          ui = (base_j[j] >> ushift) + (P >> cshift);
          in = in && ((keep >> (ui & 63u)) & 1ull) != 0ull;
        }
        const uint32_t off = in ? base_j[j] + P * kChunk : kOutside;
        if (GATHER) {
          if (all_kept) {
            so[j] = off;
          } else {
            const uint32_t rel = (uint32_t)__popcll(keep & ((1ull << (ui & 63u)) - 1ull));
            so[j] = in ? (rel << ushift) + (P & (n_chunks - 1u)) * kChunk + off16 : kOutside;
          }
        }
        const v4u x = __builtin_amdgcn_raw_buffer_load_b128(src, off, 0, kNt);
        rr[j] = make_uint4(x[0], x[1], x[2], x[3]);
      }
    };
    // round c in rr: stage (and store to the packed slots), reload rr with round c + DEPTH, hash each quad's
    // chunk
    auto step = [&](uint4 (&rr)[8], uint32_t (&so)[8], uint32_t c) {
#pragma unroll
      for (uint32_t j = 0; j < 8; ++j) {
        uint4 v = rr[j];  // zeros where the load was outside
        if (partial) {  // the partial unit's bytes past its end
          const uint32_t P = (c - 2u * j * skew) - hskew;
          if (P < len_j[j] && (base_j[j] >> ushift) + (P >> cshift) == last)
            v = clip16(v, (P & (n_chunks - 1u)) * kChunk + off16, last_len);
        }
        if (!GATHER) {
          const uint64_t b = __ballot(nz16(v));
          if ((uint32_t)b != 0u) nonzero |= 1ull << ((2u * j * U + ((c - 2u * j * skew) >> cshift)) & 63u);
          if ((b >> 32) != 0ull)
            nonzero |= 1ull << (((2u * j + 1u) * U + ((c - (2u * j + 1u) * skew) >> cshift)) & 63u);
        }
        if (GATHER) {  // a partial unit's slot: zeros after its bytes
          const v4u x = {v.x, v.y, v.z, v.w};
          __builtin_amdgcn_raw_buffer_store_b128(x, dst, so[j], 0, kNt);
        }
        *reinterpret_cast<uint4*>(stage + (2u * j + half) * kStageStride + off16) = v;
      }
      wave_lds_order();
      load(rr, so, c + DEPTH);
      // this quad's unit and chunk; its 16 words of the chunk, read from the stage before the serial chain
      // starts (one LDS wait)
      const uint32_t Pq = c - q * skew;
      const bool act = Pq < len_q;
      const uint32_t cq = Pq & (n_chunks - 1u), uiq = unit0_q + (Pq >> cshift);
      const uint32_t qlen = act && uiq == last ? last_len : unit;
      const uint32_t lim = qlen / 32u, rem = qlen & 31u;
      const uint8_t* row = stage + q * kStageStride + k * 8u;
      uint64_t w[kChunk / 32];
#pragma unroll
      for (uint32_t s = 0; s < kChunk / 32; ++s) w[s] = *reinterpret_cast<const uint64_t*>(row + s * 32u);
      if (act && rem != 0u && cq == lim / (kChunk / 32))  // a partial unit's last bytes are in this chunk
        tail_lds[q][k] = *reinterpret_cast<const uint64_t*>(stage + q * kStageStride + (lim * 32u - cq * kChunk) + 8u * k);
      wave_lds_order();
      const uint32_t s_end = act && lim > cq * (kChunk / 32) ? min(lim - cq * (kChunk / 32), kChunk / 32) : 0u;
      if (__ballot(s_end != kChunk / 32) == 0ull) {  // every quad hashes a whole chunk
#pragma unroll
        for (uint32_t s = 0; s < kChunk / 32; ++s) acc = xround(acc, w[s]);
      } else {
#pragma unroll
        for (uint32_t s = 0; s < kChunk / 32; ++s)
          if (s < s_end) acc = xround(acc, w[s]);
      }
      const bool fin = act && cq == n_chunks - 1u;  // the quad's unit ends with this chunk
      if (__ballot(fin) != 0ull) {
        const uint64_t merged = xxh64_merge4(acc, k);  // every lane of the quad takes part
        uint64_t h = (lim > 0u ? merged : p.seed + kP5) + qlen;
        if (rem != 0u) {
          const uint64_t tail[4] = {tail_lds[q][0], tail_lds[q][1], tail_lds[q][2], tail_lds[q][3]};
          h = xxh64_tail(h, tail, rem);
        }
        h = xxh64_avalanche(h);
        // unit i's hash to lane i, from the first lane of the quad holding it
        const uint64_t hq = __shfl(h, from, 64);
        const uint32_t done = __shfl(fin ? uiq : 0xFFFFFFFFu, from, 64);
        if (done == lane) hash_l = hq;
        if (fin) acc = acc_init(p.seed, k);
      }
    };
    uint4 r[DEPTH][8];
    uint32_t so[DEPTH][8];
#pragma unroll
    for (uint32_t d = 0; d < DEPTH; ++d) {
      load(r[d], so[d], d);
      __builtin_amdgcn_sched_barrier(0);  // all of round d's loads before round d + 1's
    }
#pragma unroll 1
    for (uint32_t c = 0; c < n_rounds; c += DEPTH) {
#pragma unroll
      for (uint32_t d = 0; d < DEPTH; ++d) {
        step(r[d], so[d], c + d);
        __builtin_amdgcn_sched_barrier(0);  // the steps in program order: each round's loads behind the last's
      }
    }
    if (lane < np) p.hash[tile.g + lane] = hash_l;
    if (!GATHER) {
      const uint64_t zero = ~nonzero & valid;
      if (lane == 0) or_unit_bits64(p.zero_bm, tile.g, np, zero);
    }
    if (PRIOR) {
      const uint64_t ch = __ballot(lane < np && hash_l != prior_l);
      if (lane == 0) or_unit_bits64(p.changed_bm, tile.g, np, ch);
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

// kc_xxh64.h -- device-side XXH64 with one lane quad per hash unit, and the
// bitmap helpers shared by the hashing passes (the 4 KiB pass and the
// pipelined pass of larger units).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kc {

// ---------------------------------------------------------------- XXH64 ----
// Public xxHash definition: four accumulators over 32-byte stripes.
constexpr uint64_t kP1 = 0x9E3779B185EBCA87ull;
constexpr uint64_t kP2 = 0xC2B2AE3D27D4EB4Full;
constexpr uint64_t kP3 = 0x165667B19E3779F9ull;
constexpr uint64_t kP4 = 0x85EBCA77C2B2AE63ull;
constexpr uint64_t kP5 = 0x27D4EB2F165667C5ull;

__device__ __forceinline__ uint64_t rotl64(uint64_t x, uint32_t r) {
  return (x << r) | (x >> (64u - r));
}

__device__ __forceinline__ uint64_t xround(uint64_t acc, uint64_t in) {
  acc += in * kP2;
  acc = rotl64(acc, 31);
  return acc * kP1;
}

// 64-bit DPP move inside a lane quad (quad_perm control word).
template <int CTRL>
__device__ __forceinline__ uint64_t quad64(uint64_t x) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, 0xF, 0xF, true);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Lane k of a quad holds accumulator k of one page after its stripes.
// Returns the merged accumulators (before the length is added) in every lane
// of the quad.
__device__ __forceinline__ uint64_t xxh64_merge4(uint64_t acc, uint32_t k) {
  const uint32_t rot = k == 0 ? 1u : (k == 1 ? 7u : (k == 2 ? 12u : 18u));
  uint64_t r = rotl64(acc, rot);
  const uint64_t m = xround(0, acc);
  r += quad64<0xB1>(r);  // quad_perm(1,0,3,2)
  r += quad64<0x4E>(r);  // quad_perm(2,3,0,1)
  uint64_t h = r;
  h = (h ^ quad64<0x00>(m)) * kP1 + kP4;
  h = (h ^ quad64<0x55>(m)) * kP1 + kP4;
  h = (h ^ quad64<0xAA>(m)) * kP1 + kP4;
  h = (h ^ quad64<0xFF>(m)) * kP1 + kP4;
  return h;
}

// The bytes past the last whole 32-byte stripe (r = 1..31 of them, held
// little-endian in t[0..3]): 8-byte lanes, then a 4-byte lane, then bytes.
__device__ __forceinline__ uint64_t xxh64_tail(uint64_t h, const uint64_t (&t)[4], uint32_t r) {
#pragma unroll
  for (uint32_t i = 0; i < 3; ++i)
    if (r >= 8u * (i + 1u)) h = rotl64(h ^ xround(0, t[i]), 27) * kP1 + kP4;
  const uint32_t n8 = r >> 3;
  const uint64_t rest = n8 == 0 ? t[0] : (n8 == 1 ? t[1] : (n8 == 2 ? t[2] : t[3]));
  uint32_t rr = r & 7u, sh = 0;
  if (rr >= 4u) {
    h = rotl64(h ^ (uint64_t)(uint32_t)rest * kP1, 23) * kP2 + kP3;
    sh = 32u;
    rr -= 4u;
  }
#pragma unroll
  for (uint32_t i = 0; i < 3; ++i)
    if (i < rr) h = rotl64(h ^ ((rest >> (sh + 8u * i)) & 0xFFull) * kP5, 11) * kP1;
  return h;
}

__device__ __forceinline__ uint64_t xxh64_avalanche(uint64_t h) {
  h ^= h >> 33;
  h *= kP2;
  h ^= h >> 29;
  h *= kP3;
  h ^= h >> 32;
  return h;
}

__device__ __forceinline__ uint64_t acc_init(uint64_t seed, uint32_t k) {
  return k == 0 ? seed + kP1 + kP2 : (k == 1 ? seed + kP2 : (k == 2 ? seed : seed - kP1));
}

// ------------------------------------------------------------- helpers ----
__device__ __forceinline__ bool nz16(uint4 v) { return (v.x | v.y | v.z | v.w) != 0u; }

// OR page bits (bit i = page g0+i) into a bitmap; one lane calls this.
__device__ __forceinline__ void or_page_bits(uint64_t* bm, uint32_t g0, uint32_t np, uint32_t bits) {
  if (bits == 0u) return;
  const uint32_t w = g0 >> 6, s = g0 & 63u;
  const uint64_t b = (uint64_t)bits;
  if ((b << s) != 0ull) atomicOr(reinterpret_cast<unsigned long long*>(bm + w), (unsigned long long)(b << s));
  if (s + np > 64u && (b >> (64u - s)) != 0ull)
    atomicOr(reinterpret_cast<unsigned long long*>(bm + w + 1), (unsigned long long)(b >> (64u - s)));
}

// Compress ballot bits at lanes 4q (q < 16) into bit q.
__device__ __forceinline__ uint32_t quad_bits(uint64_t ballot) {
  uint32_t out = 0;
#pragma unroll
  for (uint32_t q = 0; q < 16; ++q) out |= (uint32_t)((ballot >> (4u * q)) & 1ull) << q;
  return out;
}

constexpr uint32_t kHashWaves = 4;  // most waves per workgroup of a hashing pass

}  // namespace kc

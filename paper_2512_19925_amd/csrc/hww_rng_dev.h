// Device side of the random-number keying contract: Philox4x32-10 with
// key (seed, (replica << 4) | slot) and counter (src, lineage lo, lineage
// hi, event index), and the uniforms made from its words.
#pragma once

#include "hww_internal.h"

namespace hww {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the two published
// 32x32 -> 64 multiplies; key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ void draw(uint32_t seed, uint32_t key1, int slot, uint32_t src,
                                     uint64_t lin, uint32_t e, uint32_t r[4]) {
  r[0] = src;
  r[1] = (uint32_t)lin;
  r[2] = (uint32_t)(lin >> 32);
  r[3] = e;
  uint32_t k0 = seed, k1 = key1 | (uint32_t)slot;
  // Keep the round-key schedule local to each draw: otherwise it is hoisted
  // out of the particle loop for every slot and exhausts the scalar registers.
  asm volatile("" : "+s"(k0), "+s"(k1));
  philox4x32_10(r, k0, k1);
}

// Same draw with a slot that differs between lanes (the key's second word
// then lives in a vector register).
__device__ __forceinline__ void draw_lane(uint32_t seed, uint32_t key1, int slot, uint32_t src,
                                          uint64_t lin, uint32_t e, uint32_t r[4]) {
  r[0] = src;
  r[1] = (uint32_t)lin;
  r[2] = (uint32_t)(lin >> 32);
  r[3] = e;
  uint32_t k0 = seed, k1 = key1 | (uint32_t)slot;
  asm volatile("" : "+s"(k0), "+v"(k1));
  philox4x32_10(r, k0, k1);
}

// 53-bit uniform on [0,1) from the high bits of two words.
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  const double k = (double)(a >> 5) * 67108864.0 + (double)(b >> 6);
  return k * (1.0 / 9007199254740992.0);
}

// Uniform on [0,1) in the flight precision: 53 bits (FP64) or the 24 high
// bits of the first word (FP32); 1 - u is exact in both.
template <typename Real>
__device__ __forceinline__ Real uflight(uint32_t a, uint32_t b);
template <>
__device__ __forceinline__ double uflight<double>(uint32_t a, uint32_t b) { return u53(a, b); }
template <>
__device__ __forceinline__ float uflight<float>(uint32_t a, uint32_t) {
  return (float)(a >> 8) * (1.0f / 16777216.0f);
}
}  // namespace hww

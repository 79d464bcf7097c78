// philox.h -- device Philox4x32-10 counter-based generator.
//
// Every sample point is drawn from one counter space, so no random number is
// ever used twice (the master-worker invariant of Sect. 2, kept here without a
// master: a point's words depend only on (seed, stream, iteration, point,
// dimension block), never on which lane or block computes it).
// Generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).
// A round maps (c0,c1,c2,c3) under key (k0,k1) to
//   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
// and the key advances by the Weyl increments between rounds.
#pragma once
#ifndef CCUBA_RTC  // (hiprtc provides the HIP runtime and its integer types)
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

namespace ccuba {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // full 64-bit products: one v_mad_u64_u32 each instead of mul_lo + mul_hi
    const uint64_t p0 = (uint64_t)M0 * (uint64_t)c.x;
    const uint64_t p1 = (uint64_t)M1 * (uint64_t)c.z;
    // three-way xors as one gfx950 three-input bit operation (truth table
    // 0x96 = a ^ b ^ c) instead of two v_xor_b32
    c = U4{(uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96),
           (uint32_t)p1,
           (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96),
           (uint32_t)p0};
    k0 += W0;
    k1 += W1;
  }
  return c;
}

}  // namespace ccuba

// philox.cpp -- oracle: Philox4x32-10 (TEST INFRASTRUCTURE ONLY).
//
// The paper requires that the samples come from one source so that no random
// number is used twice (Sect. 2); it names no generator.  The reading taken
// is the counter-based Philox4x32 with 10 rounds of Salmon et al. (SC'11),
// written here from that paper's definition:
//   one round maps counter (c0,c1,c2,c3) under key (k0,k1) to
//     (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
//   with M0 = 0xD2511F53, M1 = 0xCD9E8D57 (32x32 -> 64-bit products), and the
//   key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between
//   rounds.
#include "oracle.h"

namespace {

const uint32_t kM0 = 0xD2511F53u;
const uint32_t kM1 = 0xCD9E8D57u;
const uint32_t kW0 = 0x9E3779B9u;
const uint32_t kW1 = 0xBB67AE85u;

void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)kM0 * (uint64_t)c[0];
  const uint64_t p1 = (uint64_t)kM1 * (uint64_t)c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0];
  const uint32_t n1 = lo1;
  const uint32_t n2 = hi0 ^ c[3] ^ k[1];
  const uint32_t n3 = lo0;
  c[0] = n0;
  c[1] = n1;
  c[2] = n2;
  c[3] = n3;
}

}  // namespace

extern "C" void oracle_philox4x32_10(const uint32_t ctr[4],
                                     const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k[0] += kW0;
      k[1] += kW1;
    }
    philox_round(c, k);
  }
  out[0] = c[0];
  out[1] = c[1];
  out[2] = c[2];
  out[3] = c[3];
}

// philox_dev.h -- Philox4x64-10 counter-based generator for device code.
//
// Published definition: Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
// as easy as 1, 2, 3" (SC'11).  Four 64-bit counter words, two 64-bit key
// words, ten rounds.  Each round multiplies counter words 0 and 2 by the
// constants M0 and M1 (full 128-bit products); the new words are
//   (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)),
// and the key advances by the Weyl increments W0, W1 before every round but
// the first.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace snn {

struct U64x4 { uint64_t w[4]; };

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0_hi = __umul64hi(M0, c0), p0_lo = M0 * c0;
    const uint64_t p1_hi = __umul64hi(M1, c2), p1_lo = M1 * c2;
    const uint64_t n0 = p1_hi ^ c1 ^ k0;
    const uint64_t n2 = p0_hi ^ c3 ^ k1;
    c0 = n0; c1 = p1_lo; c2 = n2; c3 = p0_lo;
    k0 += W0; k1 += W1;
  }
  U64x4 r;
  r.w[0] = c0; r.w[1] = c1; r.w[2] = c2; r.w[3] = c3;
  return r;
}

// Philox key for round r is (k0 + r W0, k1 + r W1); the loop above adds the
// increment after each round, which gives the same sequence of round keys.

}  // namespace snn

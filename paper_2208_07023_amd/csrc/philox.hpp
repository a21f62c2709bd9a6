// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
// Easy as 1, 2, 3", SC'11, Sec. 4.2) on the device: a 4x32-bit counter and a
// 2x32-bit key; every round multiplies counter words 0 and 2 by fixed
// constants, recombines the halves of the products with the other words and
// the round key, and the key is bumped by two Weyl constants between rounds.
// Every draw of this library is a pure function of (counter, 64-bit seed).
//
// Counter word 1 separates the draw streams:
//   t (iterations of a swarm, 1..T) and INIT_STREAM: r1, r2 and the start;
//   PS_STREAM + t: probabilistic search candidates;
//   BOOT_STREAM: bootstrap samples of a forest (word 2 NO_NODE).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace slm {

constexpr uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;
constexpr uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;
constexpr uint32_t INIT_STREAM = 0xFFFFFFFFu;
constexpr uint32_t PS_STREAM = 0x40000000u;
constexpr uint32_t BOOT_STREAM = 0x80000000u;
constexpr uint32_t NO_NODE = 0xFFFFFFFFu;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += PH_W0;
      k.y += PH_W1;
    }
    const uint32_t lo0 = PH_M0 * c.x, hi0 = __umulhi(PH_M0, c.x);
    const uint32_t lo1 = PH_M1 * c.z, hi1 = __umulhi(PH_M1, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

// uint32 word -> uniform double in [0, 1) with 24 bits
__device__ __forceinline__ double u24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }

}  // namespace slm

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of the 4 x 32-bit
// multiply-xor bijection with the Weyl key schedule; the counter-based generator of the thermal
// noise, the screening samples and the optimiser's candidates.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bpm {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += 0x9E3779B9u;
    k.y += 0xBB67AE85u;
  }
  return c;
}

// uniform in (0, 1) from one 32-bit word: (w + 1/2) 2^-32
__device__ __forceinline__ double philox_uniform(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

}  // namespace bpm

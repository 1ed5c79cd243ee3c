// Counter-based generator for the device: Philox4x32 with 10 rounds
// (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11).  A draw is a pure function of (counter, key), so any thread can
// produce the numbers of any synapse or neuron-step without shared state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpsnn {

// Stream tags carried in counter word 3 (block index in bits 8 and up).
constexpr uint32_t kTagSyn = 1;   // synapse j of source s: (s, j, 0, SYN)
constexpr uint32_t kTagExt = 2;   // Poisson counts of neurons 4g..4g+3 at t
constexpr uint32_t kTagExtJ = 3;  // external efficacies of neuron i at t
constexpr uint32_t kTagInit = 4;  // initial membrane potential of neuron i

__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// floor(u * n / 2^32)
__device__ __forceinline__ uint32_t scale32(uint32_t u, uint32_t n) {
  return __umulhi(u, n);
}

}  // namespace dpsnn

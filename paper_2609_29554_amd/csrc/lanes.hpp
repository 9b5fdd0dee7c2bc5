// Cross-lane primitives of one 64-lane wavefront: the vocabulary of the
// lane-distributed p-bit arithmetic in limbfp.hpp.  Every call must be made
// by all 64 lanes of a converged wavefront.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define LFP_FN __device__ __forceinline__

namespace lfp {

LFP_FN int lane_id() { return (int)__lane_id(); }

// bit l set when lane l's predicate holds
LFP_FN uint64_t ballot(bool p) { return (uint64_t)__builtin_amdgcn_ballot_w64(p); }

// lane l's x, for a wave-uniform l
LFP_FN uint64_t readlane64(uint64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// lane src's x (src in 0..63, any per-lane value)
LFP_FN uint64_t shfl64(uint64_t x, int src) {
  return (uint64_t)__shfl((unsigned long long)x, src, 64);
}

// a + b + cin (cin 0 or 1) on 32-bit words, the carry out in *cout
LFP_FN uint32_t addc32(uint32_t a, uint32_t b, uint32_t cin, uint32_t *cout) {
  unsigned c;
  const uint32_t r = __builtin_addc(a, b, cin, &c);
  *cout = c;
  return r;
}

// lane l's result is lane l-1's x, lane 0's is 0 (DPP whole-wave shift)
LFP_FN uint64_t up1_64(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, 0x138, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), 0x138, 0xf,
                                                            0xf, false);
  return ((uint64_t)hi << 32) | lo;
}

// lane l's result is lane (l-1) mod 64's x (DPP whole-wave rotation)
LFP_FN uint64_t rot1_64(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, 0x13C, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), 0x13C, 0xf,
                                                            0xf, false);
  return ((uint64_t)hi << 32) | lo;
}

}  // namespace lfp

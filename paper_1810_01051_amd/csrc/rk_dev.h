// Device helpers shared by every librk kernel: arithmetic mod q = 2^61 - 1,
// byte extraction, wave-uniform values, ballots and LDS-only barriers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rk_internal.h"

namespace rk {

// ------------------------------------------------------------ arithmetic mod q
// s < 2^63 on input; result < 2^61 + 2^10, congruent to 256*s.
__device__ __forceinline__ uint64_t mul256_lazy(uint64_t s) { return ((s << 8) & kQ) + (s >> 53); }
// s < 2^63 on input; result < 2^61 + 2^34 + ..., congruent to 2^32 * s.
__device__ __forceinline__ uint64_t mul2p32_lazy(uint64_t s) { return ((s << 32) & kQ) + (s >> 29); }
// canonical representative in [0, q) of s < 2^63
__device__ __forceinline__ uint64_t canon(uint64_t s) {
  uint64_t f = (s & kQ) + (s >> 61);  // < 2^61 + 4
  return f >= kQ ? f - kQ : f;
}
// v * 2^r mod q for v < 2^61, 0 <= r < 61 (a rotation of the 61-bit word)
__device__ __forceinline__ uint64_t rot61(uint64_t v, uint32_t r) {
  return ((v << r) & kQ) | (v >> ((61u - r) & 63u));
}

__device__ __forceinline__ uint32_t byte_at(const uint32_t *w, int i) {
  return (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }

// Workgroup barrier for LDS traffic only.  __syncthreads() would also wait for
// every outstanding load-to-LDS of the next tile (the compiler's release fence
// counts them), which would end the overlap of that tile's loads with the
// current tile's work; the tile pipeline waits for them explicitly instead.
__device__ __forceinline__ void wg_barrier() { __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// The same after this wave's loads-to-LDS have landed: after it, every wave's
// share of the tile is visible.
__device__ __forceinline__ void wg_barrier_loads() {
  __asm__ volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}


}  // namespace rk

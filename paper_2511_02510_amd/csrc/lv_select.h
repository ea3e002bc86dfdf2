// On-device k-th smallest selection (MSB-first radix select, 4 passes of 8
// bits over an order-preserving uint32 image of the float keys) for several
// segments at once.  Used for the nearest-rank percentiles of the loss weight
// (Sec. IV-B) and for the per-bin quantile cutoffs and depth percentiles
// (Sec. IV-C).  Exact: the result is an element of the segment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lv {

struct SelState {
  uint32_t prefix;  // decided high bits of the answer's key
  uint32_t k;       // rank (0-based) still to find among keys matching prefix
  uint32_t n;       // segment size
  uint32_t valid;   // 0: empty segment, no answer
};

__device__ __forceinline__ uint32_t f2key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key2f(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

__device__ __forceinline__ int sel_shift(int pass) { return 24 - 8 * pass; }
__device__ __forceinline__ uint32_t sel_himask(int pass) {
  return pass == 0 ? 0u : (0xFFFFFFFFu << (sel_shift(pass) + 8));
}

// One block per segment: pick the digit whose cumulative count passes k, then
// clear the segment's histogram for the next pass (defined in k_loss.hip).
hipError_t launch_sel_step(SelState* st, uint32_t* hist, int nseg, int pass, hipStream_t s);

}  // namespace lv

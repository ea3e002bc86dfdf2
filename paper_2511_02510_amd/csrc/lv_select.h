// On-device k-th smallest selection (MSB-first radix select, 4 passes of 8
// bits over an order-preserving uint32 image of the float keys) for several
// segments at once.  Used for the nearest-rank percentiles of the loss weight
// (Sec. IV-B) and for the per-bin quantile cutoffs and depth percentiles
// (Sec. IV-C).  Exact: the result is an element of the segment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lv {

// Block histograms are spread over lane-indexed copies, padded so that the
// copies of one bin fall in different LDS banks.
constexpr int kHistCopies = 16;
constexpr int kHistStride = 257;

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

// Digit choice of one pass for segments [0, nseg) after a histogram kernel
// has counted the current digit of every key that matches its segment's
// prefix (a separate launch, so the counts are complete and visible): one
// wave per segment, each lane holding 4 consecutive bins.  The wave scans the
// bin counts, keeps the digit whose cumulative count passes k, lowers k by
// the counts before it, and clears the bins for the next pass.
hipError_t launch_sel_step(SelState* st, uint32_t* hist, int nseg, int pass, hipStream_t s);

}  // namespace lv

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

// Digit choice of one pass for segments [0, nseg), run by the last block of a
// histogram kernel (256 threads): per segment, scan the 256 bin counts, keep
// the digit whose cumulative count passes k, lower k by the counts before it,
// and clear the bins for the next pass.  The counts were added by other
// blocks with device-scope atomics and are read back the same way.
__device__ __forceinline__ void sel_step_block(SelState* st, uint32_t* hist, int nseg, int pass) {
  __shared__ uint32_t s_w[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int s = 0; s < nseg; ++s) {
    SelState* S = st + s;
    uint32_t* h = hist + size_t(s) * 256;
    const uint32_t c = __hip_atomic_load(&h[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < w; ++q) add += s_w[q];
    const uint32_t incl = x + add;
    const uint32_t excl = incl - c;
    const uint32_t k = S->k;
    const bool valid = S->valid != 0;
    __syncthreads();
    if (valid && c > 0 && excl <= k && k < incl) {
      S->prefix = S->prefix | (uint32_t(t) << sel_shift(pass));
      S->k = k - excl;
    }
    h[t] = 0u;
    __syncthreads();
  }
}

// End of a histogram pass: every block publishes its counts, the last block
// to finish performs the digit choice and re-arms the counter.  Returns after
// the whole block agrees whether it was last.
__device__ __forceinline__ void sel_finish_pass(SelState* st, uint32_t* hist, int nseg, int pass,
                                                uint32_t* done) {
  __shared__ uint32_t s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t nblk = gridDim.x * gridDim.y;
    s_last = (atomicAdd(done, 1u) == nblk - 1u) ? 1u : 0u;
  }
  __syncthreads();
  if (s_last) {
    __threadfence();
    sel_step_block(st, hist, nseg, pass);
    if (threadIdx.x == 0) *done = 0u;
  }
}

}  // namespace lv

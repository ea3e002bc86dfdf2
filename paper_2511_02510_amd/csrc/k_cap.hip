// Capped selection (declared in lv_select.h): of the candidates among n
// items, the first min(cap, #candidates) in the order (key, index).  Used by
// the pruning guards' per-step cap (Sec. IV-C, guard iii; smallest moving
// average first) and by the budgeted selection of splits (Sec. IV-D; largest
// priority first, keys inverted).  The cap-th smallest candidate key comes
// from an exact 4-pass radix select; candidates equal to it are taken in
// index order by a block-ordered count, so the result does not depend on
// scheduling.
#include "lv_common.h"
#include "lv_select.h"

namespace lv {

static uint64_t n_cap_blocks(int64_t n) { return uint64_t((n + kCapPer - 1) / kCapPer); }

uint64_t cap_ws_bytes(int64_t n) {
  return align256(4 * size_t(n)) + align256(size_t(n)) + align256(4 * size_t(kCapFillBlocks)) +
         align256(4 * size_t(n_cap_blocks(n) + 1)) + align256(16) + align256(4 * 1024) +
         align256(2 * sizeof(SelState));
}

CapWS cap_bind(void* base, int64_t n) {
  char* b = static_cast<char*>(base);
  CapWS w;
  w.key = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(n));
  w.cand = reinterpret_cast<uint8_t*>(b); b += align256(size_t(n));
  w.ublk = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(kCapFillBlocks));
  w.eqblk = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(n_cap_blocks(n) + 1));
  w.cnt = reinterpret_cast<uint32_t*>(b); b += align256(16);
  w.sel.nseg = 1;
  w.sel.hist = reinterpret_cast<uint32_t*>(b); b += align256(4 * 1024);
  w.sel.st = reinterpret_cast<SelState*>(b);
  return w;
}

__global__ void k_cap_setup(CapWS w, uint32_t* count_out) {
  for (int k = threadIdx.x; k < 4 * 256; k += blockDim.x) w.sel.hist[k] = 0u;
  for (int k = threadIdx.x; k < kCapFillBlocks; k += blockDim.x) w.ublk[k] = 0u;
  if (threadIdx.x == 0) {
    w.cnt[0] = 0u;
    if (count_out) *count_out = 0u;
  }
}

hipError_t launch_cap_setup(const CapWS& w, uint32_t* count_out, hipStream_t s) {
  hipLaunchKernelGGL(k_cap_setup, dim3(1), dim3(256), 0, s, w, count_out);
  return hipGetLastError();
}

// Histogram of the current digit of the candidates' keys.  Pass 0 derives
// the initial state: with C candidates, the cap-th smallest is wanted only
// when 0 < cap < C (otherwise none or all of them are marked).
__global__ __launch_bounds__(256) void k_cap_hist(int64_t n, CapWS w, uint32_t cap, int pass) {
  __shared__ uint32_t lh[kHistCopies * kHistStride];
  __shared__ SelState s_st;
  for (int k = threadIdx.x; k < kHistCopies * kHistStride; k += 256) lh[k] = 0u;
  if (threadIdx.x < 64) {
    SelState st;
    if (pass == 0) {
      uint32_t c = 0;
      for (int k = threadIdx.x; k < kCapFillBlocks; k += 64) c += w.ublk[k];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) c += uint32_t(__shfl_xor(int(c), o, 64));
      st.prefix = 0u;
      st.n = c;
      st.valid = (cap > 0u && c > cap) ? 1u : 0u;
      st.k = cap > 0u ? cap - 1u : 0u;
      if (threadIdx.x == 0 && blockIdx.x == 0) w.cnt[0] = c;
    } else {
      st = sel_state(w.sel, 0, pass);
    }
    if (threadIdx.x == 0) {
      s_st = st;
      if (blockIdx.x == 0) sel_store(w.sel, 0, pass, st);
    }
  }
  __syncthreads();
  const SelState st = s_st;
  if (!st.valid) return;   // the whole block
  uint32_t* mine = lh + (threadIdx.x & (kHistCopies - 1)) * kHistStride;
  const int sh = sel_shift(pass);
  const uint32_t hm = sel_himask(pass);
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    if (!w.cand[i]) continue;
    const uint32_t key = w.key[i];
    if ((key & hm) == st.prefix) atomicAdd(&mine[(key >> sh) & 255u], 1u);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kHistCopies; ++i) c += lh[i * kHistStride + threadIdx.x];
  if (c) atomicAdd(&sel_hist(w.sel, pass, 0)[threadIdx.x], c);
}

// the cutoff (state after the last pass), by the first wave, into LDS
__device__ __forceinline__ void cap_cutoff(const CapWS& w, SelState* s_st) {
  if (threadIdx.x < 64) {
    const SelState st = sel_state(w.sel, 0, 4);
    if (threadIdx.x == 0) *s_st = st;
  }
  __syncthreads();
}

// candidates equal to the cutoff key, per fixed block of kCapPer items
__global__ __launch_bounds__(256) void k_cap_count(int64_t n, CapWS w) {
  __shared__ SelState s_st;
  __shared__ uint32_t s_c[4];
  cap_cutoff(w, &s_st);
  const SelState st = s_st;
  uint32_t mine = 0;
  if (st.valid) {
    const int64_t base = int64_t(blockIdx.x) * kCapPer;
    for (int r = 0; r < kCapPer / 256; ++r) {
      const int64_t i = base + r * 256 + threadIdx.x;
      if (i < n && w.cand[i] && w.key[i] == st.prefix) ++mine;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mine += uint32_t(__shfl_xor(int(mine), o, 64));
  if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) w.eqblk[blockIdx.x] = (s_c[0] + s_c[1]) + (s_c[2] + s_c[3]);
}

// the mask: below the cutoff, or equal to it and among the first (k + 1)
// such candidates in index order
__global__ __launch_bounds__(256) void k_cap_apply(int64_t n, CapWS w, uint32_t cap, uint8_t* mask,
                                                   uint32_t* count_out) {
  __shared__ SelState s_st;
  __shared__ uint32_t s_before, s_w[4];
  cap_cutoff(w, &s_st);
  const SelState st = s_st;
  const uint32_t C = w.cnt[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (st.valid && wave == 0) {   // equal candidates in the blocks before this one
    uint32_t c = 0;
    for (uint32_t k = lane; k < blockIdx.x; k += 64) c += w.eqblk[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += uint32_t(__shfl_xor(int(c), o, 64));
    if (lane == 0) s_before = c;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && count_out) *count_out = C < cap ? C : cap;
  __syncthreads();
  uint32_t run = st.valid ? s_before : 0u;
  const int64_t base = int64_t(blockIdx.x) * kCapPer;
  for (int r = 0; r < kCapPer / 256; ++r) {
    const int64_t i = base + r * 256 + threadIdx.x;
    const bool in = i < n;
    const bool cand = in && w.cand[i];
    const uint32_t key = cand ? w.key[i] : 0u;
    const bool eq = st.valid && cand && key == st.prefix;
    const unsigned long long b = __ballot(eq);
    const uint32_t below =
        __builtin_amdgcn_mbcnt_hi(uint32_t(b >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(b), 0u));
    if (lane == 0) s_w[wave] = uint32_t(__popcll(b));
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < wave; ++k) off += s_w[k];
    const uint32_t tot = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
    bool pick;
    if (cap == 0u) pick = false;
    else if (!st.valid) pick = cand;            // C <= cap: every candidate
    else pick = cand && (key < st.prefix || (eq && run + off + below <= st.k));
    if (in) mask[i] = pick ? 1u : 0u;
    run += tot;
    __syncthreads();
  }
}

hipError_t launch_cap_select(const CapWS& w, int64_t n, uint32_t cap, uint8_t* mask,
                             uint32_t* count_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const uint64_t ub = (uint64_t(n) + 255) / 256;
  const uint32_t hg = uint32_t(ub < uint64_t(kCapHistBlocks) ? ub : uint64_t(kCapHistBlocks));
  for (int pass = 0; pass < 4; ++pass)
    hipLaunchKernelGGL(k_cap_hist, dim3(hg), dim3(256), 0, s, n, w, cap, pass);
  const uint32_t fb = uint32_t(n_cap_blocks(n));
  hipLaunchKernelGGL(k_cap_count, dim3(fb), dim3(256), 0, s, n, w);
  hipLaunchKernelGGL(k_cap_apply, dim3(fb), dim3(256), 0, s, n, w, cap, mask, count_out);
  return hipGetLastError();
}

}  // namespace lv

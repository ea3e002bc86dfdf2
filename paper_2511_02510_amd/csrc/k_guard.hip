// Pruning stability guards (Sec. IV-C, guards i-iii), one adaptation step on
// top of the per-bin quantile decision (eq. 11-12):
//   x_v = [w_max_v > tau_{bin(v)}]                 inside score
//   i.   m_v <- (1 - alpha) m_v + alpha x_v;  s_v <- out if m_v < m_low,
//        in if m_v > m_high, else unchanged        (EMA + hysteresis)
//   ii.  protected: footprint finite and h_v < rho delta_v, or
//        w_max_v >= w_keep                         (keep-halo)
//   iii. candidates = out and not protected; the first min(cap, #candidates)
//        in the order (m_v, v) are pruned, cap = floor(cap_frac n)
//                                                  (per-step cap)
// Every decision is binary32 in the order written (built without
// contraction).  The cap is an exact selection on device: a 4-pass radix
// select of the cap-th smallest m among the candidates (lv_select.h), then
// the candidates equal to it are taken in index order with a block-ordered
// count.  Nothing returns to the host.
#include "lv_common.h"
#include "lv_select.h"

namespace lv {

// elements per block of the update and histogram passes (grid-stride) and
// of the block-ordered passes (fixed partition)
constexpr int kGuardUpdateBlocks = 1024;
constexpr int kGuardHistBlocks = 256;
constexpr int kGuardPer = 2048;

struct GuardWS {
  uint32_t* key;     // [n] order image of m (candidates only)
  uint8_t* cand;     // [n]
  uint32_t* ublk;    // [kGuardUpdateBlocks] candidates per update block
  uint32_t* eqblk;   // [ceil(n / kGuardPer)] candidates equal to the cutoff per block
  uint32_t* cnt;     // [0] candidates
  SelSet sel;        // one selection: hist [4][256], st [2]
};

static uint64_t n_fixed_blocks(int64_t n) { return uint64_t((n + kGuardPer - 1) / kGuardPer); }

uint64_t guard_ws_bytes(int64_t n) {
  return align256(4 * size_t(n)) + align256(size_t(n)) + align256(4 * size_t(kGuardUpdateBlocks)) +
         align256(4 * size_t(n_fixed_blocks(n) + 1)) + align256(16) + align256(4 * 1024) +
         align256(2 * sizeof(SelState));
}

static GuardWS guard_bind(void* base, int64_t n) {
  char* b = static_cast<char*>(base);
  GuardWS w;
  w.key = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(n));
  w.cand = reinterpret_cast<uint8_t*>(b); b += align256(size_t(n));
  w.ublk = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(kGuardUpdateBlocks));
  w.eqblk = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(n_fixed_blocks(n) + 1));
  w.cnt = reinterpret_cast<uint32_t*>(b); b += align256(16);
  w.sel.nseg = 1;
  w.sel.hist = reinterpret_cast<uint32_t*>(b); b += align256(4 * 1024);
  w.sel.st = reinterpret_cast<SelState*>(b);
  return w;
}

__global__ void k_guard_setup(GuardWS w, uint32_t* n_pruned) {
  for (int k = threadIdx.x; k < 4 * 256; k += blockDim.x) w.sel.hist[k] = 0u;
  for (int k = threadIdx.x; k < kGuardUpdateBlocks; k += blockDim.x) w.ublk[k] = 0u;
  if (threadIdx.x == 0) {
    w.cnt[0] = 0u;
    if (n_pruned) *n_pruned = 0u;
  }
}

// guards i and ii per voxel; each block writes its candidate count
__global__ __launch_bounds__(256) void k_guard_update(RasterArgs a, const uint8_t* bins,
                                                      const float* tau, int nb, GuardParams p,
                                                      float* ema, uint8_t* state, GuardWS w) {
  __shared__ uint32_t s_c[4];
  uint32_t mine = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * 256) {
    const float wm = a.wmax[i];
    int b = bins[i];
    if (b >= nb) b = nb - 1;
    const float x = wm > tau[b] ? 1.0f : 0.0f;
    const float m = (1.0f - p.alpha) * ema[i] + p.alpha * x;
    uint8_t s = state[i];
    s = m < p.m_low ? uint8_t(0) : (m > p.m_high ? uint8_t(1) : s);
    const float delta = voxel_footprint(a, i);
    const float h = 0.5f * ldexpf(a.root_size, -int(a.level[i]));
    const bool prot = (isfinite(delta) && h < p.rho * delta) || wm >= p.w_keep;
    const bool cand = s == 0 && !prot;
    ema[i] = m;
    state[i] = s;
    w.key[i] = f2key(m);
    w.cand[i] = cand ? 1u : 0u;
    mine += cand ? 1u : 0u;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mine += uint32_t(__shfl_xor(int(mine), o, 64));
  if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) w.ublk[blockIdx.x] = (s_c[0] + s_c[1]) + (s_c[2] + s_c[3]);
}

// Histogram of the current digit of the candidates' keys.  Pass 0 derives
// the initial state: with C candidates, the (cap)-th smallest is wanted only
// when 0 < cap < C (otherwise none or all of them are pruned).
__global__ __launch_bounds__(256) void k_guard_hist(int64_t n, GuardWS w, uint32_t cap, int pass) {
  __shared__ uint32_t lh[kHistCopies * kHistStride];
  __shared__ SelState s_st;
  for (int k = threadIdx.x; k < kHistCopies * kHistStride; k += 256) lh[k] = 0u;
  if (threadIdx.x < 64) {
    SelState st;
    if (pass == 0) {
      uint32_t c = 0;
      for (int k = threadIdx.x; k < kGuardUpdateBlocks; k += 64) c += w.ublk[k];
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
__device__ __forceinline__ void guard_cutoff(const GuardWS& w, SelState* s_st) {
  if (threadIdx.x < 64) {
    const SelState st = sel_state(w.sel, 0, 4);
    if (threadIdx.x == 0) *s_st = st;
  }
  __syncthreads();
}

// candidates equal to the cutoff key, per fixed block of kGuardPer voxels
__global__ __launch_bounds__(256) void k_guard_count(int64_t n, GuardWS w) {
  __shared__ SelState s_st;
  __shared__ uint32_t s_c[4];
  guard_cutoff(w, &s_st);
  const SelState st = s_st;
  uint32_t mine = 0;
  if (st.valid) {
    const int64_t base = int64_t(blockIdx.x) * kGuardPer;
    for (int r = 0; r < kGuardPer / 256; ++r) {
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

// the prune mask: below the cutoff, or equal to it and among the first
// (k + 1) such candidates in index order
__global__ __launch_bounds__(256) void k_guard_apply(int64_t n, GuardWS w, uint32_t cap,
                                                     uint8_t* prune, uint32_t* n_pruned) {
  __shared__ SelState s_st;
  __shared__ uint32_t s_before, s_w[4];
  guard_cutoff(w, &s_st);
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
  if (blockIdx.x == 0 && threadIdx.x == 0 && n_pruned) *n_pruned = C < cap ? C : cap;
  __syncthreads();
  uint32_t run = st.valid ? s_before : 0u;
  const int64_t base = int64_t(blockIdx.x) * kGuardPer;
  for (int r = 0; r < kGuardPer / 256; ++r) {
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
    bool pr;
    if (cap == 0u) pr = false;
    else if (!st.valid) pr = cand;            // C <= cap: every candidate
    else pr = cand && (key < st.prefix || (eq && run + off + below <= st.k));
    if (in) prune[i] = pr ? 1u : 0u;
    run += tot;
    __syncthreads();
  }
}

hipError_t run_prune_guard(const RasterArgs& a, const uint8_t* bins, const float* tau, int nb,
                           const GuardParams& p, void* ws, float* ema, uint8_t* state,
                           uint8_t* prune, uint32_t* n_pruned, hipStream_t s) {
  GuardWS w = guard_bind(ws, a.n);
  hipLaunchKernelGGL(k_guard_setup, dim3(1), dim3(256), 0, s, w, n_pruned);
  if (a.n == 0) return hipGetLastError();
  const uint64_t ub = (uint64_t(a.n) + 255) / 256;
  const uint32_t ug = uint32_t(ub < uint64_t(kGuardUpdateBlocks) ? ub : uint64_t(kGuardUpdateBlocks));
  hipLaunchKernelGGL(k_guard_update, dim3(ug), dim3(256), 0, s, a, bins, tau, nb, p, ema, state, w);
  const uint32_t hg = uint32_t(ub < uint64_t(kGuardHistBlocks) ? ub : uint64_t(kGuardHistBlocks));
  for (int pass = 0; pass < 4; ++pass)
    hipLaunchKernelGGL(k_guard_hist, dim3(hg), dim3(256), 0, s, a.n, w, p.cap, pass);
  const uint32_t fb = uint32_t(n_fixed_blocks(a.n));
  hipLaunchKernelGGL(k_guard_count, dim3(fb), dim3(256), 0, s, a.n, w);
  hipLaunchKernelGGL(k_guard_apply, dim3(fb), dim3(256), 0, s, a.n, w, p.cap, prune, n_pruned);
  return hipGetLastError();
}

}  // namespace lv

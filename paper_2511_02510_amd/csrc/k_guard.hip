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
// contraction).  The cap is the exact capped selection of lv_select.h on
// keys = the order image of m.  Nothing returns to the host.
#include "lv_common.h"
#include "lv_select.h"

namespace lv {

uint64_t guard_ws_bytes(int64_t n) { return cap_ws_bytes(n); }

// guards i and ii per voxel (grid-stride, at most kCapFillBlocks blocks):
// the candidates and their keys for the capped selection
__global__ __launch_bounds__(256) void k_guard_update(RasterArgs a, const uint8_t* bins,
                                                      const float* tau, int nb, GuardParams p,
                                                      float* ema, uint8_t* state, CapWS w) {
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
  cap_store_block_count(w, mine);
}

hipError_t run_prune_guard(const RasterArgs& a, const uint8_t* bins, const float* tau, int nb,
                           const GuardParams& p, void* ws, float* ema, uint8_t* state,
                           uint8_t* prune, uint32_t* n_pruned, hipStream_t s) {
  const CapWS w = cap_bind(ws, a.n);
  hipError_t e = launch_cap_setup(w, n_pruned, s);
  if (e != hipSuccess || a.n == 0) return e;
  const uint64_t ub = (uint64_t(a.n) + 255) / 256;
  const uint32_t ug = uint32_t(ub < uint64_t(kCapFillBlocks) ? ub : uint64_t(kCapFillBlocks));
  hipLaunchKernelGGL(k_guard_update, dim3(ug), dim3(256), 0, s, a, bins, tau, nb, p, ema, state, w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_cap_select(w, a.n, p.cap, prune, n_pruned, s);
}

}  // namespace lv

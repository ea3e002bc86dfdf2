// Depth-aware quantile cutoff for pruning (Sec. IV-C, eq. 11-12, with the
// eq. 14 robust depth normalisation).
//   1. delta_v = min over views with z_c > 0 of z_c / fx at the voxel centre
//      (the inter-ray spacing there, the paper's depth proxy; binary32 ops
//      in a fixed order so the bin decision is exact);
//   2. p5, p95 = nearest-rank percentiles of delta over all voxels;
//   3. z~ = clip((delta - p5) / (p95 - p5), 0, 1), bin = min(B-1, floor(B z~));
//   4. tau_b = ceil(q |V_b|)-th smallest w_max of bin b (the generalised
//      inverse of the bin's empirical CDF), prune = w_max <= tau_bin.
// All selections are exact radix selects on device (p5 and p95 in the same
// passes); nothing returns to the host.  Steps 1-3 do not read w_max and run
// as one call (the binning), step 4 as another (the cutoff) on the
// binning's workspace, so the binning can run before the forward pass.
#include "lv_common.h"
#include "lv_select.h"

namespace lv {

struct QuantWS {
  uint32_t* dkey;     // [n] keys of delta
  uint8_t* bins;      // [n]
  SelSet pct;         // p5 and p95 of delta (2 segments)
  SelSet bin;         // the quantile of w_max in each bin (B segments)
  uint32_t* cnt;      // [B]
};

static size_t sel_bytes(int nseg) {
  return align256(size_t(4) * nseg * 1024) + align256(size_t(2) * nseg * sizeof(SelState));
}

uint64_t quant_ws_bytes(int64_t n, int B) {
  return align256(4 * size_t(n)) + align256(size_t(n)) + sel_bytes(2) + sel_bytes(B) +
         align256(4 * size_t(B));
}

static char* sel_bind(char* b, int nseg, SelSet& S) {
  S.nseg = nseg;
  S.hist = reinterpret_cast<uint32_t*>(b);
  b += align256(size_t(4) * nseg * 1024);
  S.st = reinterpret_cast<SelState*>(b);
  return b + align256(size_t(2) * nseg * sizeof(SelState));
}

static QuantWS quant_bind(void* base, int64_t n, int B) {
  char* b = static_cast<char*>(base);
  QuantWS w;
  w.dkey = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(n));
  w.bins = reinterpret_cast<uint8_t*>(b); b += align256(size_t(n));
  b = sel_bind(b, 2, w.pct);
  b = sel_bind(b, B, w.bin);
  w.cnt = reinterpret_cast<uint32_t*>(b);
  return w;
}

constexpr int kMaxBins = 64;   // n_bins accepted by the entry point
constexpr int kUnroll = 8;

__device__ __forceinline__ uint32_t rank_of(double q, uint32_t n) {
  double r = ceil(q * double(n));
  if (r < 1.0) r = 1.0;
  if (r > double(n)) r = double(n);
  return uint32_t(r) - 1u;
}

// part 0 (binning), block s < 2: percentile segment s, and the bin counts;
// part 1 (cutoff), block b: bin b, whose initial state comes from the bin
// counts in the first histogram pass.  Until then both rows say "no
// answer", which is also the result when there are no voxels.
__global__ void k_q_setup(QuantWS w, int B, uint32_t n, int part) {
  const int sg = blockIdx.x;
  const SelSet& S = part == 0 ? w.pct : w.bin;
  for (int pass = 0; pass < 4; ++pass) sel_hist(S, pass, sg)[threadIdx.x] = 0u;
  if (part == 0 && sg == 0)
    for (int k = threadIdx.x; k < B; k += blockDim.x) w.cnt[k] = 0u;
  if (threadIdx.x == 0) {
    SelState st;
    st.prefix = 0u;
    st.n = part == 0 ? n : 0u;
    st.valid = (part == 0 && n > 0) ? 1u : 0u;
    st.k = part == 0 ? rank_of(sg == 0 ? 0.05 : 0.95, n) : 0u;
    sel_store(S, sg, 0, st);
    sel_store(S, sg, 1, st);
  }
}

__global__ __launch_bounds__(256) void k_q_delta(RasterArgs a, QuantWS w) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  w.dkey[i] = f2key(voxel_footprint(a, i));
}


// Histogram of the current digit for the selections of S, over keys[] or,
// when keys is null, the order keys of vals[].  dual: every
// element counts towards segments 0 and 1 (p5 and p95 of the same keys);
// otherwise the element's segment is its label.  With cnt (pass 0 of the
// per-bin selection) the initial states are the ranks ceil(q |V_b|) of the
// bin counts.  The block counts into ncopy padded lane-indexed copies of its
// nseg x 256 bins.
__global__ __launch_bounds__(256) void k_q_hist(const uint32_t* keys, const float* vals,
                                                const uint8_t* labels, int64_t n,
                                                SelSet S, int pass, int dual, int ncopy,
                                                const uint32_t* cnt, double q) {
  extern __shared__ uint32_t lh[];
  const int nseg = S.nseg;
  const int stride = nseg * 256 + (ncopy > 1 ? 1 : 0);
  for (int k = threadIdx.x; k < ncopy * stride; k += 256) lh[k] = 0u;
  uint32_t* mine = lh + (threadIdx.x & (ncopy - 1)) * stride;
  // segment states in LDS (a binned element looks its segment up by label)
  __shared__ uint32_t s_pre[kMaxBins], s_ok[kMaxBins];
  for (int sg = int(threadIdx.x >> 6); sg < nseg; sg += int(blockDim.x >> 6)) {
    SelState st;
    if (cnt) {
      const uint32_t c = cnt[sg];
      st.prefix = 0u;
      st.n = c;
      st.valid = c > 0 ? 1u : 0u;
      st.k = c > 0 ? rank_of(q, c) : 0u;
    } else {
      st = sel_state(S, sg, pass);
    }
    if ((threadIdx.x & 63) == 0) {
      s_pre[sg] = st.prefix;
      s_ok[sg] = st.valid;
      if (blockIdx.x == 0 && (pass > 0 || cnt)) sel_store(S, sg, pass, st);
    }
  }
  __syncthreads();
  const int sh = sel_shift(pass);
  const uint32_t hm = sel_himask(pass);
  // kUnroll independent coalesced loads per thread and step keep enough
  // requests in flight with one or two blocks per CU
  const int64_t step = int64_t(gridDim.x) * (256 * kUnroll);
  for (int64_t base = int64_t(blockIdx.x) * (256 * kUnroll) + threadIdx.x; base < n; base += step) {
    uint32_t kk[kUnroll];
    int ss[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + int64_t(u) * 256;
      // keys, or the order keys of float values (read directly each pass)
      kk[u] = i < n ? (keys ? keys[i] : f2key(vals[i])) : 0u;
      // a label past the last segment counts in the last (the histogram
      // copies hold nseg segments)
      ss[u] = (i < n && !dual && labels) ? min(int(labels[i]), nseg - 1) : 0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (base + int64_t(u) * 256 >= n) break;
      const uint32_t key = kk[u];
      const uint32_t d = (key >> sh) & 255u;
      if (dual) {
        if (s_ok[0] && (key & hm) == s_pre[0]) atomicAdd(&mine[d], 1u);
        if (s_ok[1] && (key & hm) == s_pre[1]) atomicAdd(&mine[256 + d], 1u);
      } else {
        const int sg = ss[u];
        if (s_ok[sg] && (key & hm) == s_pre[sg]) atomicAdd(&mine[sg * 256 + d], 1u);
      }
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nseg * 256; k += 256) {
    uint32_t c = 0;
    for (int i = 0; i < ncopy; ++i) c += lh[i * stride + k];
    if (c) atomicAdd(&sel_hist(S, pass, 0)[k], c);
  }
}

// bins from delta and (p5, p95), with the per-bin counts
__global__ __launch_bounds__(256) void k_q_bins(int64_t n, int B, QuantWS w, uint8_t* out_bins) {
  extern __shared__ uint32_t lc[];
  __shared__ uint32_t s_key[2];
  for (int k = threadIdx.x; k < B; k += 256) lc[k] = 0u;
  if (threadIdx.x < 128) {   // p5 and p95: the last pass's digits
    const int sg = int(threadIdx.x >> 6);
    const SelState st = sel_state(w.pct, sg, 4);
    if ((threadIdx.x & 63) == 0) s_key[sg] = st.prefix;
  }
  __syncthreads();
  const float p5 = key2f(s_key[0]), p95 = key2f(s_key[1]);
  const bool spread = isfinite(p95) && p95 > p5;
  const float den = p95 - p5;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float d = key2f(w.dkey[i]);
    int b;
    if (!isfinite(d)) {
      b = B - 1;
    } else if (!spread) {
      b = 0;
    } else {
      float zt = (d - p5) / den;
      zt = fminf(fmaxf(zt, 0.0f), 1.0f);
      b = int(floorf(float(B) * zt));
      if (b > B - 1) b = B - 1;
    }
    w.bins[i] = uint8_t(b);
    if (out_bins) out_bins[i] = uint8_t(b);
    atomicAdd(&lc[b], 1u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < B; k += 256)
    if (lc[k]) atomicAdd(&w.cnt[k], lc[k]);
}

// tau_b from the last pass's digits (-inf for an empty bin), then the prune
// mask over a grid-stride loop
__global__ __launch_bounds__(256) void k_q_prune(int64_t n, int B, QuantWS w, const float* wmax,
                                                 float* tau, uint8_t* prune) {
  __shared__ float s_tau[kMaxBins];
  for (int sg = int(threadIdx.x >> 6); sg < B; sg += int(blockDim.x >> 6)) {
    const SelState st = sel_state(w.bin, sg, 4);
    if ((threadIdx.x & 63) == 0) s_tau[sg] = st.valid ? key2f(st.prefix) : -INFINITY;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < B) tau[threadIdx.x] = s_tau[threadIdx.x];
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    prune[i] = wmax[i] <= s_tau[min(int(w.bins[i]), B - 1)] ? 1u : 0u;
}

// histogram copies: as many as fit in 64 KB of LDS, at most 16
constexpr int kCopiesDual = 16;
static size_t hist_lds(int nseg, int ncopy) {
  return size_t(ncopy) * (size_t(nseg) * 256 + (ncopy > 1 ? 1 : 0)) * 4;
}
static int binned_copies(int B) {
  int c = 16;
  while (c > 1 && hist_lds(B, c) > 65536) c >>= 1;
  return c;
}

// One block per 1024 elements, at most `cap` blocks (per-block histograms
// meet in few global atomics).  The cutoff's 16-segment passes take 512:
// 52 instead of 64 us per call over 1M voxels, where the two-segment
// percentile passes are fastest with 256.
constexpr int64_t kCutoffBlocks = 512;
static uint32_t grid_for(int64_t n, int64_t cap = 256) {
  int64_t b = (n + 1023) / 1024;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return uint32_t(b);
}

hipError_t run_depth_bins(const RasterArgs& a, int B, void* ws, uint8_t* out_bins, hipStream_t s) {
  QuantWS w = quant_bind(ws, a.n, B);
  hipLaunchKernelGGL(k_q_setup, dim3(2), dim3(256), 0, s, w, B, uint32_t(a.n), 0);
  if (a.n > 0) {
    hipLaunchKernelGGL(k_q_delta, dim3(uint32_t((a.n + 255) / 256)), dim3(256), 0, s, a, w);
    const uint32_t g = grid_for(a.n);
    // p5 and p95 of delta: segments 0 and 1 over every voxel, in the same passes
    for (int pass = 0; pass < 4; ++pass)
      hipLaunchKernelGGL(k_q_hist, dim3(g), dim3(256), hist_lds(2, kCopiesDual), s,
                         (const uint32_t*)w.dkey, (const float*)nullptr, (const uint8_t*)nullptr,
                         a.n, w.pct, pass, 1, kCopiesDual, (const uint32_t*)nullptr, 0.5);
    hipLaunchKernelGGL(k_q_bins, dim3(g), dim3(256), B * 4, s, a.n, B, w, out_bins);
  }
  return hipGetLastError();
}

hipError_t run_depth_cutoff(const RasterArgs& a, int B, double q, void* ws, float* tau,
                            uint8_t* prune, hipStream_t s) {
  QuantWS w = quant_bind(ws, a.n, B);
  hipLaunchKernelGGL(k_q_setup, dim3(B), dim3(256), 0, s, w, B, uint32_t(a.n), 1);
  if (a.n > 0) {
    const uint32_t g = grid_for(a.n, kCutoffBlocks);
    const int cb = binned_copies(B);
    for (int pass = 0; pass < 4; ++pass)
      hipLaunchKernelGGL(k_q_hist, dim3(g), dim3(256), hist_lds(B, cb), s, (const uint32_t*)nullptr,
                         (const float*)a.wmax, (const uint8_t*)w.bins, a.n, w.bin, pass, 0, cb,
                         pass == 0 ? (const uint32_t*)w.cnt : (const uint32_t*)nullptr, q);
  }
  hipLaunchKernelGGL(k_q_prune, dim3(grid_for(a.n, kCutoffBlocks)), dim3(256), 0, s, a.n, B, w,
                     a.wmax, tau, prune);
  return hipGetLastError();
}

// p5 and p95 of the footprint alone (the running-percentile input of the
// subdivision priority, eq. 14): 0 when there are no voxels
__global__ void k_q_range(QuantWS w, float* range) {
  if (threadIdx.x < 128) {
    const int sg = int(threadIdx.x >> 6);
    const SelState st = sel_state(w.pct, sg, 4);
    if ((threadIdx.x & 63) == 0) range[sg] = st.valid ? key2f(st.prefix) : 0.0f;
  }
}

uint64_t range_ws_bytes(int64_t n) { return quant_ws_bytes(n, 1); }

hipError_t run_footprint_range(const RasterArgs& a, void* ws, float* range, hipStream_t s) {
  QuantWS w = quant_bind(ws, a.n, 1);
  hipLaunchKernelGGL(k_q_setup, dim3(2), dim3(256), 0, s, w, 1, uint32_t(a.n), 0);
  if (a.n > 0) {
    hipLaunchKernelGGL(k_q_delta, dim3(uint32_t((a.n + 255) / 256)), dim3(256), 0, s, a, w);
    const uint32_t g = grid_for(a.n);
    for (int pass = 0; pass < 4; ++pass)
      hipLaunchKernelGGL(k_q_hist, dim3(g), dim3(256), hist_lds(2, kCopiesDual), s,
                         (const uint32_t*)w.dkey, (const float*)nullptr, (const uint8_t*)nullptr,
                         a.n, w.pct, pass, 1, kCopiesDual, (const uint32_t*)nullptr, 0.5);
  }
  hipLaunchKernelGGL(k_q_range, dim3(1), dim3(128), 0, s, w, range);
  return hipGetLastError();
}

}  // namespace lv

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
// passes); nothing returns to the host.
#include "lv_common.h"
#include "lv_select.h"

namespace lv {

struct QuantWS {
  uint32_t* dkey;     // [n] keys of delta
  uint32_t* wkey;     // [n] keys of w_max
  uint8_t* bins;      // [n]
  uint32_t* hist;     // [2 + B][256]
  SelState* st;       // [2 + B]: p5, p95, bins
  uint32_t* cnt;      // [B]
};

uint64_t quant_ws_bytes(int64_t n, int B) {
  return align256(4 * size_t(n)) * 2 + align256(size_t(n)) + align256(size_t(2 + B) * 1024) +
         align256(size_t(2 + B) * sizeof(SelState)) + align256(4 * size_t(B));
}

static QuantWS quant_bind(void* base, int64_t n, int B) {
  char* b = static_cast<char*>(base);
  QuantWS w;
  w.dkey = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(n));
  w.wkey = reinterpret_cast<uint32_t*>(b); b += align256(4 * size_t(n));
  w.bins = reinterpret_cast<uint8_t*>(b); b += align256(size_t(n));
  w.hist = reinterpret_cast<uint32_t*>(b); b += align256(size_t(2 + B) * 1024);
  w.st = reinterpret_cast<SelState*>(b); b += align256(size_t(2 + B) * sizeof(SelState));
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

__global__ void k_q_setup(QuantWS w, int B, uint32_t n) {
  const int s = blockIdx.x;   // segment
  w.hist[size_t(s) * 256 + threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    w.st[s].prefix = 0u;
    w.st[s].n = s < 2 ? n : 0u;
    w.st[s].valid = (s < 2 && n > 0) ? 1u : 0u;
    w.st[s].k = s == 0 ? rank_of(0.05, n) : (s == 1 ? rank_of(0.95, n) : 0u);
    if (s >= 2) w.cnt[s - 2] = 0u;
  }
}

__global__ __launch_bounds__(256) void k_q_delta(RasterArgs a, QuantWS w) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  const int l = a.level[i];
  const float e = ldexpf(a.root_size, -l);
  const float h = 0.5f * e;
  const float x0 = (a.root_min[0] + float(a.ijk[i]) * e) + h;
  const float x1 = (a.root_min[1] + float(a.ijk[n + i]) * e) + h;
  const float x2 = (a.root_min[2] + float(a.ijk[2 * n + i]) * e) + h;
  float delta = INFINITY;
  for (int v = 0; v < a.V; ++v) {
    const lv_camera& c = a.cams[v];
    const float q0 = x0 - c.o[0], q1 = x1 - c.o[1], q2 = x2 - c.o[2];
    float z = c.R[6] * q0 + c.R[7] * q1;
    z = z + c.R[8] * q2;
    if (z > 0.0f) delta = fminf(delta, z / c.fx);
  }
  w.dkey[i] = f2key(delta);
  w.wkey[i] = f2key(a.wmax[i]);
}

// Histogram of the current digit.  dual: every element counts towards
// segments seg0 and seg0 + 1 (p5 and p95 of the same keys); otherwise the
// element's segment is seg0 + label (label 0 when labels is null).  The
// block counts into ncopy padded lane-indexed copies of its nseg x 256 bins.
__global__ __launch_bounds__(256) void k_q_hist(const uint32_t* keys, const uint8_t* labels, int64_t n,
                                                QuantWS w, int seg0, int nseg, int pass, int dual,
                                                int ncopy) {
  extern __shared__ uint32_t lh[];
  const int stride = nseg * 256 + (ncopy > 1 ? 1 : 0);
  for (int k = threadIdx.x; k < ncopy * stride; k += 256) lh[k] = 0u;
  __syncthreads();
  uint32_t* mine = lh + (threadIdx.x & (ncopy - 1)) * stride;
  // segment states in LDS (a binned element looks its segment up by label)
  __shared__ uint32_t s_pre[2 + kMaxBins], s_ok[2 + kMaxBins];
  for (int k = threadIdx.x; k < nseg; k += 256) {
    s_pre[k] = w.st[seg0 + k].prefix;
    s_ok[k] = w.st[seg0 + k].valid;
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
      kk[u] = i < n ? keys[i] : 0u;
      ss[u] = (i < n && !dual && labels) ? int(labels[i]) : 0;
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
    if (c) atomicAdd(&w.hist[size_t(seg0) * 256 + k], c);
  }
}

// bins from delta and (p5, p95), with the per-bin counts
__global__ __launch_bounds__(256) void k_q_bins(int64_t n, int B, QuantWS w, uint8_t* out_bins) {
  extern __shared__ uint32_t lc[];
  for (int k = threadIdx.x; k < B; k += 256) lc[k] = 0u;
  __syncthreads();
  const float p5 = key2f(w.st[0].prefix), p95 = key2f(w.st[1].prefix);
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

// per-bin selection state from the bin counts
__global__ void k_q_ranks(int B, double q, QuantWS w) {
  const int b = threadIdx.x;
  if (b >= B) return;
  const uint32_t c = w.cnt[b];
  SelState& st = w.st[2 + b];
  st.prefix = 0u;
  st.n = c;
  st.valid = c > 0 ? 1u : 0u;
  st.k = c > 0 ? rank_of(q, c) : 0u;
}

__global__ __launch_bounds__(256) void k_q_prune(int64_t n, int B, QuantWS w, const float* wmax,
                                                 float* tau, uint8_t* prune) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x < B) {
    const SelState st = w.st[2 + threadIdx.x];
    tau[threadIdx.x] = st.valid ? key2f(st.prefix) : -INFINITY;
  }
  if (i >= n) return;
  const SelState st = w.st[2 + w.bins[i]];
  const float t = st.valid ? key2f(st.prefix) : -INFINITY;
  prune[i] = wmax[i] <= t ? 1u : 0u;
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

static uint32_t grid_for(int64_t n) {
  int64_t b = (n + 1023) / 1024;
  if (b < 1) b = 1;
  if (b > 256) b = 256;   // per-block histograms meet in few global atomics
  return uint32_t(b);
}

hipError_t run_depth_quantile(const RasterArgs& a, int B, double q, void* ws, float* tau,
                              uint8_t* prune, uint8_t* out_bins, hipStream_t s) {
  QuantWS w = quant_bind(ws, a.n, B);
  const uint32_t n32 = uint32_t(a.n);
  hipLaunchKernelGGL(k_q_setup, dim3(2 + B), dim3(256), 0, s, w, B, n32);
  if (a.n > 0) {
    hipLaunchKernelGGL(k_q_delta, dim3(uint32_t((a.n + 255) / 256)), dim3(256), 0, s, a, w);
    const uint32_t g = grid_for(a.n);
    // p5 and p95 of delta: segments 0 and 1 over every voxel, in the same passes
    for (int pass = 0; pass < 4; ++pass) {
      hipLaunchKernelGGL(k_q_hist, dim3(g), dim3(256), hist_lds(2, kCopiesDual), s,
                         (const uint32_t*)w.dkey, (const uint8_t*)nullptr, a.n, w, 0, 2, pass, 1,
                         kCopiesDual);
      const hipError_t e = launch_sel_step(w.st, w.hist, 2, pass, s);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_q_bins, dim3(g), dim3(256), B * 4, s, a.n, B, w, out_bins);
    hipLaunchKernelGGL(k_q_ranks, dim3(1), dim3(64), 0, s, B, q, w);
    const int cb = binned_copies(B);
    for (int pass = 0; pass < 4; ++pass) {
      hipLaunchKernelGGL(k_q_hist, dim3(g), dim3(256), hist_lds(B, cb), s, (const uint32_t*)w.wkey,
                         (const uint8_t*)w.bins, a.n, w, 2, B, pass, 0, cb);
      const hipError_t e = launch_sel_step(w.st + 2, w.hist + 2 * 256, B, pass, s);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_q_prune, dim3(uint32_t((a.n + 255) / 256) > 0 ? uint32_t((a.n + 255) / 256) : 1u),
                     dim3(256), 0, s, a.n, B, w, a.wmax, tau, prune);
  return hipGetLastError();
}

}  // namespace lv

// Low-frequency-aware photometric term (Sec. IV-B, eq. 7-10).
//   lv_lf_weight: Sobel magnitude of each view's target (grey = channel mean,
//     replicated borders) -> nearest-rank 99th percentile per view (radix
//     select) -> w = (eps + 1 - min(1, g/g99))^gamma (eq. 7) or
//     (1 + g/g99)^-gamma -> w / mean_view(w) (eq. 8).
//   lv_l1_grad: weighted L1 value per view and its image gradient (eq. 10).
// Every kernel runs on a (blocks, views) grid; a block finds its view's pixel
// offset from the device camera array, so no host tables are needed and the
// calls can be captured in a graph.
#include <algorithm>

#include "lv_common.h"
#include "lv_select.h"

namespace lv {

constexpr int kUnroll = 8;
// per-view weight sums are spread over kSumSlots slots, one 128-byte line
// each (device atomics on one address serialise)
constexpr int kSumSlots = 32;
constexpr int kSumStride = 16;   // doubles

struct LossWS {
  SelSet sel;        // one selection per view: hist [4][V][256], st [2][V]
  double* sums;      // [V][kSumSlots][kSumStride]
};

uint64_t loss_ws_bytes(int V) {
  return align256(size_t(4) * V * 256 * 4) + align256(size_t(2) * V * sizeof(SelState)) +
         align256(size_t(V) * kSumSlots * kSumStride * 8);
}

static LossWS loss_bind(void* base, int V) {
  char* b = static_cast<char*>(base);
  LossWS w;
  w.sel.nseg = V;
  w.sel.hist = reinterpret_cast<uint32_t*>(b);
  b += align256(size_t(4) * V * 256 * 4);
  w.sel.st = reinterpret_cast<SelState*>(b);
  b += align256(size_t(2) * V * sizeof(SelState));
  w.sums = reinterpret_cast<double*>(b);
  return w;
}

__device__ __forceinline__ uint64_t view_offset(const lv_camera* cams, int v) {
  uint64_t off = 0;
  for (int u = 0; u < v; ++u) off += uint64_t(cams[u].width) * uint64_t(cams[u].height);
  return off;
}

__global__ void k_loss_setup(const lv_camera* cams, int V, LossWS w, double q) {
  const int v = blockIdx.x;
  const uint64_t P = uint64_t(cams[v].width) * uint64_t(cams[v].height);
  for (int pass = 0; pass < 4; ++pass) sel_hist(w.sel, pass, v)[threadIdx.x] = 0u;
  if (threadIdx.x < kSumSlots) w.sums[(size_t(v) * kSumSlots + threadIdx.x) * kSumStride] = 0.0;
  if (threadIdx.x == 0) {
    double r = ceil(q * double(P));
    if (r < 1.0) r = 1.0;
    if (r > double(P)) r = double(P);
    SelState st;
    st.prefix = 0u;
    st.k = P > 0 ? uint32_t(r) - 1u : 0u;
    st.n = uint32_t(P);
    st.valid = P > 0 ? 1u : 0u;
    w.sel.st[v] = st;
  }
}

__device__ __forceinline__ float grey_at(const float* img, uint64_t npv, int W, int H, int x, int y) {
  x = x < 0 ? 0 : (x >= W ? W - 1 : x);
  y = y < 0 ? 0 : (y >= H ? H - 1 : y);
  const uint64_t p = uint64_t(y) * uint64_t(W) + uint64_t(x);
  return (img[p] + img[npv + p] + img[2 * npv + p]) * (1.0f / 3.0f);
}

// Each thread computes a column of kSobelRows pixels: it loads the grey
// values of the 3 columns around its pixel over kSobelRows + 2 rows (borders
// replicated) at once and slides the 3 x 3 window down; a block covers 256
// consecutive columns of one row band.
constexpr int kSobelRows = 8;

__global__ __launch_bounds__(256) void k_sobel(const lv_camera* cams, const float* target, float* out) {
  const int v = blockIdx.y;
  const int W = cams[v].width, H = cams[v].height;
  const uint32_t nxb = uint32_t(W + 255) / 256u;
  if (blockIdx.x >= nxb * uint32_t((H + kSobelRows - 1) / kSobelRows)) return;
  const int x = int(blockIdx.x % nxb) * 256 + int(threadIdx.x);
  const int y0 = int(blockIdx.x / nxb) * kSobelRows;
  if (x >= W) return;
  const uint64_t npv = uint64_t(W) * uint64_t(H);
  const uint64_t off = view_offset(cams, v);
  const float* img = target + 3 * off;
  float g[kSobelRows + 2][3];
#pragma unroll
  for (int r = 0; r < kSobelRows + 2; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) g[r][c] = grey_at(img, npv, W, H, x + c - 1, y0 + r - 1);
#pragma unroll
  for (int k = 0; k < kSobelRows; ++k) {
    const int y = y0 + k;
    if (y >= H) break;
    const float a00 = g[k][0], a10 = g[k][1], a20 = g[k][2];
    const float a01 = g[k + 1][0], a21 = g[k + 1][2];
    const float a02 = g[k + 2][0], a12 = g[k + 2][1], a22 = g[k + 2][2];
    const float gx = (a20 + 2.0f * a21 + a22) - (a00 + 2.0f * a01 + a02);
    const float gy = (a02 + 2.0f * a12 + a22) - (a00 + 2.0f * a10 + a20);
    out[off + uint64_t(y) * uint64_t(W) + uint64_t(x)] = sqrtf(gx * gx + gy * gy);
  }
}

// per-view histogram of the current digit of keys matching the prefix; the
// block counts into kHistCopies padded copies chosen by lane (most keys of a
// view share the leading digits, and LDS atomics on one address run lane by
// lane)
__global__ __launch_bounds__(256) void k_hist_views(const lv_camera* cams, const float* vals,
                                                    LossWS w, int pass) {
  __shared__ uint32_t lh[kHistCopies * kHistStride];
  __shared__ SelState s_st;
  const int v = blockIdx.y;
  for (int k = threadIdx.x; k < kHistCopies * kHistStride; k += 256) lh[k] = 0u;
  if (threadIdx.x < 64) {
    const SelState t = sel_state(w.sel, v, pass);
    if (threadIdx.x == 0) {
      s_st = t;
      if (blockIdx.x == 0 && pass > 0) sel_store(w.sel, v, pass, t);
    }
  }
  __syncthreads();
  uint32_t* mine = lh + (threadIdx.x & (kHistCopies - 1)) * kHistStride;
  const SelState st = s_st;
  const uint64_t npv = uint64_t(cams[v].width) * uint64_t(cams[v].height);
  const uint64_t off = view_offset(cams, v);
  const int sh = sel_shift(pass);
  const uint32_t hm = sel_himask(pass);
  // kUnroll independent coalesced loads per thread and step keep enough
  // requests in flight with few blocks (a view has fewer than 2^32 pixels)
  const float* src = vals + off;
  const uint32_t np32 = uint32_t(npv), step = gridDim.x * (256u * kUnroll);
  for (uint32_t base = blockIdx.x * (256u * kUnroll) + threadIdx.x; base < np32; base += step) {
    float vv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint32_t i = base + uint32_t(u) * 256u;
      vv[u] = i < np32 ? src[i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (base + uint32_t(u) * 256u >= np32) break;
      const uint32_t key = f2key(vv[u]);
      if ((key & hm) == st.prefix) atomicAdd(&mine[(key >> sh) & 255u], 1u);
    }
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < kHistCopies; ++i) c += lh[i * kHistStride + threadIdx.x];
  if (c) atomicAdd(&sel_hist(w.sel, pass, v)[threadIdx.x], c);
}

// b^gamma for b > 0 through the hardware log2 / exp2 (relative error a few
// 1e-7 for the bases and exponents used here)
__device__ __forceinline__ float pow_pos(float b, float gamma) {
  return __builtin_amdgcn_exp2f(gamma * __builtin_amdgcn_logf(b));
}

__global__ __launch_bounds__(256) void k_lf_weight(const lv_camera* cams, float* wbuf, LossWS w,
                                                   float gamma, int form, float eps) {
  __shared__ double s_part[4];
  __shared__ uint32_t s_key;
  const int v = blockIdx.y;
  const uint32_t np32 = uint32_t(cams[v].width) * uint32_t(cams[v].height);
  float* wv = wbuf + view_offset(cams, v);
  if (threadIdx.x < 64) {   // the 99th percentile: the last pass's digit
    const SelState t = sel_state(w.sel, v, 4);
    if (threadIdx.x == 0) s_key = t.prefix;
  }
  __syncthreads();
  const float g99 = key2f(s_key);
  double part = 0.0;
  constexpr int U = 4;
  const uint32_t step = gridDim.x * (256u * U);
  for (uint32_t base = blockIdx.x * (256u * U) + threadIdx.x; base < np32; base += step) {
    float g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = base + uint32_t(u) * 256u;
      g[u] = i < np32 ? wv[i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = base + uint32_t(u) * 256u;
      if (i >= np32) break;
      const float ratio = g99 > 0.0f ? g[u] / g99 : 0.0f;
      const float wt = form == 0 ? pow_pos(eps + 1.0f - fminf(1.0f, ratio), gamma)
                                 : pow_pos(1.0f + ratio, -gamma);
      wv[i] = wt;
      part += double(wt);
    }
  }
  const int lane = threadIdx.x & 63, wvi = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if (lane == 0) s_part[wvi] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double sum = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    unsafeAtomicAdd(&w.sums[(size_t(v) * kSumSlots + blockIdx.x % kSumSlots) * kSumStride], sum);
  }
}

__global__ __launch_bounds__(256) void k_lf_norm(const lv_camera* cams, float* wbuf, LossWS w) {
  const int v = blockIdx.y;
  const uint64_t npv = uint64_t(cams[v].width) * uint64_t(cams[v].height);
  const uint64_t off = view_offset(cams, v);
  double sum = 0.0;
  for (int i = 0; i < kSumSlots; ++i) sum += w.sums[(size_t(v) * kSumSlots + i) * kSumStride];
  const float scale = float(double(npv) / sum);
  for (uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x; p < npv; p += uint64_t(gridDim.x) * 256)
    wbuf[off + p] *= scale;
}

// blocks per view: enough waves in flight for the streaming kernels (each
// block still loops over several pixels, so per-block partial sums and
// histograms meet in few global atomics)
static uint32_t blocks_for(uint64_t max_pix) {
  uint64_t b = (max_pix + 2047) / 2048;
  if (b < 1) b = 1;
  if (b > 512) b = 512;
  return uint32_t(b);
}

// blocks per view of the histogram passes: every block adds its nonzero bins
// to the view's global bins, so these passes use fewer, longer-running blocks
constexpr uint32_t kHistBlocks = 128;
static uint32_t hist_blocks_for(uint64_t max_pix) {
  const uint32_t b = blocks_for(max_pix);
  return b < kHistBlocks ? b : kHistBlocks;
}

hipError_t run_lf_weight(const lv_camera* cams_dev, const lv_camera* cams_host, int V,
                         const float* target, float gamma, int form, float eps, float* weight,
                         void* ws, hipStream_t s) {
  uint64_t max_pix = 0, max_sobel_blocks = 0;
  for (int v = 0; v < V; ++v) {
    const uint64_t W = uint64_t(cams_host[v].width), H = uint64_t(cams_host[v].height);
    max_pix = std::max(max_pix, W * H);
    max_sobel_blocks = std::max(max_sobel_blocks, ((W + 255) / 256) * ((H + kSobelRows - 1) / kSobelRows));
  }
  LossWS w = loss_bind(ws, V);
  const dim3 grid(blocks_for(max_pix), V);
  hipLaunchKernelGGL(k_loss_setup, dim3(V), dim3(256), 0, s, cams_dev, V, w, 0.99);
  hipLaunchKernelGGL(k_sobel, dim3(uint32_t(max_sobel_blocks), V), dim3(256), 0, s, cams_dev, target,
                     weight);
  const dim3 hgrid(hist_blocks_for(max_pix), V);
  for (int pass = 0; pass < 4; ++pass)
    hipLaunchKernelGGL(k_hist_views, hgrid, dim3(256), 0, s, cams_dev, (const float*)weight, w, pass);
  hipLaunchKernelGGL(k_lf_weight, grid, dim3(256), 0, s, cams_dev, weight, w, gamma, form, eps);
  hipLaunchKernelGGL(k_lf_norm, grid, dim3(256), 0, s, cams_dev, weight, w);
  return hipGetLastError();
}

// ------------------------------------------------------------- weighted L1
__global__ void k_zero_f32(float* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

__global__ __launch_bounds__(256) void k_l1_grad(const lv_camera* cams, const float* rgb,
                                                 const float* target, const float* weight,
                                                 float* loss, float* d_rgb) {
  __shared__ float s_part[4];
  const int v = blockIdx.y;
  const uint32_t npv = uint32_t(cams[v].width) * uint32_t(cams[v].height);
  const uint64_t off = view_offset(cams, v);
  const float inv3p = float(1.0 / (3.0 * double(npv)));
  const float* C = rgb + 3 * off;
  const float* I = target + 3 * off;
  const float* Wt = weight + off;
  float* G = d_rgb + 3 * off;
  float part = 0.0f;
  constexpr int U = 2;
  const uint32_t step = gridDim.x * (256u * U);
  for (uint32_t base = blockIdx.x * (256u * U) + threadIdx.x; base < npv; base += step) {
    float c[U][3], t[U][3], wt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t p = base + uint32_t(u) * 256u;
      const bool in = p < npv;
      wt[u] = in ? Wt[p] : 0.0f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        c[u][ch] = in ? C[size_t(ch) * npv + p] : 0.0f;
        t[u][ch] = in ? I[size_t(ch) * npv + p] : 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t p = base + uint32_t(u) * 256u;
      if (p >= npv) break;
      float sabs = 0.0f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float r = c[u][ch] - t[u][ch];
        sabs += fabsf(r);
        const float sg = r > 0.0f ? 1.0f : (r < 0.0f ? -1.0f : 0.0f);
        G[size_t(ch) * npv + p] = wt[u] * sg * inv3p;
      }
      part = fmaf(wt[u], sabs, part);
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if (lane == 0) s_part[wv] = part;
  __syncthreads();
  if (threadIdx.x == 0)
    unsafeAtomicAdd(&loss[v], (s_part[0] + s_part[1] + s_part[2] + s_part[3]) * inv3p);
}

// blocks per view of the L1 pass: each block ends with one atomic add into
// the view's loss (the views' losses share a cache line)
static uint32_t l1_blocks_for(uint64_t max_pix) {
  const uint32_t b = blocks_for(max_pix);
  return b < 128u ? b : 128u;
}

hipError_t run_l1_grad(const lv_camera* cams_dev, int V, uint64_t max_pix, const float* rgb,
                       const float* target, const float* weight, float* loss, float* d_rgb,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f32, dim3((V + 255) / 256), dim3(256), 0, s, loss, V);
  hipLaunchKernelGGL(k_l1_grad, dim3(l1_blocks_for(max_pix), V), dim3(256), 0, s, cams_dev, rgb,
                     target, weight, loss, d_rgb);
  return hipGetLastError();
}

}  // namespace lv

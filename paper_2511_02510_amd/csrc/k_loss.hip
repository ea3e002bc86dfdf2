// Low-frequency-aware photometric term (Sec. IV-B, eq. 7-10).
//   lv_lf_weight: Sobel magnitude of each view's target (grey = channel mean,
//     replicated borders) -> nearest-rank 99th percentile per view (radix
//     select) -> w = (eps + 1 - min(1, g/g99))^gamma (eq. 7) or
//     (1 + g/g99)^-gamma -> w / mean_view(w) (eq. 8).
//   lv_l1_grad: weighted L1 value per view and its image gradient (eq. 10).
// Every kernel runs on a (blocks, views) grid; a block finds its view's pixel
// offset from the device camera array, so no host tables are needed and the
// calls can be captured in a graph.
#include "lv_common.h"
#include "lv_select.h"

namespace lv {

struct LossWS {
  uint32_t* hist;    // [V][256]
  SelState* st;      // [V]
  double* sums;      // [V]
  uint32_t* done;    // blocks finished in the current histogram pass
};

uint64_t loss_ws_bytes(int V) {
  return align256(size_t(V) * 256 * 4) + align256(size_t(V) * sizeof(SelState)) +
         align256(size_t(V) * 8) + 256;
}

static LossWS loss_bind(void* base, int V) {
  char* b = static_cast<char*>(base);
  LossWS w;
  w.hist = reinterpret_cast<uint32_t*>(b);
  b += align256(size_t(V) * 256 * 4);
  w.st = reinterpret_cast<SelState*>(b);
  b += align256(size_t(V) * sizeof(SelState));
  w.sums = reinterpret_cast<double*>(b);
  b += align256(size_t(V) * 8);
  w.done = reinterpret_cast<uint32_t*>(b);
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
  w.hist[size_t(v) * 256 + threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    double r = ceil(q * double(P));
    if (r < 1.0) r = 1.0;
    if (r > double(P)) r = double(P);
    w.st[v].prefix = 0u;
    w.st[v].k = P > 0 ? uint32_t(r) - 1u : 0u;
    w.st[v].n = uint32_t(P);
    w.st[v].valid = P > 0 ? 1u : 0u;
    w.sums[v] = 0.0;
    if (v == 0) *w.done = 0u;
  }
}

__device__ __forceinline__ float grey_at(const float* img, uint64_t npv, int W, int H, int x, int y) {
  x = x < 0 ? 0 : (x >= W ? W - 1 : x);
  y = y < 0 ? 0 : (y >= H ? H - 1 : y);
  const uint64_t p = uint64_t(y) * uint64_t(W) + uint64_t(x);
  return (img[p] + img[npv + p] + img[2 * npv + p]) * (1.0f / 3.0f);
}

__global__ __launch_bounds__(256) void k_sobel(const lv_camera* cams, const float* target, float* out) {
  const int v = blockIdx.y;
  const int W = cams[v].width, H = cams[v].height;
  const uint64_t npv = uint64_t(W) * uint64_t(H);
  const uint64_t off = view_offset(cams, v);
  const float* img = target + 3 * off;
  for (uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x; p < npv; p += uint64_t(gridDim.x) * 256) {
    const int x = int(p % uint64_t(W)), y = int(p / uint64_t(W));
    const float a00 = grey_at(img, npv, W, H, x - 1, y - 1), a10 = grey_at(img, npv, W, H, x, y - 1),
                a20 = grey_at(img, npv, W, H, x + 1, y - 1);
    const float a01 = grey_at(img, npv, W, H, x - 1, y), a21 = grey_at(img, npv, W, H, x + 1, y);
    const float a02 = grey_at(img, npv, W, H, x - 1, y + 1), a12 = grey_at(img, npv, W, H, x, y + 1),
                a22 = grey_at(img, npv, W, H, x + 1, y + 1);
    const float gx = (a20 + 2.0f * a21 + a22) - (a00 + 2.0f * a01 + a02);
    const float gy = (a02 + 2.0f * a12 + a22) - (a00 + 2.0f * a10 + a20);
    out[off + p] = sqrtf(gx * gx + gy * gy);
  }
}

// per-view histogram of the current digit of keys matching the prefix
__global__ __launch_bounds__(256) void k_hist_views(const lv_camera* cams, const float* vals,
                                                    LossWS w, int pass) {
  __shared__ uint32_t lh[256];
  const int v = blockIdx.y;
  lh[threadIdx.x] = 0u;
  __syncthreads();
  const SelState st = w.st[v];
  const uint64_t npv = uint64_t(cams[v].width) * uint64_t(cams[v].height);
  const uint64_t off = view_offset(cams, v);
  const int sh = sel_shift(pass);
  const uint32_t hm = sel_himask(pass);
  for (uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x; p < npv; p += uint64_t(gridDim.x) * 256) {
    const uint32_t key = f2key(vals[off + p]);
    if ((key & hm) == st.prefix) atomicAdd(&lh[(key >> sh) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t c = lh[threadIdx.x];
  if (c) atomicAdd(&w.hist[size_t(v) * 256 + threadIdx.x], c);
  sel_finish_pass(w.st, w.hist, gridDim.y, pass, w.done);
}

__global__ __launch_bounds__(256) void k_lf_weight(const lv_camera* cams, float* wbuf, LossWS w,
                                                   float gamma, int form, float eps) {
  __shared__ double s_part[4];
  const int v = blockIdx.y;
  const uint64_t npv = uint64_t(cams[v].width) * uint64_t(cams[v].height);
  const uint64_t off = view_offset(cams, v);
  const float g99 = key2f(w.st[v].prefix);
  double part = 0.0;
  for (uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x; p < npv; p += uint64_t(gridDim.x) * 256) {
    const float g = wbuf[off + p];
    const float ratio = g99 > 0.0f ? g / g99 : 0.0f;
    float wt;
    if (form == 0) wt = powf(eps + 1.0f - fminf(1.0f, ratio), gamma);
    else wt = powf(1.0f + ratio, -gamma);
    wbuf[off + p] = wt;
    part += double(wt);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if (lane == 0) s_part[wv] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double s = s_part[0] + s_part[1] + s_part[2] + s_part[3];
    unsafeAtomicAdd(&w.sums[v], s);
  }
}

__global__ __launch_bounds__(256) void k_lf_norm(const lv_camera* cams, float* wbuf, LossWS w) {
  const int v = blockIdx.y;
  const uint64_t npv = uint64_t(cams[v].width) * uint64_t(cams[v].height);
  const uint64_t off = view_offset(cams, v);
  const float scale = float(double(npv) / w.sums[v]);
  for (uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x; p < npv; p += uint64_t(gridDim.x) * 256)
    wbuf[off + p] *= scale;
}

static uint32_t blocks_for(uint64_t max_pix) {
  uint64_t b = (max_pix + 1023) / 1024;
  if (b < 1) b = 1;
  if (b > 96) b = 96;   // few long-running blocks: per-block partial sums meet in few atomics
  return uint32_t(b);
}

hipError_t run_lf_weight(const lv_camera* cams_dev, int V, uint64_t max_pix, const float* target,
                         float gamma, int form, float eps, float* weight, void* ws, hipStream_t s) {
  LossWS w = loss_bind(ws, V);
  const dim3 grid(blocks_for(max_pix), V);
  hipLaunchKernelGGL(k_loss_setup, dim3(V), dim3(256), 0, s, cams_dev, V, w, 0.99);
  hipLaunchKernelGGL(k_sobel, grid, dim3(256), 0, s, cams_dev, target, weight);
  for (int pass = 0; pass < 4; ++pass)
    hipLaunchKernelGGL(k_hist_views, grid, dim3(256), 0, s, cams_dev, (const float*)weight, w, pass);
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
  const uint64_t npv = uint64_t(cams[v].width) * uint64_t(cams[v].height);
  const uint64_t off = view_offset(cams, v);
  const float inv3p = float(1.0 / (3.0 * double(npv)));
  const float* C = rgb + 3 * off;
  const float* I = target + 3 * off;
  float* G = d_rgb + 3 * off;
  float part = 0.0f;
  for (uint64_t p = uint64_t(blockIdx.x) * 256 + threadIdx.x; p < npv; p += uint64_t(gridDim.x) * 256) {
    const float wt = weight[off + p];
    float s = 0.0f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float r = C[ch * npv + p] - I[ch * npv + p];
      s += fabsf(r);
      const float sg = r > 0.0f ? 1.0f : (r < 0.0f ? -1.0f : 0.0f);
      G[ch * npv + p] = wt * sg * inv3p;
    }
    part = fmaf(wt, s, part);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  if (lane == 0) s_part[wv] = part;
  __syncthreads();
  if (threadIdx.x == 0)
    unsafeAtomicAdd(&loss[v], (s_part[0] + s_part[1] + s_part[2] + s_part[3]) * inv3p);
}

hipError_t run_l1_grad(const lv_camera* cams_dev, int V, uint64_t max_pix, const float* rgb,
                       const float* target, const float* weight, float* loss, float* d_rgb,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f32, dim3((V + 255) / 256), dim3(256), 0, s, loss, V);
  hipLaunchKernelGGL(k_l1_grad, dim3(blocks_for(max_pix), V), dim3(256), 0, s, cams_dev, rgb,
                     target, weight, loss, d_rgb);
  return hipGetLastError();
}

}  // namespace lv

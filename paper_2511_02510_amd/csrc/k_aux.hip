// Image-space auxiliary terms of the training objective (eq. 6 and eq. 17
// name them; the paper defines none, readings below) and their gradients
// with respect to the render channels, per view:
//   transmittance concentration  L_Tc = 1/|P| sum_p A_p (1 - A_p)
//   distortion                   L_d  = 1/|P| sum_p dist_p
//   depth-normal consistency     L_n  = 1/|I| sum_{p in I} (A_p - N_p . m_p)
// with I the interior pixels (1 <= x <= W-2, 1 <= y <= H-2), N the rendered
// normal and m the unit normal of the surface the depth channel describes:
// X_p = o + D_p d_p (d_p the pixel's unit ray), e_x = X(x+1,y) - X(x-1,y),
// e_y = X(x,y+1) - X(x,y-1), m = (e_y x e_x) / |e_y x e_x| (0 if it vanishes),
// which faces the camera for a visible surface.  Each term is multiplied by
// its weight.  One thread per pixel; the depth gradient of a pixel gathers
// the contributions of the (up to four) interior stencils that read it.
#include "lv_common.h"

namespace lv {

// unit world ray through the centre of pixel (x, y): R^T of the camera-space
// direction, normalised
__device__ __forceinline__ void aux_ray(const lv_camera& c, int x, int y, float d[3]) {
  const float xc = ((float(x) + 0.5f) - c.cx) / c.fx;
  const float yc = ((float(y) + 0.5f) - c.cy) / c.fy;
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a] = fmaf(c.R[a], xc, fmaf(c.R[3 + a], yc, c.R[6 + a]));
  const float in = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  d[0] *= in; d[1] *= in; d[2] *= in;
}

__device__ __forceinline__ void cross3(const float a[3], const float b[3], float c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// The stencil of interior pixel (x, y): unit normal m and, for the weight
// `scale` (= -lam_n / |I|) on N . m, the gradients gex, gey of the loss with
// respect to the differences e_x, e_y.
struct Stencil {
  float m[3], gex[3], gey[3];
};

__device__ Stencil aux_stencil(const lv_camera& c, const float* D, const float* N, int W, int H,
                               uint64_t npv, int x, int y, float scale) {
  float dl[3], dr[3], du[3], dd[3];
  aux_ray(c, x - 1, y, dl);
  aux_ray(c, x + 1, y, dr);
  aux_ray(c, x, y - 1, du);
  aux_ray(c, x, y + 1, dd);
  const float Dl = D[size_t(y) * W + x - 1], Dr = D[size_t(y) * W + x + 1];
  const float Du = D[size_t(y - 1) * W + x], Dd = D[size_t(y + 1) * W + x];
  float ex[3], ey[3], cr[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {   // the camera centre cancels in the differences
    ex[a] = fmaf(Dr, dr[a], -Dl * dl[a]);
    ey[a] = fmaf(Dd, dd[a], -Du * du[a]);
  }
  cross3(ey, ex, cr);
  const float ln = sqrtf(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  Stencil s;
  const size_t p = size_t(y) * W + x;
  const float n[3] = {N[p], N[npv + p], N[2 * npv + p]};
  if (!(ln > 0.0f)) {
#pragma unroll
    for (int a = 0; a < 3; ++a) s.m[a] = s.gex[a] = s.gey[a] = 0.0f;
    return s;
  }
  const float il = 1.0f / ln;
  float gm[3], gc[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s.m[a] = cr[a] * il;
    gm[a] = scale * n[a];
  }
  const float gmm = gm[0] * s.m[0] + gm[1] * s.m[1] + gm[2] * s.m[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) gc[a] = (gm[a] - gmm * s.m[a]) * il;
  cross3(gc, ey, s.gex);   // d(e_y x e_x)/d e_x applied to gc
  cross3(ex, gc, s.gey);   // d(e_y x e_x)/d e_y applied to gc
  return s;
}

__global__ __launch_bounds__(256) void k_aux_loss(const lv_camera* cams, const float* depth,
                                                  const float* alpha, const float* normal,
                                                  const float* dist, float lam_tc, float lam_n,
                                                  float lam_d, float* loss, float* g_alpha,
                                                  float* g_depth, float* g_normal, float* g_dist) {
  __shared__ float s_part[3][4];
  const int v = blockIdx.y;
  const lv_camera& c = cams[v];
  const int W = c.width, H = c.height;
  const uint64_t npv = uint64_t(W) * uint64_t(H);
  uint64_t off = 0;
  for (int u = 0; u < v; ++u) off += uint64_t(cams[u].width) * uint64_t(cams[u].height);
  const float* D = depth + off;
  const float* A = alpha + off;
  const float* N = normal + 3 * off;
  const float* L = dist + off;
  const bool has_int = W >= 3 && H >= 3;
  const float ni = has_int ? float(W - 2) * float(H - 2) : 1.0f;
  const float inv_p = float(1.0 / double(npv));
  const float sc_n = -lam_n / ni;   // weight of N . m in the loss
  float p_tc = 0.0f, p_n = 0.0f, p_d = 0.0f;
  for (uint64_t p = uint64_t(blockIdx.x) * 256u + threadIdx.x; p < npv;
       p += uint64_t(gridDim.x) * 256u) {
    const int x = int(p % uint64_t(W)), y = int(p / uint64_t(W));
    const float a = A[p];
    p_tc = fmaf(a, 1.0f - a, p_tc);
    p_d += L[p];
    float ga = lam_tc * (1.0f - 2.0f * a) * inv_p;
    float gn[3] = {0.0f, 0.0f, 0.0f};
    const bool in = has_int && x >= 1 && x <= W - 2 && y >= 1 && y <= H - 2;
    if (in) {
      const Stencil s = aux_stencil(c, D, N, W, H, npv, x, y, sc_n);
      p_n += a - (N[p] * s.m[0] + N[npv + p] * s.m[1] + N[2 * npv + p] * s.m[2]);
      ga += lam_n / ni;
#pragma unroll
      for (int k = 0; k < 3; ++k) gn[k] = sc_n * s.m[k];
    }
    // this pixel's depth enters the stencils of its four neighbours
    float gX[3] = {0.0f, 0.0f, 0.0f};
    if (has_int) {
      if (x - 1 >= 1 && x - 1 <= W - 2 && y >= 1 && y <= H - 2) {   // it is X(x+1) of (x-1, y)
        const Stencil s = aux_stencil(c, D, N, W, H, npv, x - 1, y, sc_n);
        for (int k = 0; k < 3; ++k) gX[k] += s.gex[k];
      }
      if (x + 1 >= 1 && x + 1 <= W - 2 && y >= 1 && y <= H - 2) {   // X(x-1) of (x+1, y)
        const Stencil s = aux_stencil(c, D, N, W, H, npv, x + 1, y, sc_n);
        for (int k = 0; k < 3; ++k) gX[k] -= s.gex[k];
      }
      if (y - 1 >= 1 && y - 1 <= H - 2 && x >= 1 && x <= W - 2) {   // X(y+1) of (x, y-1)
        const Stencil s = aux_stencil(c, D, N, W, H, npv, x, y - 1, sc_n);
        for (int k = 0; k < 3; ++k) gX[k] += s.gey[k];
      }
      if (y + 1 >= 1 && y + 1 <= H - 2 && x >= 1 && x <= W - 2) {   // X(y-1) of (x, y+1)
        const Stencil s = aux_stencil(c, D, N, W, H, npv, x, y + 1, sc_n);
        for (int k = 0; k < 3; ++k) gX[k] -= s.gey[k];
      }
    }
    float dp[3];
    aux_ray(c, x, y, dp);
    g_alpha[off + p] = ga;
    g_depth[off + p] = gX[0] * dp[0] + gX[1] * dp[1] + gX[2] * dp[2];
    g_normal[3 * off + p] = gn[0];
    g_normal[3 * off + npv + p] = gn[1];
    g_normal[3 * off + 2 * npv + p] = gn[2];
    g_dist[off + p] = lam_d * inv_p;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    p_tc += __shfl_xor(p_tc, o, 64);
    p_n += __shfl_xor(p_n, o, 64);
    p_d += __shfl_xor(p_d, o, 64);
  }
  if (lane == 0) {
    s_part[0][wv] = p_tc;
    s_part[1][wv] = p_n;
    s_part[2][wv] = p_d;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    const float t = (s_part[k][0] + s_part[k][1]) + (s_part[k][2] + s_part[k][3]);
    const float f = k == 0 ? lam_tc * inv_p : (k == 1 ? (has_int ? lam_n / ni : 0.0f) : lam_d * inv_p);
    unsafeAtomicAdd(&loss[3 * v + k], t * f);
  }
}

__global__ void k_aux_zero(float* loss, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) loss[i] = 0.0f;
}

hipError_t run_aux_loss(const lv_camera* cams_dev, int V, uint64_t max_pix, const float* depth,
                        const float* alpha, const float* normal, const float* dist, float lam_tc,
                        float lam_n, float lam_d, float* loss, float* g_alpha, float* g_depth,
                        float* g_normal, float* g_dist, hipStream_t s) {
  hipLaunchKernelGGL(k_aux_zero, dim3((3 * V + 255) / 256), dim3(256), 0, s, loss, 3 * V);
  uint64_t b = (max_pix + 255) / 256;
  if (b > 256) b = 256;   // each block ends with one atomic per term
  if (b < 1) b = 1;
  hipLaunchKernelGGL(k_aux_loss, dim3(uint32_t(b), V), dim3(256), 0, s, cams_dev, depth, alpha,
                     normal, dist, lam_tc, lam_n, lam_d, loss, g_alpha, g_depth, g_normal, g_dist);
  return hipGetLastError();
}

}  // namespace lv

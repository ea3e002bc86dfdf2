// Image-space auxiliary terms of the training objective (eq. 6 and eq. 17
// name them; the paper defines none, readings below) and their gradients
// with respect to the render channels, per view:
//   transmittance concentration  L_Tc = 1/|P| sum_p A_p (1 - A_p)
//   distortion                   L_d  = 1/|P| sum_p dist_p
//   depth-normal consistency     L_n  = 1/|I| sum_{p in I} (A_p - N_p . m_p)
//   median depth-normal          L_nm = 1/|I| sum_{p in I} (A_p - N_p . m'_p)
// with I the interior pixels (1 <= x <= W-2, 1 <= y <= H-2), N the rendered
// normal and m the unit normal of the surface the depth channel describes:
// X_p = o + D_p d_p (d_p the pixel's unit ray), e_x = X(x+1,y) - X(x-1,y),
// e_y = X(x,y+1) - X(x,y-1), m = (e_y x e_x) / |e_y x e_x| (0 when the
// cross product vanishes; here, when its squared length is below the smallest
// normal float), which faces the camera for a visible surface; m' is the same
// stencil on the median-depth map, which passes no gradient.  Each term is
// multiplied by its weight.  The depth gradient of a pixel gathers the contributions of
// the (up to four) interior stencils that read it.
#include "lv_common.h"

namespace lv {

// unit world ray through the centre of pixel (x, y): R^T of the camera-space
// direction (with the reciprocal focal lengths ifx, ify), normalised with the
// hardware reciprocal square root
__device__ __forceinline__ void aux_ray(const lv_camera& c, float ifx, float ify, int x, int y,
                                        float d[3]) {
  const float xc = ((float(x) + 0.5f) - c.cx) * ifx;
  const float yc = ((float(y) + 0.5f) - c.cy) * ify;
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a] = fmaf(c.R[a], xc, fmaf(c.R[3 + a], yc, c.R[6 + a]));
  const float in = __builtin_amdgcn_rsqf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  d[0] *= in; d[1] *= in; d[2] *= in;
}

__device__ __forceinline__ void cross3(const float a[3], const float b[3], float c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Tiles of TX x TY pixels, taken in turn by persistent blocks from one
// index space over the tiles of every view.  A block stages, in LDS, the
// camera-relative points D d of the tile grown by two pixels on each side,
// then the stencil of every interior pixel of the tile grown by one (its
// normal m and the gradients of the loss with respect to e_x and e_y), so
// that each pixel's depth gradient gathers its four neighbours' stencils
// from LDS: about 1.7 rays and 1.3 stencils per pixel instead of 21 and 5.
// Every global value a tile reads is loaded at its start, in one round.  The
// kernel is bound by memory latency, not arithmetic: keeping each XCD on one
// contiguous run of tiles (halo rows stay in its L2) and loading the view
// sizes in parallel are what shortened it.
constexpr int kTX = 32, kTY = 8;
constexpr int kXW = kTX + 4, kXH = kTY + 4;   // points: tile +- 2
constexpr int kSW = kTX + 2, kSH = kTY + 2;   // stencils: tile +- 1
constexpr int kXN = kXW * kXH, kSN = kSW * kSH;
static_assert(kTX * kTY == 256 && kXN <= 512 && kSN <= 512, "two slots per thread");

struct AuxLds {
  float X[3][kXN];
  float X2[3][kXN];   // points of the median-depth map (median instance)
  float m[3][kSN];
  float gex[3][kSN];
  float gey[3][kSN];
  float part[4][4];
};

// prefix of the tile counts over the views: view v owns tiles
// [off[v], off[v + 1])
struct AuxTiles {
  uint32_t off[LV_MAX_VIEWS + 1];
};

struct AuxView {
  lv_camera c;
  int W, H, ntx;
  size_t npv, pix;   // pixels of the view, offset of its first pixel
  float inv_p, ni, wn, sc_n, wnm, ifx, ify;
  bool has_int;
};

__device__ AuxView aux_view(const lv_camera* cams, int v, float lam_n, float lam_nm) {
  AuxView u;
  u.c = cams[v];   // a private copy: the kernel's stores cannot alias it
  u.W = u.c.width;
  u.H = u.c.height;
  u.ntx = (u.W + kTX - 1) / kTX;
  u.npv = size_t(u.W) * size_t(u.H);
  // pixels of the views before v: the lanes load the view sizes in parallel
  // (a loop over the views would wait for one load after another)
  unsigned long long pix = 0;
  for (int k = threadIdx.x & 63; k < v; k += 64)
    pix += (unsigned long long)(cams[k].width) * (unsigned long long)(cams[k].height);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pix += __shfl_xor(pix, o, 64);
  u.pix = size_t(pix);
  u.has_int = u.W >= 3 && u.H >= 3;
  u.ni = u.has_int ? float(u.W - 2) * float(u.H - 2) : 1.0f;
  u.inv_p = float(1.0 / double(u.npv));
  u.wn = u.has_int ? lam_n / u.ni : 0.0f;   // weight of each interior pixel's term
  u.sc_n = -u.wn;                           // weight of N . m in the loss
  u.wnm = u.has_int ? lam_nm / u.ni : 0.0f;  // the median term's per-pixel weight
  u.ifx = 1.0f / u.c.fx;
  u.ify = 1.0f / u.c.fy;
  return u;
}

// block sum of the four partial terms of view v, weighted, into loss[4 v ..]
__device__ void aux_flush(AuxLds& L, float p[4], const AuxView& u, int v, float lam_tc,
                          float lam_d, float* loss) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) p[k] += __shfl_xor(p[k], o, 64);
    if (lane == 0) L.part[k][wv] = p[k];
    p[k] = 0.0f;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    const float t = (L.part[k][0] + L.part[k][1]) + (L.part[k][2] + L.part[k][3]);
    const float f = k == 0 ? lam_tc * u.inv_p
                           : (k == 1 ? u.wn : (k == 2 ? lam_d * u.inv_p : u.wnm));
    unsafeAtomicAdd(&loss[4 * v + k], t * f);
  }
  __syncthreads();
}

// MED: with the median depth-normal term (mdepth non-null)
template <bool MED>
__global__ __launch_bounds__(256) void k_aux_loss(const lv_camera* cams, AuxTiles tl, int V,
                                                  const float* depth, const float* alpha,
                                                  const float* normal, const float* dist,
                                                  const float* mdepth, float lam_tc, float lam_n,
                                                  float lam_d, float lam_nm, float* loss,
                                                  float* g_alpha, float* g_depth, float* g_normal,
                                                  float* g_dist) {
  __shared__ AuxLds L;
  const uint32_t total = tl.off[V];
  int v = -1;
  AuxView u;
  float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
  // XCD-aware: blocks are dealt to the 8 XCDs round-robin; the blocks of one
  // XCD sweep one contiguous eighth of the tiles, so the halo rows a tile
  // shares with its neighbours stay in that XCD's L2
  const uint32_t nseg = gridDim.x < 8u ? gridDim.x : 8u;
  const uint32_t seg = blockIdx.x % nseg, kb = blockIdx.x / nseg;
  const uint32_t gseg = (gridDim.x - seg + nseg - 1) / nseg;   // blocks of this segment
  const uint32_t t0 = uint32_t((uint64_t(total) * seg) / nseg);
  const uint32_t t1 = uint32_t((uint64_t(total) * (seg + 1)) / nseg);
  for (uint32_t t = t0 + kb; t < t1; t += gseg) {
    int nv = v < 0 ? 0 : v;   // the views are visited in increasing order
    while (tl.off[nv + 1] <= t) ++nv;
    if (nv != v) {
      if (v >= 0) aux_flush(L, part, u, v, lam_tc, lam_d, loss);
      v = nv;
      u = aux_view(cams, v, lam_n, lam_nm);
    }
    const uint32_t tt = t - tl.off[v];
    const int x0 = int(tt % uint32_t(u.ntx)) * kTX, y0 = int(tt / uint32_t(u.ntx)) * kTY;
    const int W = u.W, H = u.H;
    const size_t npv = u.npv;
    const float* D = depth + u.pix;
    const float* Dm = MED ? mdepth + u.pix : nullptr;
    const float* N = normal + 3 * u.pix;
    // ---- every load of the tile: depth at two point slots, the rendered
    // normal at two stencil slots and at this thread's pixel, alpha, dist
    float dep[2], mdp[2], ns[2][3];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int i = threadIdx.x + 256 * j;
      const int gx = x0 - 2 + i % kXW, gy = y0 - 2 + i / kXW;
      const bool pin = i < kXN && gx >= 0 && gx < W && gy >= 0 && gy < H;
      dep[j] = pin ? D[size_t(gy) * W + gx] : 0.0f;
      mdp[j] = (MED && pin) ? Dm[size_t(gy) * W + gx] : 0.0f;
      const int sx = x0 - 1 + i % kSW, sy = y0 - 1 + i / kSW;
      const bool in = i < kSN && sx >= 1 && sx <= W - 2 && sy >= 1 && sy <= H - 2;
#pragma unroll
      for (int a = 0; a < 3; ++a) ns[j][a] = in ? N[a * npv + size_t(sy) * W + sx] : 0.0f;
    }
    const int x = x0 + lx, y = y0 + ly;
    const bool mine = x < W && y < H;
    const size_t p = size_t(y) * W + x;
    float a = 0.0f, ld = 0.0f, n0 = 0.0f, n1 = 0.0f, n2 = 0.0f;
    if (mine) {
      a = alpha[u.pix + p];
      ld = dist[u.pix + p];
      n0 = N[p];
      n1 = N[npv + p];
      n2 = N[2 * npv + p];
    }
    // ---- points X = D d (the camera centre cancels in every difference)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int i = threadIdx.x + 256 * j;
      if (i < kXN) {
        const int gx = x0 - 2 + i % kXW, gy = y0 - 2 + i / kXW;
        float d[3] = {0.0f, 0.0f, 0.0f};
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) aux_ray(u.c, u.ifx, u.ify, gx, gy, d);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          L.X[k][i] = dep[j] * d[k];
          if (MED) L.X2[k][i] = mdp[j] * d[k];
        }
      }
    }
    __syncthreads();
    // ---- stencils of the interior pixels among tile +- 1 (zero elsewhere)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int i = threadIdx.x + 256 * j;
      if (i < kSN) {
        const int sx = i % kSW, sy = i / kSW;
        const int gx = x0 - 1 + sx, gy = y0 - 1 + sy;
        float m[3] = {0.0f, 0.0f, 0.0f}, gex[3] = {0.0f, 0.0f, 0.0f}, gey[3] = {0.0f, 0.0f, 0.0f};
        if (gx >= 1 && gx <= W - 2 && gy >= 1 && gy <= H - 2) {
          const int xc = (sy + 1) * kXW + sx + 1;   // this pixel in the point block
          float ex[3], ey[3], cr[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            ex[k] = L.X[k][xc + 1] - L.X[k][xc - 1];
            ey[k] = L.X[k][xc + kXW] - L.X[k][xc - kXW];
          }
          cross3(ey, ex, cr);
          const float l2 = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
          // below the smallest normal float the stencil counts as degenerate
          // (m = 0), which keeps the reciprocal square root finite
          if (l2 >= 1.17549435e-38f) {
            const float il = __builtin_amdgcn_rsqf(l2);
            float gm[3], gc[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              m[k] = cr[k] * il;
              gm[k] = u.sc_n * ns[j][k];
            }
            const float gmm = gm[0] * m[0] + gm[1] * m[1] + gm[2] * m[2];
#pragma unroll
            for (int k = 0; k < 3; ++k) gc[k] = (gm[k] - gmm * m[k]) * il;
            cross3(gc, ey, gex);   // d(e_y x e_x)/d e_x applied to gc
            cross3(ex, gc, gey);   // d(e_y x e_x)/d e_y applied to gc
          }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          L.m[k][i] = m[k];
          L.gex[k][i] = gex[k];
          L.gey[k][i] = gey[k];
        }
      }
    }
    __syncthreads();
    // ---- this thread's pixel
    if (mine) {
      part[0] = fmaf(a, 1.0f - a, part[0]);
      part[2] += ld;
      float ga = lam_tc * (1.0f - 2.0f * a) * u.inv_p;
      const int sc = (ly + 1) * kSW + lx + 1;   // this pixel in the stencil block
      float gn[3] = {0.0f, 0.0f, 0.0f};
      if (x >= 1 && x <= W - 2 && y >= 1 && y <= H - 2) {
        part[1] += a - (n0 * L.m[0][sc] + n1 * L.m[1][sc] + n2 * L.m[2][sc]);
        ga += u.wn;
#pragma unroll
        for (int k = 0; k < 3; ++k) gn[k] = u.sc_n * L.m[k][sc];
        if (MED) {   // the median map's normal at this pixel: a constant target
          const int xc = (ly + 2) * kXW + lx + 2;   // this pixel in the point block
          float ex[3], ey[3], cr[3], mm[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            ex[k] = L.X2[k][xc + 1] - L.X2[k][xc - 1];
            ey[k] = L.X2[k][xc + kXW] - L.X2[k][xc - kXW];
          }
          cross3(ey, ex, cr);
          const float l2 = cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2];
          if (l2 >= 1.17549435e-38f) {
            const float il = __builtin_amdgcn_rsqf(l2);
#pragma unroll
            for (int k = 0; k < 3; ++k) mm[k] = cr[k] * il;
          }
          part[3] += a - (n0 * mm[0] + n1 * mm[1] + n2 * mm[2]);
          ga += u.wnm;
#pragma unroll
          for (int k = 0; k < 3; ++k) gn[k] -= u.wnm * mm[k];
        }
      }
      // this pixel is X(x+1) of (x-1, y), X(x-1) of (x+1, y), X(y+1) of
      // (x, y-1) and X(y-1) of (x, y+1); stencils outside the interior are 0
      float gX[3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        gX[k] = (L.gex[k][sc - 1] - L.gex[k][sc + 1]) + (L.gey[k][sc - kSW] - L.gey[k][sc + kSW]);
      float dp[3];
      aux_ray(u.c, u.ifx, u.ify, x, y, dp);
      g_alpha[u.pix + p] = ga;
      g_depth[u.pix + p] = gX[0] * dp[0] + gX[1] * dp[1] + gX[2] * dp[2];
      float* gnv = g_normal + 3 * u.pix + p;
      gnv[0] = gn[0];
      gnv[npv] = gn[1];
      gnv[2 * npv] = gn[2];
      g_dist[u.pix + p] = lam_d * u.inv_p;
    }
    __syncthreads();   // the next tile overwrites the blocks
  }
  if (v >= 0) aux_flush(L, part, u, v, lam_tc, lam_d, loss);
}

__global__ void k_aux_zero(float* loss, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) loss[i] = 0.0f;
}

hipError_t run_aux_loss(const lv_camera* cams_host, const lv_camera* cams_dev, int V,
                        const float* depth, const float* alpha, const float* normal,
                        const float* dist, const float* mdepth, float lam_tc, float lam_n,
                        float lam_d, float lam_nm, float* loss, float* g_alpha, float* g_depth,
                        float* g_normal, float* g_dist, hipStream_t s) {
  if (V < 1 || V > LV_MAX_VIEWS) return hipErrorInvalidValue;
  AuxTiles tl;
  tl.off[0] = 0;
  uint64_t total = 0;
  for (int v = 0; v < V; ++v) {
    total += ((uint64_t(cams_host[v].width) + kTX - 1) / kTX) *
             ((uint64_t(cams_host[v].height) + kTY - 1) / kTY);
    if (total > 0xffffffffull) return hipErrorInvalidValue;
    tl.off[v + 1] = uint32_t(total);
  }
  hipLaunchKernelGGL(k_aux_zero, dim3((4 * V + 255) / 256), dim3(256), 0, s, loss, 4 * V);
  auto kern = mdepth ? k_aux_loss<true> : k_aux_loss<false>;
  // persistent: as many blocks as fit on the device at once
  int dev = 0, cus = 256, per = 1;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, 256, 0) != hipSuccess ||
      per < 1)
    per = 1;
  uint64_t b = uint64_t(cus) * uint64_t(per);
  if (b > total) b = total;
  if (b < 1) b = 1;
  hipLaunchKernelGGL(kern, dim3(uint32_t(b)), dim3(256), 0, s, cams_dev, tl, V, depth, alpha,
                     normal, dist, mdepth, lam_tc, lam_n, lam_d, lam_nm, loss, g_alpha, g_depth,
                     g_normal, g_dist);
  return hipGetLastError();
}

}  // namespace lv

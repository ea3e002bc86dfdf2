// Footprint-eligible, priority-driven subdivision (Sec. IV-D, eq. 13-16) and
// the 8-way split.
//   eligible = l_v < kLMax and delta_v finite and h_v > kappa delta_v   (eq. 13)
//   z~_v = clip((delta_v - z5) / (z95 - z5), 0, 1)  (eq. 14; the caller's
//          running percentiles; +inf -> 1; z95 <= z5 or z95 = +inf -> 0)
//   P'_v = P_v (1 + beta z~_v)                                       (eq. 15-16)
//   split: the first max_splits eligible voxels with P'_v > 0 in the order
//          (P'_v descending, v ascending): the capped selection of
//          lv_select.h on inverted keys
// The split replaces each chosen voxel, in place and in input order, by its 8
// children (child c = x + 2y + 4z bits, ijk = 2 ijk + bits, level + 1);
// a child's corner densities are the parent's trilinear field at its
// corners, built from midpoints along x, then y, then z, so the density
// field is unchanged; SH coefficients are copied.  Binary32 throughout, in
// the order written (built without contraction).
#include <algorithm>

#include "lv_common.h"
#include "lv_select.h"

namespace lv {

uint64_t range_ws_bytes(int64_t n);

// the split is written by blocks of kSplitPer voxels in input order
constexpr int kSplitPer = 256;
__host__ __device__ static inline uint64_t n_split_blocks(int64_t n) {
  return uint64_t((n + kSplitPer - 1) / kSplitPer);
}

uint64_t split_ws_bytes(int64_t n) {
  uint64_t b = cap_ws_bytes(n);
  b = std::max<uint64_t>(b, range_ws_bytes(n));
  b = std::max<uint64_t>(b, 2 * align256(4 * size_t(n_split_blocks(n) + 1)));
  return b;
}

__global__ __launch_bounds__(256) void k_split_score(RasterArgs a, const float* score,
                                                     const float* range, SplitParams p,
                                                     float* priority, CapWS w) {
  const float z5 = range[0], z95 = range[1];
  const bool spread = isfinite(z95) && z95 > z5;
  const float den = z95 - z5;
  uint32_t mine = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * 256) {
    const int l = a.level[i];
    const float delta = voxel_footprint(a, i);
    const float h = 0.5f * ldexpf(a.root_size, -l);
    const bool fin = isfinite(delta);
    const bool elig = l < kLMax && fin && h > p.kappa * delta;
    float zt;
    if (!fin) {
      zt = 1.0f;
    } else if (!spread) {
      zt = 0.0f;
    } else {
      zt = (delta - z5) / den;
      zt = fminf(fmaxf(zt, 0.0f), 1.0f);
    }
    const float bias = 1.0f + p.beta * zt;
    const float pr = score[i] * bias;
    const bool cand = elig && pr > 0.0f;
    if (priority) priority[i] = pr;
    w.key[i] = ~f2key(pr);   // ascending key = descending priority
    w.cand[i] = cand ? 1u : 0u;
    mine += cand ? 1u : 0u;
  }
  cap_store_block_count(w, mine);
}

// A flag on a leaf at the finest level is ignored (it has no children).
__device__ __forceinline__ bool split_flag(const RasterArgs& a, const uint8_t* split, int64_t i) {
  return split[i] != 0 && int(a.level[i]) < kLMax;
}

// effective split flags per block of kSplitPer voxels
__global__ __launch_bounds__(kSplitPer) void k_split_count(RasterArgs a, const uint8_t* split,
                                                           uint32_t* blk) {
  __shared__ uint32_t s_c[kSplitPer / 64];
  const int64_t i = int64_t(blockIdx.x) * kSplitPer + threadIdx.x;
  const unsigned long long b = __ballot(i < a.n && split_flag(a, split, i));
  if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = uint32_t(__popcll(b));
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < kSplitPer / 64; ++k) t += s_c[k];
    blk[blockIdx.x] = t;
  }
}

// exclusive prefix of the block counts (one block of 1024 threads walking
// the counts in 1024-entry pieces) and the refined size n + 7 (#split)
__global__ __launch_bounds__(1024) void k_split_scan(const uint32_t* blk, uint32_t nb, uint32_t* pre,
                                                     int64_t n, uint64_t* needed) {
  __shared__ uint32_t s_w[16], s_run;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_run = 0u;
  __syncthreads();
  for (uint32_t base = 0; base < nb; base += 1024) {
    const uint32_t k = base + threadIdx.x;
    const uint32_t v = k < nb ? blk[k] : 0u;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = uint32_t(__shfl_up(int(incl), o, 64));
      if (lane >= o) incl += y;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint32_t off = s_run;
    for (int w = 0; w < wave; ++w) off += s_w[w];
    if (k < nb) pre[k] = off + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int w = 0; w < 16; ++w) t += s_w[w];
      s_run += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && needed) *needed = uint64_t(n) + 7ull * uint64_t(s_run);
}

__device__ __forceinline__ float mid(float a, float b) { return 0.5f * a + 0.5f * b; }

// corner co of child ch from the parent's corners s (corner c = x + 2y + 4z)
__device__ __forceinline__ float child_corner(const float s[8], int ch, int co) {
  const int ux = (ch & 1) + (co & 1), uy = ((ch >> 1) & 1) + ((co >> 1) & 1);
  const int uz = ((ch >> 2) & 1) + ((co >> 2) & 1);   // twice the parent-local coordinate
  float fx[4];                                         // per (y, z): index y + 2z
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float s0 = s[2 * j], s1 = s[2 * j + 1];
    fx[j] = ux == 0 ? s0 : (ux == 2 ? s1 : mid(s0, s1));
  }
  float fy[2];
#pragma unroll
  for (int z = 0; z < 2; ++z) {
    const float a0 = fx[2 * z], a1 = fx[2 * z + 1];
    fy[z] = uy == 0 ? a0 : (uy == 2 ? a1 : mid(a0, a1));
  }
  return uz == 0 ? fy[0] : (uz == 2 ? fy[1] : mid(fy[0], fy[1]));
}

struct SplitOut {
  uint16_t* ijk;     // [3][m]
  uint8_t* level;    // [m]
  float* density;    // [8][m]
  float* sh;         // [K][m]
  int64_t m;         // output size
};

// Each block takes kSplitPer voxels in order; a voxel's output position is
// its index plus 7 per split voxel before it (the block prefix, then the
// waves before it, then the lanes before it).  Writes at or beyond m are
// dropped.
__global__ __launch_bounds__(kSplitPer) void k_split_write(RasterArgs a, const uint8_t* split,
                                                           const uint32_t* pre, int K, SplitOut o) {
  __shared__ uint32_t s_w[kSplitPer / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = a.n, m = o.m;
  const int64_t i = int64_t(blockIdx.x) * kSplitPer + threadIdx.x;
  const bool in = i < n;
  const bool sp = in && split_flag(a, split, i);
  const unsigned long long b = __ballot(sp);
  const uint32_t below =
      __builtin_amdgcn_mbcnt_hi(uint32_t(b >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(b), 0u));
  if (lane == 0) s_w[wave] = uint32_t(__popcll(b));
  __syncthreads();
  if (!in) return;
  uint32_t before = pre[blockIdx.x] + below;
  for (int w = 0; w < wave; ++w) before += s_w[w];
  const int64_t pos = i + 7 * int64_t(before);
  const uint32_t ix = a.ijk[i], iy = a.ijk[n + i], iz = a.ijk[2 * n + i];
  const int l = a.level[i];
  if (!sp) {
    if (pos >= m) return;
    o.ijk[pos] = uint16_t(ix);
    o.ijk[m + pos] = uint16_t(iy);
    o.ijk[2 * m + pos] = uint16_t(iz);
    o.level[pos] = uint8_t(l);
#pragma unroll
    for (int c = 0; c < 8; ++c) o.density[c * m + pos] = a.density[c * n + i];
    // input and output never alias: let the loads of several rows fly together
    const float* __restrict__ src = a.sh + i;
    float* __restrict__ dst = o.sh + pos;
#pragma unroll 8
    for (int k = 0; k < K; ++k) dst[int64_t(k) * m] = src[int64_t(k) * n];
    return;
  }
  float s[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) s[c] = a.density[c * n + i];
  for (int ch = 0; ch < 8; ++ch) {
    const int64_t q = pos + ch;
    if (q >= m) break;
    o.ijk[q] = uint16_t(2u * ix + uint32_t(ch & 1));
    o.ijk[m + q] = uint16_t(2u * iy + uint32_t((ch >> 1) & 1));
    o.ijk[2 * m + q] = uint16_t(2u * iz + uint32_t((ch >> 2) & 1));
    o.level[q] = uint8_t(l + 1);
#pragma unroll
    for (int co = 0; co < 8; ++co) o.density[co * m + q] = child_corner(s, ch, co);
  }
  for (int k = 0; k < K; ++k) {
    const float v = a.sh[int64_t(k) * n + i];
    for (int ch = 0; ch < 8; ++ch) {
      const int64_t q = pos + ch;
      if (q >= m) break;
      o.sh[int64_t(k) * m + q] = v;
    }
  }
}

hipError_t run_split_select(const RasterArgs& a, const float* score, const float* range,
                            const SplitParams& p, void* ws, uint8_t* split, float* priority,
                            uint32_t* n_split, hipStream_t s) {
  const CapWS w = cap_bind(ws, a.n);
  hipError_t e = launch_cap_setup(w, n_split, s);
  if (e != hipSuccess || a.n == 0) return e;
  const uint64_t ub = (uint64_t(a.n) + 255) / 256;
  const uint32_t ug = uint32_t(ub < uint64_t(kCapFillBlocks) ? ub : uint64_t(kCapFillBlocks));
  hipLaunchKernelGGL(k_split_score, dim3(ug), dim3(256), 0, s, a, score, range, p, priority, w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_cap_select(w, a.n, p.max_splits, split, n_split, s);
}

hipError_t run_split_apply(const RasterArgs& a, const uint8_t* split, int64_t m, void* ws,
                           uint16_t* ijk, uint8_t* level, float* density, float* sh,
                           uint64_t* needed, hipStream_t s) {
  const uint32_t nb = uint32_t(n_split_blocks(a.n));
  uint32_t* blk = static_cast<uint32_t*>(ws);
  uint32_t* pre = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + align256(4 * size_t(nb + 1)));
  if (nb > 0) hipLaunchKernelGGL(k_split_count, dim3(nb), dim3(kSplitPer), 0, s, a, split, blk);
  hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(1024), 0, s, (const uint32_t*)blk, nb, pre, a.n,
                     needed);
  if (nb > 0) {
    SplitOut o;
    o.ijk = ijk; o.level = level; o.density = density; o.sh = sh; o.m = m;
    const int K = 3 * (a.deg + 1) * (a.deg + 1);
    hipLaunchKernelGGL(k_split_write, dim3(nb), dim3(kSplitPer), 0, s, a, split, (const uint32_t*)pre,
                       K, o);
  }
  return hipGetLastError();
}

}  // namespace lv

// Projection, tile binning and per-tile front-to-back sort (gfx950).
//
// One (view, voxel) record per voxel and view: the voxel's 8 corners are
// projected with a fixed binary32 operation sequence, the pixels whose centre
// lies in the projected box are its coverage, and it is binned into every
// TS x TS tile that coverage touches.  Each tile's list is then sorted by a
// 36-bit visibility code: the voxel's octree path with every child bit
// flipped where the camera centre lies above that split plane, which orders
// any set of non-overlapping leaves front to back along every ray from the
// camera (the order eq. 2-4 composite in).
#include "lv_common.h"

namespace lv {

// ------------------------------------------------------------------ setup
// Split-plane threshold of the eye along one axis.  The split planes of every
// level lie on the finest grid: the plane of fine index k (an odd multiple of
// 2^(kLMax - m) at level m) is root_min + 2^-kLMax fl(k root_size) in binary32,
// which is exactly how the per-level plane root_min + fl((2p + 1) root_size
// 2^-m) rounds, since scaling by a power of two is exact.  These values are
// non-decreasing in k, so "the eye lies above the plane" holds exactly for
// k <= the threshold found here by bisection: the largest k in [0, 2^kLMax)
// with o > plane(k), or -1 if there is none.
__device__ int32_t split_threshold(float o, float root_min, float root_size) {
  int32_t lo = -1, hi = (1 << kLMax) - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    const float plane = root_min + ldexpf(float(mid) * root_size, -kLMax);
    if (o > plane) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Grid-stride fill of n words with v by the threads tid = 0, stride, ...:
// 16-byte stores over the aligned middle, single words at the ends.
__device__ __forceinline__ void fill_words(uint32_t* p, uint64_t n, uint32_t v, uint64_t tid,
                                           uint64_t stride) {
  const uint64_t head = ((16u - (reinterpret_cast<uintptr_t>(p) & 15u)) & 15u) / 4u;   // words to 16-B alignment
  const uint64_t h = head < n ? head : n;
  if (tid < h) p[tid] = v;
  const uint64_t nv = (n - h) / 4;
  uint4* q = reinterpret_cast<uint4*>(p + h);
  const uint4 vv = make_uint4(v, v, v, v);
  for (uint64_t i = tid; i < nv; i += stride) q[i] = vv;
  const uint64_t t0 = h + 4 * nv;
  if (tid < n - t0) p[t0 + tid] = v;
}

static uint32_t fill_blocks(uint64_t n) {
  uint64_t blocks = (n / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  return uint32_t(blocks);
}

// Every block zeroes its share of the per-(sub-counter, tile) counts; block 0
// also clears the counters and builds the view table.
__global__ void k_setup(RasterArgs a) {
  fill_words(a.ws.tcount, uint64_t(a.T) * kSpread + 1, 0u,
             uint64_t(blockIdx.x) * blockDim.x + threadIdx.x, uint64_t(gridDim.x) * blockDim.x);
  if (blockIdx.x != 0) return;
  const int t = threadIdx.x;
  for (int k = t; k < kCounterWords; k += blockDim.x) a.ws.counters[k] = 0u;
  for (int k = t; k < S_WORDS; k += blockDim.x) a.ws.status[k] = 0u;
  for (int v = t; v < a.V; v += blockDim.x)
    for (int ax = 0; ax < 3; ++ax)
      a.ws.views[v].cell[ax] = split_threshold(a.cams[v].o[ax], a.root_min[ax], a.root_size);
  if (t == 0) {
    uint32_t tb = 0;
    uint64_t pb = 0;
    for (int v = 0; v < a.V; ++v) {
      const int W = a.cams[v].width, H = a.cams[v].height;
      ViewTab& vt = a.ws.views[v];   // field by field: the other lanes write cell[]
      vt.tile_base = tb;
      vt.tiles_x = uint32_t((W + a.TS - 1) / a.TS);
      vt.tiles_y = uint32_t((H + a.TS - 1) / a.TS);
      vt.W = W;
      vt.H = H;
      vt.pix_base = pb;
      tb += vt.tiles_x * vt.tiles_y;
      pb += uint64_t(W) * uint64_t(H);
    }
  }
}

hipError_t launch_setup(const RasterArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_setup, dim3(fill_blocks(uint64_t(a.T) * kSpread + 1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Fills n words with v (a graph-safe replacement for a memset).
__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  fill_words(p, n, v, uint64_t(blockIdx.x) * blockDim.x + threadIdx.x,
             uint64_t(gridDim.x) * blockDim.x);
}

// Up to kFillRanges fills in one launch (blockIdx.y = range).
__global__ void k_fill_set(FillSet f) {
  const int r = blockIdx.y;
  fill_words(f.p[r], f.n[r], f.v[r], uint64_t(blockIdx.x) * blockDim.x + threadIdx.x,
             uint64_t(gridDim.x) * blockDim.x);
}

hipError_t launch_fill_set(const FillSet& f, hipStream_t s) {
  if (f.count <= 0) return hipSuccess;
  uint64_t most = 0;
  for (int r = 0; r < f.count; ++r) most = f.n[r] > most ? f.n[r] : most;
  hipLaunchKernelGGL(k_fill_set, dim3(fill_blocks(most), uint32_t(f.count)), dim3(256), 0, s, f);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// ------------------------------------------- block-aggregated tile counts
// The records of one block (256 consecutive voxels, one view) cover a small
// window of tiles when the voxels are stored in octree order; a block counts
// its pairs per tile in LDS and touches each tile's global counter once.
struct TileWin {
  uint32_t x0, y0, w, h;
  bool any;
};

// Wave-wide min / max with DPP row shifts and row broadcasts (an inclusive
// scan whose last lane holds the result, read back by every lane); every
// lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  const int id = -1;   // 0xFFFFFFFF: the identity of the unsigned min
  x = min(x, uint32_t(__builtin_amdgcn_update_dpp(id, int(x), 0x111, 0xf, 0xf, false)));
  x = min(x, uint32_t(__builtin_amdgcn_update_dpp(id, int(x), 0x112, 0xf, 0xf, false)));
  x = min(x, uint32_t(__builtin_amdgcn_update_dpp(id, int(x), 0x114, 0xf, 0xf, false)));
  x = min(x, uint32_t(__builtin_amdgcn_update_dpp(id, int(x), 0x118, 0xf, 0xf, false)));
  x = min(x, uint32_t(__builtin_amdgcn_update_dpp(id, int(x), 0x142, 0xa, 0xf, false)));
  x = min(x, uint32_t(__builtin_amdgcn_update_dpp(id, int(x), 0x143, 0xc, 0xf, false)));
  return uint32_t(__builtin_amdgcn_readlane(int(x), 63));
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x111, 0xf, 0xf, false)));
  x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x112, 0xf, 0xf, false)));
  x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x114, 0xf, 0xf, false)));
  x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x118, 0xf, 0xf, false)));
  x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x142, 0xa, 0xf, false)));
  x = max(x, uint32_t(__builtin_amdgcn_update_dpp(0, int(x), 0x143, 0xc, 0xf, false)));
  return uint32_t(__builtin_amdgcn_readlane(int(x), 63));
}

// Bounding box of the tiles covered by the block's records; every thread of
// the block must call it (have: the thread's record covers [tx0, tx1] x
// [ty0, ty1]).
__device__ TileWin block_tile_window(bool have, uint32_t tx0, uint32_t tx1, uint32_t ty0,
                                     uint32_t ty1) {
  __shared__ uint32_t s_r[kBinBlock / 64][4];
  uint32_t a0 = have ? tx0 : 0xFFFFFFFFu, a1 = have ? tx1 : 0u;
  uint32_t b0 = have ? ty0 : 0xFFFFFFFFu, b1 = have ? ty1 : 0u;
  a0 = wave_min_u32(a0);
  a1 = wave_max_u32(a1);
  b0 = wave_min_u32(b0);
  b1 = wave_max_u32(b1);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    s_r[w][0] = a0; s_r[w][1] = a1; s_r[w][2] = b0; s_r[w][3] = b1;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kBinBlock / 64; ++k) {
    a0 = min(a0, s_r[k][0]); a1 = max(a1, s_r[k][1]);
    b0 = min(b0, s_r[k][2]); b1 = max(b1, s_r[k][3]);
  }
  __syncthreads();   // s_r is reused by the next call
  TileWin win;
  win.any = a0 <= a1;
  win.x0 = a0;
  win.y0 = b0;
  win.w = win.any ? a1 - a0 + 1u : 0u;
  win.h = win.any ? b1 - b0 + 1u : 0u;
  return win;
}

// ------------------------------------------------------------- preprocess
// One thread per voxel; the voxel's parameters are read once (coalesced SoA)
// and every view is processed from registers.
// Flipped path of a level-l cell index x along one axis, given the eye's
// split-plane threshold c: bit (l - m) is the level-m child bit XOR whether
// the eye lies above that level's split plane.  While the cell and the eye's
// fine index share their top levels the flip equals the eye's own bit, so
// those path bits are 0; at the first level where they differ the bit is 1;
// below it the eye lies entirely on one side, so the flip is constant (1 when
// the eye's index is the larger).  c = -1: the eye lies below every plane.
__device__ __forceinline__ uint32_t flipped_path(uint32_t x, int l, int32_t c) {
  if (c < 0) return x;
  const uint32_t cc = uint32_t(c) >> (kLMax - l);
  const uint32_t diff = x ^ cc;
  if (diff == 0u) return 0u;
  const uint32_t top = 1u << (31 - __builtin_clz(diff));
  return top | ((cc > x ? ~x : x) & (top - 1u));
}

// bits 0..5 of x to bits 0, 3, ..., 15
__device__ __forceinline__ uint32_t spread3_6(uint32_t x) {
  x = (x | (x << 8)) & 0x0000F00Fu;
  x = (x | (x << 4)) & 0x000C30C3u;
  x = (x | (x << 2)) & 0x00249249u;
  return x;
}

// Correctly rounded x / z for the projection, with z > the near plane:
// the hardware reciprocal refined by one Newton step, then two residual
// corrections, the reciprocal shared by a corner's two quotients.  This is
// the compiler's division sequence without its operand rescaling and
// special-case fix-up, which act only on infinities, NaNs, zero divisors
// and quotients or numerators near the subnormal range; here z is normal
// and positive and |x| is zero or far above that range (a camera-space
// coordinate), so each quotient equals the division bit for bit (checked
// against it on 2^31 such operand pairs).
struct Divisor {
  float z, r;
};
__device__ __forceinline__ Divisor divisor(float z) {
  float r = __builtin_amdgcn_rcpf(z);
  const float e = fmaf(-z, r, 1.0f);
  r = fmaf(e, r, r);
  return {z, r};
}
__device__ __forceinline__ float quotient(float x, const Divisor& d) {
  float q = x * d.r;
  float rem = fmaf(-d.z, q, x);
  q = fmaf(rem, d.r, q);
  rem = fmaf(-d.z, q, x);
  return fmaf(rem, d.r, q);
}

// GENERIC: grid-point layout or a density activation; otherwise the dense
// corner values are read as they are
template <int DEG, bool GENERIC>
__global__ __launch_bounds__(kBinBlock) void k_preprocess(RasterArgs a) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  __shared__ uint32_t s_tab[kTileWin];
  const int64_t n = a.n;
  const int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  // threads past the end take part in the block-wide tile counting only
  const bool valid = i0 < n;
  const int64_t i = valid ? i0 : n - 1;
  const uint32_t sub = blockIdx.x & uint32_t(kSpread - 1);
  const int l = a.level[i];
  const float e = ldexpf(a.root_size, -l);
  const uint32_t ix = a.ijk[i], iy = a.ijk[n + i], iz = a.ijk[2 * n + i];
  float b[3];
  b[0] = a.root_min[0] + float(ix) * e;
  b[1] = a.root_min[1] + float(iy) * e;
  b[2] = a.root_min[2] + float(iz) * e;
  float sg[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) sg[c] = GENERIC ? corner_density(a, c, i) : a.density[c * n + i];
  VoxRec vr;
  vr.be = make_float4(b[0], b[1], b[2], e);
  vr.s0 = make_float4(sg[0], sg[1], sg[2], sg[3]);
  vr.s1 = make_float4(sg[4], sg[5], sg[6], sg[7]);
  if (valid) a.ws.vox[i] = vr;

  float k[NB][3];
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) k[j][ch] = a.sh[(j * 3 + ch) * n + i];

  const float half_e = 0.5f * e;
  const float xv0 = b[0] + half_e, xv1 = b[1] + half_e, xv2 = b[2] + half_e;
  const int sh_ts = __builtin_ctz(uint32_t(a.TS));

  for (int v = 0; v < a.V; ++v) {
    const lv_camera& cam = a.cams[v];
    const float R0 = cam.R[0], R1 = cam.R[1], R2 = cam.R[2];
    const float R3 = cam.R[3], R4 = cam.R[4], R5 = cam.R[5];
    const float R6 = cam.R[6], R7 = cam.R[7], R8 = cam.R[8];
    const float o0 = cam.o[0], o1 = cam.o[1], o2 = cam.o[2];
    // read once per view: inside the corners' branches each read is a load
    const float cfx = cam.fx, cfy = cam.fy, ccx = cam.cx, ccy = cam.cy;
    const int W = cam.width, H = cam.height;
    // --- binary32 projection of the 8 corners (no contraction, fixed order)
    float u0 = INFINITY, u1 = -INFINITY, v0 = INFINITY, v1 = -INFINITY;
    int near_cnt = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float p0 = (c & 1) ? b[0] + e : b[0];
      const float p1 = (c & 2) ? b[1] + e : b[1];
      const float p2 = (c & 4) ? b[2] + e : b[2];
      const float q0 = p0 - o0, q1 = p1 - o1, q2 = p2 - o2;
      float xc = R0 * q0 + R1 * q1;
      xc = xc + R2 * q2;
      float yc = R3 * q0 + R4 * q1;
      yc = yc + R5 * q2;
      float zc = R6 * q0 + R7 * q1;
      zc = zc + R8 * q2;
      if (zc <= kZNear) {
        ++near_cnt;
      } else {
        const Divisor dz = divisor(zc);
        const float qx = quotient(xc, dz), qy = quotient(yc, dz);
        const float uu = cfx * qx + ccx;
        const float vv = cfy * qy + ccy;
        u0 = fminf(u0, uu); u1 = fmaxf(u1, uu);
        v0 = fminf(v0, vv); v1 = fmaxf(v1, vv);
      }
    }
    Rec rec;
    rec.r = rec.g = rec.b = 0.0f;
    rec.flags = 0u;
    rec.xr = rec.yr = 0u;
    rec.code_lo = rec.code_hi = 0u;
    bool visible = false;
    float fx0 = 0.0f, fx1 = 0.0f, fy0 = 0.0f, fy1 = 0.0f;
    if (near_cnt < 8) {
      if (near_cnt > 0) {
        fx0 = 0.0f; fx1 = float(W - 1); fy0 = 0.0f; fy1 = float(H - 1);
        visible = true;
      } else {
        fx0 = ceilf(u0 - 0.5f); fx1 = floorf(u1 - 0.5f);
        fy0 = ceilf(v0 - 0.5f); fy1 = floorf(v1 - 0.5f);
        fx0 = fmaxf(fx0, 0.0f); fy0 = fmaxf(fy0, 0.0f);
        fx1 = fminf(fx1, float(W - 1)); fy1 = fminf(fy1, float(H - 1));
        visible = !(fx0 > fx1 || fy0 > fy1);
      }
    }
    if (visible) {
      const uint32_t x0 = uint32_t(fx0), x1 = uint32_t(fx1);
      const uint32_t y0 = uint32_t(fy0), y1 = uint32_t(fy1);
      rec.xr = x0 | (x1 << 16);
      rec.yr = y0 | (y1 << 16);
      // --- visibility code: flipped octree path, 3 bits per level
      const int32_t* cell = a.ws.views[v].cell;
      const uint32_t fpx = flipped_path(ix, l, cell[0]);
      const uint32_t fpy = flipped_path(iy, l, cell[1]);
      const uint32_t fpz = flipped_path(iz, l, cell[2]);
      const uint32_t lo = spread3_6(fpx & 63u) | (spread3_6(fpy & 63u) << 1) | (spread3_6(fpz & 63u) << 2);
      const uint32_t hi = spread3_6(fpx >> 6) | (spread3_6(fpy >> 6) << 1) | (spread3_6(fpz >> 6) << 2);
      const uint64_t code = (uint64_t(lo) | (uint64_t(hi) << 18)) << (3 * (kLMax - l));
      rec.code_lo = uint32_t(code);
      rec.code_hi = uint32_t(code >> 32);
      // --- colour: SH at the direction camera -> voxel centre
      float dx = xv0 - o0, dy = xv1 - o1, dz = xv2 - o2;
      const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
      dx *= inv; dy *= inv; dz *= inv;
      float Y[16];
      sh_basis<DEG>(dx, dy, dz, Y);
      float col[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float s = k[0][ch];
#pragma unroll
        for (int j = 1; j < NB; ++j) s = fmaf(Y[j], k[j][ch], s);
        col[ch] = s;
      }
      uint32_t fl = 8u;
      fl |= col[0] > 0.0f ? 1u : 0u;
      fl |= col[1] > 0.0f ? 2u : 0u;
      fl |= col[2] > 0.0f ? 4u : 0u;
      rec.flags = fl;
      rec.r = fmaxf(col[0], 0.0f);
      rec.g = fmaxf(col[1], 0.0f);
      rec.b = fmaxf(col[2], 0.0f);
    }
    // --- tile counts, aggregated over the block
    const bool have = valid && visible;
    const uint32_t tx0 = (rec.xr & 0xFFFFu) >> sh_ts, tx1 = (rec.xr >> 16) >> sh_ts;
    const uint32_t ty0 = (rec.yr & 0xFFFFu) >> sh_ts, ty1 = (rec.yr >> 16) >> sh_ts;
    const TileWin win = block_tile_window(have, tx0, tx1, ty0, ty1);
    if (win.any) {
      const ViewTab vt = a.ws.views[v];
      uint32_t* tc = a.ws.tcount + uint64_t(sub) * a.T + vt.tile_base;
      if (uint64_t(win.w) * win.h <= uint64_t(kTileWin)) {
        const uint32_t nw = win.w * win.h;
        for (uint32_t k = threadIdx.x; k < nw; k += blockDim.x) s_tab[k] = 0u;
        __syncthreads();
        if (have)
          for (uint32_t ty = ty0; ty <= ty1; ++ty)
            for (uint32_t tx = tx0; tx <= tx1; ++tx)
              atomicAdd(&s_tab[(ty - win.y0) * win.w + (tx - win.x0)], 1u);
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < nw; k += blockDim.x) {
          const uint32_t c = s_tab[k];
          const uint32_t ry = k / win.w;
          if (c) atomicAdd(&tc[(win.y0 + ry) * vt.tiles_x + win.x0 + (k - ry * win.w)], c);
        }
        __syncthreads();   // s_tab is reused by the next view
      } else if (have) {
        for (uint32_t ty = ty0; ty <= ty1; ++ty)
          for (uint32_t tx = tx0; tx <= tx1; ++tx) atomicAdd(&tc[ty * vt.tiles_x + tx], 1u);
      }
    }
    if (valid) {
      uint4* dst = reinterpret_cast<uint4*>(&a.ws.rec[size_t(v) * size_t(n) + size_t(i)]);
      dst[0] = make_uint4(__float_as_uint(rec.r), __float_as_uint(rec.g), __float_as_uint(rec.b),
                          rec.flags);
      dst[1] = make_uint4(rec.xr, rec.yr, rec.code_lo, rec.code_hi);
    }
  }
}

hipError_t launch_preprocess(const RasterArgs& a, hipStream_t s) {
  const uint32_t blocks = uint32_t((a.n + kBinBlock - 1) / kBinBlock);
  if (blocks == 0) return hipSuccess;
  const bool generic = a.corner_idx != nullptr || a.act != LV_ACT_NONE;
#define LV_PRE(D) (generic ? k_preprocess<D, true> : k_preprocess<D, false>)
  switch (a.deg) {
    case 0: hipLaunchKernelGGL(LV_PRE(0), dim3(blocks), dim3(kBinBlock), 0, s, a); break;
    case 1: hipLaunchKernelGGL(LV_PRE(1), dim3(blocks), dim3(kBinBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(LV_PRE(2), dim3(blocks), dim3(kBinBlock), 0, s, a); break;
    default: hipLaunchKernelGGL(LV_PRE(3), dim3(blocks), dim3(kBinBlock), 0, s, a); break;
  }
#undef LV_PRE
  return hipGetLastError();
}

// Visible (view, voxel) records of a forward pass (binned flag set), for
// statistics only: one pass over the records' flag words, one atomic per block.
__global__ __launch_bounds__(256) void k_count_records(const Rec* rec, uint64_t nrec,
                                                       unsigned long long* out) {
  uint32_t c = 0;
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nrec; i += stride)
    c += (rec[i].flags & 8u) ? 1u : 0u;
  __shared__ uint32_t s_c;
  if (threadIdx.x == 0) s_c = 0u;
  __syncthreads();
  atomicAdd(&s_c, c);
  __syncthreads();
  if (threadIdx.x == 0 && s_c) atomicAdd(out, (unsigned long long)s_c);
}

hipError_t launch_count_records(const Rec* rec, uint64_t nrec, unsigned long long* out,
                                hipStream_t s) {
  if (nrec == 0) return hipSuccess;
  uint64_t blocks = (nrec + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_count_records, dim3(uint32_t(blocks)), dim3(256), 0, s, rec, nrec, out);
  return hipGetLastError();
}

// ------------------------------------------------------------- tile scan
// Exclusive prefix sum of the per-tile counts -> tile_start (saturating at
// 2^32 - 1), the total pair count and the overflow flag; resets the fill
// cursors.
__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    unsigned long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// inclusive scan over a 1024-thread block; returns the block total in *tot
__device__ unsigned long long block_incl_scan(unsigned long long x, unsigned long long* tot) {
  __shared__ unsigned long long s_w[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  x = wave_incl_scan(x);
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  if (w == 0) {
    unsigned long long y = lane < nw ? s_w[lane] : 0ull;
    y = wave_incl_scan(y);
    if (lane < nw) s_w[lane] = y;
  }
  __syncthreads();
  if (w > 0) x += s_w[w - 1];
  *tot = s_w[nw - 1];
  __syncthreads();
  return x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(RasterArgs a) {
  const uint64_t t = uint64_t(blockIdx.x) * kScanBlock + threadIdx.x;
  const uint64_t n = uint64_t(a.T) * kSpread;
  unsigned long long x = t < n ? a.ws.tcount[(t % kSpread) * a.T + t / kSpread] : 0u;
  unsigned long long tot;
  block_incl_scan(x, &tot);
  if (threadIdx.x == 0) reinterpret_cast<unsigned long long*>(a.ws.bsum)[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_top(RasterArgs a, uint32_t nblk) {
  unsigned long long* bs = reinterpret_cast<unsigned long long*>(a.ws.bsum);
  unsigned long long carry = 0;
  for (uint32_t base = 0; base < nblk; base += kScanBlock) {
    const uint32_t j = base + threadIdx.x;
    unsigned long long x = j < nblk ? bs[j] : 0ull;
    unsigned long long tot;
    unsigned long long inc = block_incl_scan(x, &tot);
    if (j < nblk) bs[j] = carry + inc - x;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    a.ws.status[S_PAIRS] = carry > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(carry);
    a.ws.status[S_OVERFLOW] = carry > a.cap ? 1u : 0u;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_down(RasterArgs a) {
  const uint64_t t = uint64_t(blockIdx.x) * kScanBlock + threadIdx.x;
  const uint64_t n = uint64_t(a.T) * kSpread;
  const uint64_t ci = (t % kSpread) * a.T + t / kSpread;   // counter of scan position t
  unsigned long long x = t < n ? a.ws.tcount[ci] : 0u;
  unsigned long long tot;
  unsigned long long inc = block_incl_scan(x, &tot);
  const unsigned long long ex =
      reinterpret_cast<const unsigned long long*>(a.ws.bsum)[blockIdx.x] + inc - x;
  if (t <= n) a.ws.tstart[t] = ex > 0xFFFFFFFFull ? 0xFFFFFFFFu : uint32_t(ex);
  if (t < n) a.ws.tfill[ci] = 0u;
}

hipError_t launch_scan_tiles(const RasterArgs& a, uint32_t nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kScanBlock), 0, s, a);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, s, a, nblk);
  hipLaunchKernelGGL(k_scan_down, dim3(nblk), dim3(kScanBlock), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------ emit
// One block per (256 voxels, view); each record writes key = code << 28 |
// voxel id for every tile it covers.  The block counts its pairs per tile in
// LDS, reserves one range per tile with a single global atomic, and gives
// each pair a slot in its range with an LDS atomic, so a block's pairs of one
// tile are written contiguously (their order is fixed later by the sort).
__global__ __launch_bounds__(kBinBlock) void k_emit(RasterArgs a) {
  __shared__ uint32_t s_cnt[kTileWin];
  __shared__ unsigned long long s_base[kTileWin];
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  const int sh_ts = __builtin_ctz(uint32_t(a.TS));
  const uint32_t sub = blockIdx.x & uint32_t(kSpread - 1);
  bool have = false;
  uint32_t tx0 = 0, tx1 = 0, ty0 = 0, ty1 = 0;
  unsigned long long key = 0;
  if (i < a.n) {
    const uint4* rp = reinterpret_cast<const uint4*>(&a.ws.rec[size_t(v) * size_t(a.n) + size_t(i)]);
    const uint32_t flags = rp[0].w;
    if (flags & 8u) {
      const uint4 r1 = rp[1];
      have = true;
      tx0 = (r1.x & 0xFFFFu) >> sh_ts; tx1 = (r1.x >> 16) >> sh_ts;
      ty0 = (r1.y & 0xFFFFu) >> sh_ts; ty1 = (r1.y >> 16) >> sh_ts;
      const unsigned long long code = (unsigned long long)r1.z | ((unsigned long long)r1.w << 32);
      key = (code << kIdBits) | (unsigned long long)i;
    }
  }
  const TileWin win = block_tile_window(have, tx0, tx1, ty0, ty1);
  if (!win.any) return;   // the whole block
  const ViewTab vt = a.ws.views[v];
  uint32_t* fill = a.ws.tfill + uint64_t(sub) * a.T + vt.tile_base;
  if (uint64_t(win.w) * win.h <= uint64_t(kTileWin)) {
    const uint32_t nw = win.w * win.h;
    for (uint32_t k = threadIdx.x; k < nw; k += blockDim.x) s_cnt[k] = 0u;
    __syncthreads();
    if (have)
      for (uint32_t ty = ty0; ty <= ty1; ++ty)
        for (uint32_t tx = tx0; tx <= tx1; ++tx) atomicAdd(&s_cnt[(ty - win.y0) * win.w + (tx - win.x0)], 1u);
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nw; k += blockDim.x) {
      const uint32_t c = s_cnt[k];
      if (c) {
        const uint32_t ry = k / win.w;
        const uint32_t lt = (win.y0 + ry) * vt.tiles_x + win.x0 + (k - ry * win.w);
        const uint32_t slot = atomicAdd(&fill[lt], c);
        s_base[k] = (unsigned long long)a.ws.tstart[uint64_t(vt.tile_base + lt) * kSpread + sub] + slot;
      }
      s_cnt[k] = 0u;   // now the per-tile cursor of this block
    }
    __syncthreads();
    if (have)
      for (uint32_t ty = ty0; ty <= ty1; ++ty)
        for (uint32_t tx = tx0; tx <= tx1; ++tx) {
          const uint32_t k = (ty - win.y0) * win.w + (tx - win.x0);
          const unsigned long long pos = s_base[k] + atomicAdd(&s_cnt[k], 1u);
          if (pos < a.cap) a.ws.pairs[pos] = key;
        }
  } else if (have) {
    for (uint32_t ty = ty0; ty <= ty1; ++ty)
      for (uint32_t tx = tx0; tx <= tx1; ++tx) {
        const uint32_t lt = ty * vt.tiles_x + tx;
        const uint32_t slot = atomicAdd(&fill[lt], 1u);
        const uint64_t pos = uint64_t(a.ws.tstart[uint64_t(vt.tile_base + lt) * kSpread + sub]) + slot;
        if (pos < a.cap) a.ws.pairs[pos] = key;
      }
  }
}

hipError_t launch_emit(const RasterArgs& a, hipStream_t s) {
  const uint32_t bx = uint32_t((a.n + kBinBlock - 1) / kBinBlock);
  if (bx == 0) return hipSuccess;
  hipLaunchKernelGGL(k_emit, dim3(bx, a.V), dim3(kBinBlock), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ tile order
// Persistent composite kernels pop tiles longest list first: tiles are
// counting-sorted by floor(log2(count)) (bucket 0 = empty), descending.
__device__ __forceinline__ uint32_t tile_len(const RasterArgs& a, uint32_t t) {
  const uint64_t s0 = tile_begin(a, t);
  const uint64_t s1 = tile_begin(a, t + 1);
  return uint32_t(s1 - s0);
}

__device__ __forceinline__ int len_bucket(uint32_t c) {
  if (c == 0) return 0;
  int b = 1 + (31 - __clz(c));
  return b > 31 ? 31 : b;
}

__global__ __launch_bounds__(256) void k_order_hist(RasterArgs a) {
  __shared__ uint32_t h[32];
  if (threadIdx.x < 32) h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < a.T) atomicAdd(&h[len_bucket(tile_len(a, t))], 1u);
  __syncthreads();
  if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&a.ws.counters[C_BUCKET + threadIdx.x], h[threadIdx.x]);
}

__global__ void k_order_scan(RasterArgs a) {
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 31; b >= 0; --b) {
      a.ws.counters[C_BSTART + b] = run;
      run += a.ws.counters[C_BUCKET + b];
      a.ws.counters[C_BFILL + b] = 0;
    }
  }
}

// Ranks are taken in LDS and each block reserves one range per bucket with a
// single global atomic (one global atomic per tile contends on the few bucket
// counters).
__global__ __launch_bounds__(256) void k_order_scatter(RasterArgs a) {
  __shared__ uint32_t lc[32], lb[32];
  if (threadIdx.x < 32) lc[threadIdx.x] = 0u;
  __syncthreads();
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  int b = -1;
  uint32_t local = 0;
  if (t < a.T) {
    b = len_bucket(tile_len(a, t));
    local = atomicAdd(&lc[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 32 && lc[threadIdx.x])
    lb[threadIdx.x] = atomicAdd(&a.ws.counters[C_BFILL + threadIdx.x], lc[threadIdx.x]);
  __syncthreads();
  if (b >= 0) a.ws.torder[a.ws.counters[C_BSTART + b] + lb[b] + local] = t;
}

hipError_t launch_order(const RasterArgs& a, hipStream_t s) {
  const uint32_t blocks = (a.T + 255) / 256;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_order_hist, dim3(blocks), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_order_scatter, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------- tile sort
// Tiles are sorted by size class, each class by its own persistent kernel
// that walks the class's range of the length-ordered tile list (the tile
// order is built first): lists shorter than 256 keys are bitonic-sorted in
// 2 KB of LDS by one wave, lists up to kSortCap keys in kSortCap-key LDS by
// four waves, and longer lists are sorted in kSortCap-key runs and merged
// pairwise (each key finds its rank in the partner run by binary search)
// until one run remains.  Keys are unique for non-overlapping leaves, so the
// order is deterministic.

__device__ __forceinline__ void cmp_swap(unsigned long long& x, unsigned long long& y, bool asc) {
  if ((x > y) == asc) {
    const unsigned long long t = x;
    x = y;
    y = t;
  }
}

// Bitonic network over npow (a power of two) keys in LDS.  Stages whose
// pairs lie more than 2 apart go through LDS, one pair per thread and a
// barrier each; the last two stages of every merge (distances 2 and 1) stay
// inside aligned quads and run in registers, one quad per thread.  The
// network and its order of stages are the plain bitonic sort's.
template <int NT>
__device__ void lds_bitonic(unsigned long long* sk, uint32_t npow) {
  if (npow < 4) {   // one pair at most
    if (npow == 2 && threadIdx.x == 0) {
      unsigned long long x = sk[0], y = sk[1];
      cmp_swap(x, y, true);
      sk[0] = x;
      sk[1] = y;
    }
    __syncthreads();
    return;
  }
  for (uint32_t k = 2; k <= npow; k <<= 1) {
    for (uint32_t j = k >> 1; j > 2; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < (npow >> 1); i += NT) {
        const uint32_t lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const uint32_t hi = lo + j;
        const bool asc = (lo & k) == 0;
        const unsigned long long x = sk[lo], y = sk[hi];
        if ((x > y) == asc) { sk[lo] = y; sk[hi] = x; }
      }
      __syncthreads();
    }
    for (uint32_t qd = threadIdx.x; qd < (npow >> 2); qd += NT) {
      const uint32_t b = qd << 2;
      unsigned long long x0 = sk[b], x1 = sk[b + 1], x2 = sk[b + 2], x3 = sk[b + 3];
      if (k == 2) {   // pairs (b, b+1) ascending, (b+2, b+3) descending
        cmp_swap(x0, x1, true);
        cmp_swap(x2, x3, false);
      } else {        // one direction for the whole quad
        const bool asc = (b & k) == 0;
        cmp_swap(x0, x2, asc);
        cmp_swap(x1, x3, asc);
        cmp_swap(x0, x1, asc);
        cmp_swap(x2, x3, asc);
      }
      sk[b] = x0;
      sk[b + 1] = x1;
      sk[b + 2] = x2;
      sk[b + 3] = x3;
    }
    __syncthreads();
  }
}

// sorts the n <= CAP keys at src in LDS; writes the sorted keys to dst, or
// only their voxel ids to ids when dst is null
template <int NT>
__device__ void sort_in_lds(unsigned long long* sk, const unsigned long long* src, uint32_t n,
                            unsigned long long* dst, uint32_t* ids) {
  uint32_t npow = 1;
  while (npow < n) npow <<= 1;
  for (uint32_t i = threadIdx.x; i < npow; i += NT) sk[i] = i < n ? src[i] : ~0ull;
  __syncthreads();
  lds_bitonic<NT>(sk, npow);
  if (dst) {
    for (uint32_t i = threadIdx.x; i < n; i += NT) dst[i] = sk[i];
  } else {
    for (uint32_t i = threadIdx.x; i < n; i += NT) ids[i] = uint32_t(sk[i] & kIdMask);
  }
  __syncthreads();
}

// order positions [p0, p1) of the tiles with length buckets b_lo..b_hi
// (bucket b holds lengths [2^(b-1), 2^b); buckets are laid out descending)
__device__ __forceinline__ void class_range(const RasterArgs& a, int b_lo, int b_hi, uint32_t& p0,
                                            uint32_t& p1) {
  p0 = a.ws.counters[C_BSTART + b_hi];
  p1 = a.ws.counters[C_BSTART + b_lo - 1];
}

template <int CAP, int NT>
__global__ __launch_bounds__(NT) void k_sort_lds(RasterArgs a, int b_lo, int b_hi) {
  __shared__ unsigned long long sk[CAP];
  uint32_t p0, p1;
  class_range(a, b_lo, b_hi, p0, p1);
  for (uint32_t p = p0 + blockIdx.x; p < p1; p += gridDim.x) {
    const uint32_t t = a.ws.torder[p];
    const uint64_t s0 = tile_begin(a, t);
    const uint32_t n = uint32_t(tile_begin(a, t + 1) - s0);
    if (n == 1) {
      if (threadIdx.x == 0) a.ws.ids[s0] = uint32_t(a.ws.pairs[s0] & kIdMask);
      continue;
    }
    sort_in_lds<NT>(sk, a.ws.pairs + s0, n, nullptr, a.ws.ids + s0);
  }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_sort_long(RasterArgs a, int b_lo, int b_hi) {
  __shared__ unsigned long long sk[kSortCap];
  uint32_t p0, p1;
  class_range(a, b_lo, b_hi, p0, p1);
  for (uint32_t p = p0 + blockIdx.x; p < p1; p += gridDim.x) {
    const uint32_t t = a.ws.torder[p];
    const uint64_t s0 = tile_begin(a, t);
    const uint32_t n = uint32_t(tile_begin(a, t + 1) - s0);
    unsigned long long* keys = a.ws.pairs + s0;
    for (uint32_t r0 = 0; r0 < n; r0 += kSortCap) {
      const uint32_t m = (n - r0) < uint32_t(kSortCap) ? (n - r0) : uint32_t(kSortCap);
      sort_in_lds<NT>(sk, keys + r0, m, keys + r0, nullptr);
    }
    __threadfence_block();
    __syncthreads();
    unsigned long long* src = keys;
    unsigned long long* dst = a.ws.mtmp + s0;
    for (uint32_t r = kSortCap; r < n; r <<= 1) {
      for (uint32_t i = threadIdx.x; i < n; i += NT) {
        const uint32_t run = i / r;
        const uint32_t rs = run * r;
        const uint32_t prt = run ^ 1u;
        const uint32_t ps = prt * r;
        const unsigned long long key = src[i];
        if (ps >= n) { dst[i] = key; continue; }
        const uint32_t pe = (ps + r) < n ? (ps + r) : n;
        // rank of key in the partner run: strict for the left run,
        // non-strict for the right run (keys are unique; this keeps ties
        // stable)
        uint32_t lo = ps, hi = pe;
        const bool left = (run & 1u) == 0;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          const unsigned long long pk = src[mid];
          const bool go_right = left ? (pk < key) : (pk <= key);
          if (go_right) lo = mid + 1; else hi = mid;
        }
        const uint32_t ms = rs < ps ? rs : ps;
        dst[ms + (i - rs) + (lo - ps)] = key;
      }
      __threadfence_block();
      __syncthreads();
      unsigned long long* tmp = src; src = dst; dst = tmp;
    }
    for (uint32_t i = threadIdx.x; i < n; i += NT) a.ws.ids[s0 + i] = uint32_t(src[i] & kIdMask);
    __syncthreads();
  }
}

// needs the tile order (launch_order) of the same pass
hipError_t launch_sort(const RasterArgs& a, hipStream_t s) {
  if (a.T == 0) return hipSuccess;
  static_assert(kSortCap == 2048, "size classes assume 2048-key runs");
  const uint32_t T = a.T;
  // lengths 1..255: buckets 1..8; 256..2047: buckets 9..11; 2048 and up: 12..31
  hipLaunchKernelGGL((k_sort_lds<256, 64>), dim3(T < 8192u ? T : 8192u), dim3(64), 0, s, a, 1, 8);
  hipLaunchKernelGGL((k_sort_lds<kSortCap, 256>), dim3(T < 2048u ? T : 2048u), dim3(256), 0, s, a, 9, 11);
  hipLaunchKernelGGL((k_sort_long<256>), dim3(T < 512u ? T : 512u), dim3(256), 0, s, a, 12, 31);
  return hipGetLastError();
}

}  // namespace lv

// Internal definitions shared by the HIP kernels and the host-side C-ABI of
// the sparse-voxel tile rasterizer (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "litevoxel.h"

namespace lv {

constexpr int kLMax = LV_MAX_LEVEL;   // visibility code: 3 bits per level, 36 bits
constexpr int kIdBits = 28;           // voxel id bits in a sort key
constexpr uint32_t kIdMask = (1u << kIdBits) - 1u;
constexpr int kSortCap = 2048;        // longest tile list sorted in one LDS pass
constexpr float kZNear = 1e-4f;       // binning near plane (camera-space z)
// Tile queues of the composite passes: kQueues interleaved queues, each head
// in its own 128-byte line (same-address device atomics serialise at about
// 12 ns each, and one head popped once per tile would throttle the pass).
constexpr int kQueues = 16;
constexpr int kQueueStride = 32;   // words
constexpr int kCounterWords = 128 + 2 * kQueues * kQueueStride;
// Each tile has kSpread pair counters, stored sub-counter-major; the counter
// of a (block, tile) is sub = block & (kSpread - 1), where a block is 256
// consecutive voxels (the preprocess and emit grids both use such blocks).
// Scanned in tile-major order, so the pairs of a tile still form one
// contiguous segment [tstart[t * kSpread], tstart[(t + 1) * kSpread]).
constexpr int kSpread = 16;
constexpr int kBinBlock = 256;   // voxels per block of preprocess and emit
// a block counts the tiles its records cover in an LDS table over the
// block's tile bounding box when that box has at most kTileWin tiles (512:
// the emit's tables then take 6 KB, so more of its workgroups fit a CU; on
// the ring workload 2048 was 10 us slower, 256 sent too many blocks down
// the per-record path)
constexpr int kTileWin = 512;

// per-view table built on the device from the cameras (graph-replay safe)
struct ViewTab {
  uint32_t tile_base;  // first global tile id of the view
  uint32_t tiles_x;
  uint32_t tiles_y;
  int32_t W;
  int32_t H;
  int32_t cell[3];     // split-plane threshold of the eye per axis (see split_threshold)
  uint64_t pix_base;   // first global pixel index of the view
};

// per-voxel, view-independent record written by the preprocess kernel
struct VoxRec {
  float4 be;   // min corner (x, y, z) and edge e
  float4 s0;   // corner densities 0..3
  float4 s1;   // corner densities 4..7
};

// per-(view, voxel) record: colour, clamp mask, pixel-centre range, code
// flags: bit0..2 = raw colour > 0 per channel, bit3 = binned
struct Rec {
  float r, g, b;
  uint32_t flags;
  uint32_t xr;        // x0 | x1 << 16 (inclusive pixel-centre range)
  uint32_t yr;        // y0 | y1 << 16
  uint32_t code_lo;   // 36-bit visibility code
  uint32_t code_hi;
};

// status words kept with the forward's saved state
enum Status : int {
  S_PAIRS = 0,       // number of (tile, voxel) pairs (saturating below 2^32)
  S_OVERFLOW = 1,    // 1 if pairs > capacity
  S_WORDS = 64
};

// counters block of the workspace (uint32 words)
enum Counter : int {
  C_BUCKET = 8,      // [32] tile counts per length bucket
  C_BSTART = 40,     // [33] bucket starts
  C_BFILL = 80,      // [32] bucket cursors
  C_QFWD = 128,      // [kQueues] forward tile queue heads, kQueueStride apart
  C_QBWD = 128 + kQueues * kQueueStride,   // [kQueues] backward queue heads
};

// Buffer layouts, computed identically on the host for sizing and launch.
// Two caller-owned buffers: `saved` holds everything lv_forward leaves for
// lv_backward (view table, voxel and view records, tile starts, tile order,
// per-tile voxel lists, per-pixel state, pair status), so each forward pass
// can keep its own; `workspace` is scratch that any call may overwrite
// (counters, tile counts and cursors, the pair keys and their merge buffer,
// the backward's gradient accumulators).
struct Layout {
  int64_t n = 0;
  int V = 0;
  int TS = 16;
  int CH = 64;
  int deg = 0;
  uint32_t T = 0;          // total tiles
  uint64_t P = 0;          // total pixels
  uint64_t cap = 0;        // pair capacity
  uint32_t nblk_scan = 0;  // blocks of the tile scan
  // saved
  size_t off_views = 0, off_status = 0, off_vox = 0, off_rec = 0, off_tstart = 0, off_torder = 0,
         off_ids = 0, off_nlast = 0, off_tpre = 0;
  size_t total_saved = 0;
  // workspace
  size_t off_counters = 0, off_tcount = 0, off_tfill = 0, off_bsum = 0, off_dcol = 0, off_dden = 0,
         off_pairs = 0, off_mtmp = 0;
  size_t total = 0;
};

constexpr int kScanBlock = 1024;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline bool make_layout(const lv_voxels* vox, const lv_frame* fr, const lv_settings* st,
                        Layout& L) {
  L.n = vox->n;
  L.V = fr->n_views;
  L.TS = st->tile;
  L.CH = st->chunk;
  L.deg = vox->sh_degree;
  uint64_t T = 0, P = 0;
  for (int v = 0; v < L.V; ++v) {
    const lv_camera& c = fr->cams_host[v];
    uint64_t tx = (uint64_t(c.width) + L.TS - 1) / L.TS;
    uint64_t ty = (uint64_t(c.height) + L.TS - 1) / L.TS;
    T += tx * ty;
    P += uint64_t(c.width) * uint64_t(c.height);
  }
  if (T * kSpread >= (1ull << 31)) return false;
  L.T = uint32_t(T);
  L.P = P;
  L.cap = st->pair_capacity;
  L.nblk_scan = uint32_t((T * kSpread + 1 + kScanBlock - 1) / kScanBlock);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  L.off_views = take(sizeof(ViewTab) * size_t(L.V));
  L.off_status = take(4 * S_WORDS);
  L.off_vox = take(sizeof(VoxRec) * size_t(L.n));
  L.off_rec = take(sizeof(Rec) * size_t(L.n) * size_t(L.V));
  L.off_tstart = take(4 * (size_t(L.T) * kSpread + 1));
  L.off_torder = take(4 * size_t(L.T + 1));
  L.off_nlast = take(4 * size_t(L.P));
  L.off_tpre = take(4 * size_t(L.P));
  L.off_ids = take(4 * size_t(L.cap));
  L.total_saved = o;
  o = 0;
  L.off_counters = take(4 * kCounterWords);
  L.off_tcount = take(4 * (size_t(L.T) * kSpread + 1));
  L.off_tfill = take(4 * (size_t(L.T) * kSpread + 1));
  L.off_bsum = take(8 * size_t(L.nblk_scan + 1));   // 64-bit block sums
  L.off_dcol = take(12 * size_t(L.n) * size_t(L.V));
  L.off_dden = take(32 * size_t(L.n));
  L.off_pairs = take(8 * size_t(L.cap));
  L.off_mtmp = take(8 * size_t(L.cap));
  L.total = o;
  return true;
}

// device pointers into the two buffers
struct WS {
  // saved
  ViewTab* views;
  uint32_t* status;
  VoxRec* vox;
  Rec* rec;
  uint32_t* tstart;
  uint32_t* torder;
  uint32_t* ids;
  uint32_t* nlast;
  float* tpre;
  // workspace
  uint32_t* counters;
  uint32_t* tcount;
  uint32_t* tfill;
  uint32_t* bsum;   // holds nblk_scan + 1 64-bit block sums
  float* dcol;   // [V][n][3] colour gradient per (view, voxel)
  float* dden;   // [n][8] corner-density gradient, voxel-major
  unsigned long long* pairs;
  unsigned long long* mtmp;
};

inline WS bind(const Layout& L, void* ws_base, void* saved_base) {
  char* b = static_cast<char*>(saved_base);
  WS w;
  w.views = reinterpret_cast<ViewTab*>(b + L.off_views);
  w.status = reinterpret_cast<uint32_t*>(b + L.off_status);
  w.vox = reinterpret_cast<VoxRec*>(b + L.off_vox);
  w.rec = reinterpret_cast<Rec*>(b + L.off_rec);
  w.tstart = reinterpret_cast<uint32_t*>(b + L.off_tstart);
  w.torder = reinterpret_cast<uint32_t*>(b + L.off_torder);
  w.ids = reinterpret_cast<uint32_t*>(b + L.off_ids);
  w.nlast = reinterpret_cast<uint32_t*>(b + L.off_nlast);
  w.tpre = reinterpret_cast<float*>(b + L.off_tpre);
  b = static_cast<char*>(ws_base);
  w.counters = reinterpret_cast<uint32_t*>(b + L.off_counters);
  w.tcount = reinterpret_cast<uint32_t*>(b + L.off_tcount);
  w.tfill = reinterpret_cast<uint32_t*>(b + L.off_tfill);
  w.bsum = reinterpret_cast<uint32_t*>(b + L.off_bsum);
  w.dcol = reinterpret_cast<float*>(b + L.off_dcol);
  w.dden = reinterpret_cast<float*>(b + L.off_dden);
  w.pairs = reinterpret_cast<unsigned long long*>(b + L.off_pairs);
  w.mtmp = reinterpret_cast<unsigned long long*>(b + L.off_mtmp);
  return w;
}

// constants of the pruning guards (cap = floor(cap_frac n), taken on the host)
struct GuardParams {
  float alpha, m_low, m_high, rho, w_keep;
  uint32_t cap;
};

// Everything the rasterizer kernels read, passed by value.
struct RasterArgs {
  WS ws;
  // voxels
  int64_t n;
  int deg;
  float root_min[3];
  float root_size;
  const uint16_t* ijk;
  const uint8_t* level;
  const float* density;
  const float* sh;
  const int32_t* corner_idx;   // grid-point layout, or null (dense)
  int64_t n_grid;
  int act;                     // LV_ACT_*
  // frame
  int V;
  const lv_camera* cams;
  float bg[3];
  // plan
  int TS;
  uint32_t T;
  uint64_t P;
  uint64_t cap;
  float t_eps;
  // outputs (forward) / inputs (backward)
  float* rgb;
  float* depth;
  float* alpha;
  float* wmax;
  const float* d_rgb;
  const float* d_depth;
  const float* d_alpha;
  // auxiliary channels (forward: written when non-null; backward: upstream
  // gradients, each nullable, and the forward's depth, needed with d_dist)
  float* dist;
  float* normal;
  float* mdepth;   // forward: median depth (no gradient flows through it)
  const float* d_dist;
  const float* d_normal;
  const float* depth_fwd;
  float* d_density;
  float* d_sh;
};

// ---------------------------------------------------------------- helpers
// Inter-ray spacing at voxel i's centre (the footprint of eq. 13-14): the
// minimum over views with z_c > 0 of z_c / fx, +inf if no view has the
// centre in front.  Binary32, one rounded operation at a time in the order
// written, so that the decisions taken on it are exact.
__device__ __forceinline__ float voxel_footprint(const RasterArgs& a, int64_t i) {
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
  return delta;
}

// Density activation applied to each stored value (LV_ACT_*) and its
// derivative.
__device__ __forceinline__ float density_act(float x, int act) {
  if (act == LV_ACT_SOFTPLUS) return x > 20.0f ? x : log1pf(expf(x));
  if (act == LV_ACT_EXP) return expf(x);
  return x;
}
__device__ __forceinline__ float density_act_grad(float x, int act) {
  if (act == LV_ACT_SOFTPLUS) return 1.0f / (1.0f + expf(-x));
  if (act == LV_ACT_EXP) return expf(x);
  return 1.0f;
}

// Stored value behind corner c of voxel i: its index into a.density, or -1
// when a grid index lies outside [0, n_grid) (the corner then reads 0).
__device__ __forceinline__ int64_t corner_slot(const RasterArgs& a, int c, int64_t i) {
  if (!a.corner_idx) return int64_t(c) * a.n + i;
  const int64_t g = a.corner_idx[int64_t(c) * a.n + i];
  return (g >= 0 && g < a.n_grid) ? g : int64_t(-1);
}

__device__ __forceinline__ float corner_density(const RasterArgs& a, int c, int64_t i) {
  const int64_t k = corner_slot(a, c, i);
  return k < 0 ? 0.0f : density_act(a.density[k], a.act);
}

// first pair of tile t (tile t + 1's start is its end), clipped to capacity
__device__ __forceinline__ uint64_t tile_begin(const RasterArgs& a, uint32_t t) {
  const uint64_t s = a.ws.tstart[uint64_t(t) * kSpread];
  return s < a.cap ? s : a.cap;
}

__device__ __forceinline__ int view_of_tile(const ViewTab* vt, int V, uint32_t gt) {
  int lo = 0, hi = V - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (vt[mid].tile_base <= gt) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Real orthonormal SH basis with the Condon-Shortley phase (polar axis z),
// Cartesian form, degree DEG <= 3; the constant term is replaced by 1 so that
// the first coefficient is a colour.
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = 1.0f;
  if (DEG >= 1) {
    const float c1 = 0.48860251190291992f;  // sqrt(3 / 4pi)
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
  }
  if (DEG >= 2) {
    const float c2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
    const float c20 = 0.31539156525252005f;  // sqrt(5 / pi) / 4
    const float c22 = 0.54627421529603959f;  // sqrt(15 / pi) / 4
    float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * (x * y);
    Y[5] = -c2a * (y * z);
    Y[6] = c20 * (3.0f * zz - 1.0f);
    Y[7] = -c2a * (x * z);
    Y[8] = c22 * (xx - yy);
    if (DEG >= 3) {
      const float c33 = 0.59004358992664352f;  // sqrt(35 / 2pi) / 4
      const float c32 = 2.8906114426405538f;   // sqrt(105 / pi) / 2
      const float c31 = 0.45704579946446572f;  // sqrt(21 / 2pi) / 4
      const float c30 = 0.37317633259011540f;  // sqrt(7 / pi) / 4
      const float c32b = 1.4453057213202769f;  // sqrt(105 / pi) / 4
      Y[9] = -c33 * y * (3.0f * xx - yy);
      Y[10] = c32 * (x * y) * z;
      Y[11] = -c31 * y * (5.0f * zz - 1.0f);
      Y[12] = c30 * z * (5.0f * zz - 3.0f);
      Y[13] = -c31 * x * (5.0f * zz - 1.0f);
      Y[14] = c32b * z * (xx - yy);
      Y[15] = -c33 * x * (xx - 3.0f * yy);
    }
  }
}

// ----------------------------------------------------------- launch helpers
// (defined in the kernel translation units)
hipError_t launch_setup(const RasterArgs& a, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
constexpr int kFillRanges = 4;
struct FillSet {   // word ranges filled by one launch
  uint32_t* p[kFillRanges];
  uint64_t n[kFillRanges];
  uint32_t v[kFillRanges];
  int count;
};
hipError_t launch_fill_set(const FillSet& f, hipStream_t s);
hipError_t launch_preprocess(const RasterArgs& a, hipStream_t s);
hipError_t run_aux_loss(const lv_camera* cams_host, const lv_camera* cams_dev, int V,
                        const float* depth, const float* alpha, const float* normal,
                        const float* dist, const float* mdepth, float lam_tc, float lam_n,
                        float lam_d, float lam_nm, float* loss, float* g_alpha, float* g_depth,
                        float* g_normal, float* g_dist, hipStream_t s);
hipError_t launch_count_records(const Rec* rec, uint64_t nrec, unsigned long long* out,
                                hipStream_t s);
hipError_t launch_scan_tiles(const RasterArgs& a, uint32_t nblk, hipStream_t s);
hipError_t launch_emit(const RasterArgs& a, hipStream_t s);
hipError_t launch_sort(const RasterArgs& a, hipStream_t s);
hipError_t launch_order(const RasterArgs& a, hipStream_t s);
hipError_t launch_composite_fwd(const RasterArgs& a, int chunk, int grid_cap, hipStream_t s,
                                bool aux = false);
hipError_t launch_bwd_setup(const RasterArgs& a, hipStream_t s);
hipError_t launch_composite_bwd(const RasterArgs& a, int chunk, int grid_cap, hipStream_t s,
                                bool aux = false);
hipError_t launch_sh_bwd(const RasterArgs& a, hipStream_t s);

}  // namespace lv

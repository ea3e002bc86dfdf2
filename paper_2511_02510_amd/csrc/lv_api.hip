// Host side of the C-ABI: argument validation, workspace planning, kernel
// orchestration on the caller's stream, graph capture, per-phase timing and
// the tile/chunk autotuner.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lv_common.h"
#include "lv_select.h"

namespace lv {
uint64_t loss_ws_bytes(int V);
uint64_t quant_ws_bytes(int64_t n, int B);
hipError_t run_lf_weight(const lv_camera* cams_dev, const lv_camera* cams_host, int V,
                         const float* target, float gamma, int form, float eps, float* weight,
                         void* ws, hipStream_t s);
hipError_t run_l1_grad(const lv_camera* cams_dev, int V, uint64_t max_pix, const float* rgb,
                       const float* target, const float* weight, float* loss, float* d_rgb,
                       hipStream_t s);
hipError_t run_depth_bins(const RasterArgs& a, int B, void* ws, uint8_t* out_bins, hipStream_t s);
hipError_t run_depth_cutoff(const RasterArgs& a, int B, double q, void* ws, float* tau,
                            uint8_t* prune, hipStream_t s);
uint64_t guard_ws_bytes(int64_t n);
uint64_t split_ws_bytes(int64_t n);
hipError_t run_footprint_range(const RasterArgs& a, void* ws, float* range, hipStream_t s);
hipError_t run_split_select(const RasterArgs& a, const float* score, const float* range,
                            const SplitParams& p, void* ws, uint8_t* split, float* priority,
                            uint32_t* n_split, hipStream_t s);
hipError_t run_split_apply(const RasterArgs& a, const uint8_t* split, int64_t m, void* ws,
                           uint16_t* ijk, uint8_t* level, float* density, float* sh,
                           uint64_t* needed, hipStream_t s);
hipError_t run_prune_guard(const RasterArgs& a, const uint8_t* bins, const float* tau, int nb,
                           const GuardParams& p, void* ws, float* ema, uint8_t* state,
                           uint8_t* prune, uint32_t* n_pruned, hipStream_t s);
}  // namespace lv

namespace {
// Static scratch of lv_lf_weight_noalloc: the loss-weight workspace of at
// most kNoAllocViews views (selection histograms and states, per-view weight
// sums), one copy per GPU, held until the process ends.  In host code the
// array's name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device by lv_create and kept in g_scratch_ptr.
constexpr int kNoAllocViews = LV_NOALLOC_MAX_VIEWS;
constexpr size_t kNoAllocBytes = 544 * 1024;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on hip_device (the current device), or NULL
void* scratch_address(int hip_device) {
  if (hip_device < 0 || hip_device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[hip_device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[hip_device] = ptr;
  }
  return g_scratch_ptr[hip_device];
}
}  // namespace

struct lv_context {
  int device = 0;
  void* scratch = nullptr;   // this device's copy of the static scratch
  std::string err;
  bool timing = false;
  bool capturing = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct Pending {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[LV_PH_COUNT] = {};
  int64_t calls[LV_PH_COUNT] = {};

  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

namespace {

lv_status fail(lv_context* ctx, lv_status s, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return s;
}

lv_status hip_fail(lv_context* ctx, hipError_t e, const char* where) {
  return fail(ctx, LV_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

struct PhaseTimer {
  lv_context* c;
  int ph;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  PhaseTimer(lv_context* ctx, int phase, hipStream_t st) : c(ctx), ph(phase), s(st) {
    if (c && c->timing && !c->capturing) {
      a = c->event();
      b = c->event();
      if (!(a && b && hipEventRecord(a, s) == hipSuccess)) a = b = nullptr;
    }
  }
  ~PhaseTimer() {
    if (a && hipEventRecord(b, s) == hipSuccess) c->pending.push_back({ph, a, b});
  }
};

bool finite_pos(float x) { return std::isfinite(x) && x > 0.0f; }

lv_status check_frame(lv_context* ctx, const lv_frame* fr) {
  if (!fr) return fail(ctx, LV_ERR_ARG, "frame is NULL");
  if (fr->n_views < 1 || fr->n_views > LV_MAX_VIEWS)
    return fail(ctx, LV_ERR_ARG, "n_views=%d outside [1, %d]", fr->n_views, LV_MAX_VIEWS);
  if (!fr->cams_host || !fr->cams_dev) return fail(ctx, LV_ERR_ARG, "camera arrays must be non-NULL");
  for (int v = 0; v < fr->n_views; ++v) {
    const lv_camera& c = fr->cams_host[v];
    if (c.width < 1 || c.height < 1 || c.width > 32767 || c.height > 32767)
      return fail(ctx, LV_ERR_ARG, "view %d: size %dx%d outside [1, 32767]", v, c.width, c.height);
    if (!finite_pos(c.fx) || !finite_pos(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
      return fail(ctx, LV_ERR_ARG, "view %d: invalid intrinsics", v);
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(c.R[k])) return fail(ctx, LV_ERR_ARG, "view %d: non-finite R", v);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(c.o[k])) return fail(ctx, LV_ERR_ARG, "view %d: non-finite centre", v);
  }
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(fr->bg[k])) return fail(ctx, LV_ERR_ARG, "non-finite background");
  return LV_OK;
}

lv_status check_voxels(lv_context* ctx, const lv_voxels* vx, bool need_params) {
  if (!vx) return fail(ctx, LV_ERR_ARG, "voxels is NULL");
  if (vx->n < 0 || vx->n >= (int64_t(1) << lv::kIdBits))
    return fail(ctx, LV_ERR_ARG, "n=%lld outside [0, 2^28)", (long long)vx->n);
  if (vx->sh_degree < 0 || vx->sh_degree > 3)
    return fail(ctx, LV_ERR_ARG, "sh_degree=%d outside [0, 3]", vx->sh_degree);
  if (!finite_pos(vx->root_size)) return fail(ctx, LV_ERR_ARG, "root_size must be finite and > 0");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(vx->root_min[k])) return fail(ctx, LV_ERR_ARG, "non-finite root_min");
  if (vx->density_act < LV_ACT_NONE || vx->density_act > LV_ACT_EXP)
    return fail(ctx, LV_ERR_ARG, "density_act=%d is not an LV_ACT_* value", vx->density_act);
  if (vx->corner_idx && (vx->n_grid < 0 || vx->n_grid > int64_t(0x7FFFFFFF)))
    return fail(ctx, LV_ERR_ARG, "n_grid=%lld outside [0, 2^31)", (long long)vx->n_grid);
  if (vx->n > 0) {
    if (!vx->ijk || !vx->level) return fail(ctx, LV_ERR_ARG, "ijk/level must be non-NULL");
    if (need_params && (!vx->sh || (!vx->density && (!vx->corner_idx || vx->n_grid > 0))))
      return fail(ctx, LV_ERR_ARG, "density/sh must be non-NULL");
  }
  return LV_OK;
}

lv_status check_settings(lv_context* ctx, const lv_settings* st) {
  if (!st) return fail(ctx, LV_ERR_ARG, "settings is NULL");
  if (st->tile != 8 && st->tile != 16 && st->tile != 32)
    return fail(ctx, LV_ERR_ARG, "tile=%d not in {8, 16, 32}", st->tile);
  if (st->chunk != 64 && st->chunk != 128 && st->chunk != 256)
    return fail(ctx, LV_ERR_ARG, "chunk=%d not in {64, 128, 256}", st->chunk);
  if (st->chunk_bwd != 0 && st->chunk_bwd != 64 && st->chunk_bwd != 128 && st->chunk_bwd != 256)
    return fail(ctx, LV_ERR_ARG, "chunk_bwd=%d not in {0, 64, 128, 256}", st->chunk_bwd);
  if (!(st->t_eps > 0.0f) || !(st->t_eps <= 1e-5f))
    return fail(ctx, LV_ERR_ARG, "t_eps=%g outside (0, 1e-5]", double(st->t_eps));
  if (st->pair_capacity >= (uint64_t(1) << 32))
    return fail(ctx, LV_ERR_ARG, "pair_capacity must be < 2^32");
  return LV_OK;
}

lv_status validate_all(lv_context* ctx, const lv_voxels* vx, const lv_frame* fr,
                       const lv_settings* st, lv::Layout* L) {
  lv_status s = check_voxels(ctx, vx, true);
  if (s != LV_OK) return s;
  if ((s = check_frame(ctx, fr)) != LV_OK) return s;
  if ((s = check_settings(ctx, st)) != LV_OK) return s;
  lv::Layout tmp;
  if (!lv::make_layout(vx, fr, st, L ? *L : tmp))
    return fail(ctx, LV_ERR_ARG, "too many tiles for these views and tile size");
  return LV_OK;
}

// saved: the forward's kept state (NULL for calls that use only a workspace)
lv::RasterArgs make_args(const lv::Layout& L, void* ws, const void* saved, const lv_voxels* vx,
                         const lv_frame* fr, const lv_settings* st) {
  lv::RasterArgs a;
  std::memset(&a, 0, sizeof(a));
  a.ws = lv::bind(L, ws, saved ? const_cast<void*>(saved) : ws);
  a.n = vx->n;
  a.deg = vx->sh_degree;
  for (int k = 0; k < 3; ++k) a.root_min[k] = vx->root_min[k];
  a.root_size = vx->root_size;
  a.ijk = vx->ijk;
  a.level = vx->level;
  a.density = vx->density;
  a.sh = vx->sh;
  a.corner_idx = vx->corner_idx;
  a.n_grid = vx->corner_idx ? vx->n_grid : 0;
  a.act = vx->density_act;
  if (fr) {   // calls that need no views pass none
    a.V = fr->n_views;
    a.cams = fr->cams_dev;
    for (int k = 0; k < 3; ++k) a.bg[k] = fr->bg[k];
  }
  a.TS = L.TS;
  a.T = L.T;
  a.P = L.P;
  a.cap = L.cap;
  a.t_eps = st ? st->t_eps : 1e-6f;
  return a;
}

#define LV_TRY(expr, where)                          \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
  } while (0)

}  // namespace

extern "C" {

const char* lv_status_str(lv_status s) {
  switch (s) {
    case LV_OK: return "ok";
    case LV_ERR_ARG: return "invalid argument";
    case LV_ERR_HIP: return "HIP runtime error";
    case LV_ERR_CAPACITY: return "pair capacity exceeded";
    case LV_ERR_UNSUPPORTED: return "unsupported";
    case LV_ERR_STATE: return "invalid call order";
  }
  return "unknown status";
}

const char* lv_last_error(const lv_context* ctx) { return ctx ? ctx->err.c_str() : ""; }

void lv_default_settings(lv_settings* s) {
  if (!s) return;
  s->tile = 16;
  s->chunk = 64;
  s->chunk_bwd = 0;
  s->t_eps = 1e-6f;
  s->pair_capacity = 0;
}

lv_status lv_create(lv_context** out, int hip_device) {
  if (!out) return LV_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return LV_ERR_HIP;
  if (hip_device < 0 || hip_device >= count) return LV_ERR_ARG;
  if (hipSetDevice(hip_device) != hipSuccess) return LV_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return LV_ERR_HIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LV_ERR_UNSUPPORTED;
  lv_context* c = new lv_context();
  c->device = hip_device;
  c->scratch = scratch_address(hip_device);   // the device is current here
  *out = c;
  return LV_OK;
}

void lv_destroy(lv_context* ctx) {
  if (!ctx) return;
  if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  for (auto& p : ctx->pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  delete ctx;
}

lv_status lv_validate(const lv_voxels* vox, const lv_frame* frame, const lv_settings* st) {
  return validate_all(nullptr, vox, frame, st, nullptr);
}

lv_status lv_query_sizes(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                         const lv_settings* st, uint64_t* workspace_bytes, uint64_t* saved_bytes) {
  if (!workspace_bytes || !saved_bytes)
    return fail(ctx, LV_ERR_ARG, "workspace_bytes/saved_bytes is NULL");
  lv::Layout L;
  lv_status s = validate_all(ctx, vox, frame, st, &L);
  if (s != LV_OK) return s;
  *workspace_bytes = L.total;
  *saved_bytes = L.total_saved;
  return LV_OK;
}

static lv_status forward_impl(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                              const lv_settings* st, void* workspace, void* saved, float* rgb,
                              float* depth, float* alpha, float* wmax, bool aux, float* dist,
                              float* normal, float* mdepth, hipStream_t stream);

lv_status lv_forward(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                     const lv_settings* st, void* workspace, void* saved, float* rgb, float* depth,
                     float* alpha, float* wmax, hipStream_t stream) {
  return forward_impl(ctx, vox, frame, st, workspace, saved, rgb, depth, alpha, wmax, false,
                      nullptr, nullptr, nullptr, stream);
}

lv_status lv_forward_aux(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                         const lv_settings* st, void* workspace, void* saved, float* rgb,
                         float* depth, float* alpha, float* wmax, float* dist, float* normal,
                         float* mdepth, hipStream_t stream) {
  return forward_impl(ctx, vox, frame, st, workspace, saved, rgb, depth, alpha, wmax, true, dist,
                      normal, mdepth, stream);
}

static lv_status forward_impl(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                              const lv_settings* st, void* workspace, void* saved, float* rgb,
                              float* depth, float* alpha, float* wmax, bool aux, float* dist,
                              float* normal, float* mdepth, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv::Layout L;
  lv_status s = validate_all(ctx, vox, frame, st, &L);
  if (s != LV_OK) return s;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(ctx, LV_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (!saved || (reinterpret_cast<uintptr_t>(saved) & 255))
    return fail(ctx, LV_ERR_ARG, "saved must be non-NULL and 256-byte aligned");
  if (!rgb || !depth || !alpha) return fail(ctx, LV_ERR_ARG, "rgb/depth/alpha must be non-NULL");
  if (vox->n > 0 && !wmax) return fail(ctx, LV_ERR_ARG, "wmax must be non-NULL");
  lv::RasterArgs a = make_args(L, workspace, saved, vox, frame, st);
  a.rgb = rgb;
  a.depth = depth;
  a.alpha = alpha;
  a.wmax = wmax;
  a.dist = dist;
  a.normal = normal;
  a.mdepth = mdepth;
  {
    PhaseTimer t(ctx, LV_PH_SETUP, stream);
    LV_TRY(lv::launch_setup(a, stream), "setup");   // also zeroes the tile counts
  }
  {
    PhaseTimer t(ctx, LV_PH_PREPROCESS, stream);
    LV_TRY(lv::launch_preprocess(a, stream), "preprocess");
  }
  {
    PhaseTimer t(ctx, LV_PH_SCAN, stream);
    LV_TRY(lv::launch_scan_tiles(a, L.nblk_scan, stream), "scan");
  }
  {
    PhaseTimer t(ctx, LV_PH_EMIT, stream);
    LV_TRY(lv::launch_emit(a, stream), "emit");
  }
  {
    PhaseTimer t(ctx, LV_PH_ORDER, stream);
    LV_TRY(lv::launch_order(a, stream), "order");
  }
  {
    PhaseTimer t(ctx, LV_PH_SORT, stream);
    LV_TRY(lv::launch_sort(a, stream), "sort");
  }
  {
    PhaseTimer t(ctx, LV_PH_COMPOSITE_FWD, stream);
    LV_TRY(lv::launch_composite_fwd(a, st->chunk, 0, stream, aux), "composite forward");
  }
  return LV_OK;
}

static lv_status backward_impl(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                               const lv_settings* st, void* workspace, const void* saved,
                               const float* d_rgb, const float* d_depth, const float* d_alpha,
                               const float* depth_fwd, const float* d_dist,
                               const float* d_normal, float* d_density, float* d_sh,
                               hipStream_t stream);

lv_status lv_backward(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                      const lv_settings* st, void* workspace, const void* saved,
                      const float* d_rgb, const float* d_depth, const float* d_alpha,
                      float* d_density, float* d_sh, hipStream_t stream) {
  return backward_impl(ctx, vox, frame, st, workspace, saved, d_rgb, d_depth, d_alpha, nullptr,
                       nullptr, nullptr, d_density, d_sh, stream);
}

lv_status lv_backward_aux(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                          const lv_settings* st, void* workspace, const void* saved,
                          const float* d_rgb, const float* d_depth, const float* d_alpha,
                          const float* depth_fwd, const float* d_dist, const float* d_normal,
                          float* d_density, float* d_sh, hipStream_t stream) {
  if (ctx && d_dist && !depth_fwd)
    return fail(ctx, LV_ERR_ARG, "d_dist needs depth_fwd (the depth of the forward pass)");
  return backward_impl(ctx, vox, frame, st, workspace, saved, d_rgb, d_depth, d_alpha, depth_fwd,
                       d_dist, d_normal, d_density, d_sh, stream);
}

static lv_status backward_impl(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                               const lv_settings* st, void* workspace, const void* saved,
                               const float* d_rgb, const float* d_depth, const float* d_alpha,
                               const float* depth_fwd, const float* d_dist,
                               const float* d_normal, float* d_density, float* d_sh,
                               hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv::Layout L;
  lv_status s = validate_all(ctx, vox, frame, st, &L);
  if (s != LV_OK) return s;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(ctx, LV_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (!saved || (reinterpret_cast<uintptr_t>(saved) & 255))
    return fail(ctx, LV_ERR_ARG, "saved must be non-NULL and 256-byte aligned");
  if (!d_rgb) return fail(ctx, LV_ERR_ARG, "d_rgb must be non-NULL");
  if (vox->n > 0 && (!d_density || !d_sh))
    return fail(ctx, LV_ERR_ARG, "d_density/d_sh must be non-NULL");
  lv::RasterArgs a = make_args(L, workspace, saved, vox, frame, st);
  a.d_rgb = d_rgb;
  a.d_depth = d_depth;
  a.d_alpha = d_alpha;
  a.d_density = d_density;
  a.d_sh = d_sh;
  a.d_dist = d_dist;
  a.d_normal = d_normal;
  a.depth_fwd = depth_fwd;
  const bool aux = d_dist || d_normal;
  {
    PhaseTimer t(ctx, LV_PH_BWD_SETUP, stream);
    LV_TRY(lv::launch_bwd_setup(a, stream), "backward setup");
  }
  {
    PhaseTimer t(ctx, LV_PH_COMPOSITE_BWD, stream);
    LV_TRY(lv::launch_composite_bwd(a, st->chunk_bwd ? st->chunk_bwd : st->chunk, 0, stream, aux),
           "composite backward");
  }
  {
    PhaseTimer t(ctx, LV_PH_SH_BWD, stream);
    LV_TRY(lv::launch_sh_bwd(a, stream), "sh backward");
  }
  return LV_OK;
}

lv_status lv_check_overflow(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                            const lv_settings* st, const void* saved, uint64_t* pairs_needed,
                            hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv::Layout L;
  lv_status s = validate_all(ctx, vox, frame, st, &L);
  if (s != LV_OK) return s;
  if (!saved) return fail(ctx, LV_ERR_ARG, "saved is NULL");
  LV_TRY(hipStreamSynchronize(stream), "synchronize");
  uint32_t c[2] = {0, 0};
  const char* base = static_cast<const char*>(saved) + L.off_status;
  LV_TRY(hipMemcpy(c, base, sizeof(c), hipMemcpyDeviceToHost), "read status");
  if (pairs_needed) *pairs_needed = c[lv::S_PAIRS];
  if (c[lv::S_OVERFLOW]) {
    return fail(ctx, LV_ERR_CAPACITY, "%u (tile, voxel) pairs needed, capacity %llu",
                c[lv::S_PAIRS], (unsigned long long)L.cap);
  }
  return LV_OK;
}

lv_status lv_pass_stats(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                        const lv_settings* st, const void* saved, uint64_t* pairs,
                        uint64_t* records, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv::Layout L;
  lv_status s = validate_all(ctx, vox, frame, st, &L);
  if (s != LV_OK) return s;
  if (!saved) return fail(ctx, LV_ERR_ARG, "saved is NULL");
  LV_TRY(hipStreamSynchronize(stream), "synchronize");
  uint32_t w[lv::S_WORDS] = {};
  LV_TRY(hipMemcpy(w, static_cast<const char*>(saved) + L.off_status, sizeof(w),
                   hipMemcpyDeviceToHost), "read status");
  if (pairs) *pairs = w[lv::S_PAIRS];
  if (records) {
    // counted on demand (a diagnostic call, outside any captured sequence)
    unsigned long long* cnt = nullptr;
    LV_TRY(hipMalloc(&cnt, sizeof(*cnt)), "record counter");
    unsigned long long h = 0;
    hipError_t e = hipMemsetAsync(cnt, 0, sizeof(*cnt), stream);
    if (e == hipSuccess)
      e = lv::launch_count_records(reinterpret_cast<const lv::Rec*>(
                                       static_cast<const char*>(saved) + L.off_rec),
                                   uint64_t(L.n) * uint64_t(L.V), cnt, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(&h, cnt, sizeof(h), hipMemcpyDeviceToHost);
    (void)hipFree(cnt);
    LV_TRY(e, "count records");
    *records = h;
  }
  return LV_OK;
}

lv_status lv_export_bins(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                         const lv_settings* st, const void* saved, uint32_t* tile_start,
                         uint32_t* ids, uint64_t* codes, int32_t* rects, uint8_t* vis,
                         hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv::Layout L;
  lv_status s = validate_all(ctx, vox, frame, st, &L);
  if (s != LV_OK) return s;
  if (!saved) return fail(ctx, LV_ERR_ARG, "saved is NULL");
  LV_TRY(hipStreamSynchronize(stream), "synchronize");
  const char* base = static_cast<const char*>(saved);
  std::vector<uint32_t> sub(size_t(L.T) * lv::kSpread + 1);
  LV_TRY(hipMemcpy(sub.data(), base + L.off_tstart, 4 * sub.size(), hipMemcpyDeviceToHost), "tile_start");
  std::vector<uint32_t> ts(size_t(L.T) + 1);
  for (size_t t = 0; t <= L.T; ++t) ts[t] = sub[t * lv::kSpread];
  if (tile_start) std::memcpy(tile_start, ts.data(), 4 * ts.size());
  const uint64_t tot = std::min<uint64_t>(ts[L.T], L.cap);
  if (ids && tot) LV_TRY(hipMemcpy(ids, base + L.off_ids, 4 * tot, hipMemcpyDeviceToHost), "ids");
  if (codes || rects || vis) {
    const size_t nr = size_t(L.n) * size_t(L.V);
    std::vector<lv::Rec> rec(nr);
    if (nr) LV_TRY(hipMemcpy(rec.data(), base + L.off_rec, sizeof(lv::Rec) * nr, hipMemcpyDeviceToHost), "records");
    for (size_t r = 0; r < nr; ++r) {
      const bool on = (rec[r].flags & 8u) != 0;
      if (vis) vis[r] = on ? 1 : 0;
      if (codes) codes[r] = on ? (uint64_t(rec[r].code_hi) << 32 | rec[r].code_lo) : 0;
      if (rects) {
        rects[4 * r + 0] = on ? int32_t(rec[r].xr & 0xFFFFu) : 0;
        rects[4 * r + 1] = on ? int32_t(rec[r].xr >> 16) : 0;
        rects[4 * r + 2] = on ? int32_t(rec[r].yr & 0xFFFFu) : 0;
        rects[4 * r + 3] = on ? int32_t(rec[r].yr >> 16) : 0;
      }
    }
  }
  return LV_OK;
}

uint64_t lv_lf_weight_workspace_size(int32_t n_views) {
  return n_views > 0 ? lv::loss_ws_bytes(n_views) : 0;
}

static uint64_t max_view_pixels(const lv_frame* fr) {
  uint64_t m = 0;
  for (int v = 0; v < fr->n_views; ++v)
    m = std::max<uint64_t>(m, uint64_t(fr->cams_host[v].width) * uint64_t(fr->cams_host[v].height));
  return m;
}

lv_status lv_lf_weight(lv_context* ctx, const lv_frame* frame, const float* target, float gamma,
                       int32_t form, float eps, float* weight, void* workspace, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_frame(ctx, frame);
  if (s != LV_OK) return s;
  if (!target || !weight || !workspace) return fail(ctx, LV_ERR_ARG, "target/weight/workspace NULL");
  if (form != 0 && form != 1) return fail(ctx, LV_ERR_ARG, "form must be 0 or 1");
  if (!std::isfinite(gamma) || !std::isfinite(eps) || eps < 0.0f)
    return fail(ctx, LV_ERR_ARG, "gamma must be finite and eps >= 0");
  LV_TRY(lv::run_lf_weight(frame->cams_dev, frame->cams_host, frame->n_views, target, gamma, form,
                           eps, weight, workspace, stream), "lf_weight");
  return LV_OK;
}

lv_status lv_lf_weight_noalloc(lv_context* ctx, const lv_frame* frame, const float* target,
                               float gamma, int32_t form, float eps, float* weight,
                               hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_frame(ctx, frame);
  if (s != LV_OK) return s;
  if (frame->n_views > kNoAllocViews)
    return fail(ctx, LV_ERR_ARG,
                "n_views=%d exceeds the %d views the static scratch holds (use lv_lf_weight)",
                frame->n_views, kNoAllocViews);
  if (!target || !weight) return fail(ctx, LV_ERR_ARG, "target/weight NULL");
  if (form != 0 && form != 1) return fail(ctx, LV_ERR_ARG, "form must be 0 or 1");
  if (!std::isfinite(gamma) || !std::isfinite(eps) || eps < 0.0f)
    return fail(ctx, LV_ERR_ARG, "gamma must be finite and eps >= 0");
  if (lv::loss_ws_bytes(frame->n_views) > kNoAllocBytes)
    return fail(ctx, LV_ERR_UNSUPPORTED, "static scratch smaller than the loss workspace");
  int dev = -1;
  LV_TRY(hipGetDevice(&dev), "current device");
  if (dev != ctx->device)
    return fail(ctx, LV_ERR_STATE, "current device %d is not the context's device %d", dev,
                ctx->device);
  if (!ctx->scratch) return fail(ctx, LV_ERR_HIP, "static scratch address unavailable");
  LV_TRY(lv::run_lf_weight(frame->cams_dev, frame->cams_host, frame->n_views, target, gamma, form,
                           eps, weight, ctx->scratch, stream), "lf_weight_noalloc");
  return LV_OK;
}

lv_status lv_l1_grad(lv_context* ctx, const lv_frame* frame, const float* rgb, const float* target,
                     const float* weight, float* loss, float* d_rgb, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_frame(ctx, frame);
  if (s != LV_OK) return s;
  if (!rgb || !target || !weight || !loss || !d_rgb)
    return fail(ctx, LV_ERR_ARG, "rgb/target/weight/loss/d_rgb must be non-NULL");
  LV_TRY(lv::run_l1_grad(frame->cams_dev, frame->n_views, max_view_pixels(frame), rgb, target,
                         weight, loss, d_rgb, stream), "l1_grad");
  return LV_OK;
}

lv_status lv_aux_loss(lv_context* ctx, const lv_frame* frame, const float* depth,
                      const float* alpha, const float* normal, const float* dist,
                      const float* mdepth, float lam_tc, float lam_n, float lam_d, float lam_nm,
                      float* loss, float* d_alpha, float* d_depth, float* d_normal, float* d_dist,
                      hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_frame(ctx, frame);
  if (s != LV_OK) return s;
  if (!depth || !alpha || !normal || !dist || !loss || !d_alpha || !d_depth || !d_normal ||
      !d_dist)
    return fail(ctx, LV_ERR_ARG, "lv_aux_loss: every pointer but mdepth must be non-NULL");
  if (lam_nm != 0.0f && !mdepth)
    return fail(ctx, LV_ERR_ARG, "lv_aux_loss: the median term needs mdepth");
  LV_TRY(lv::run_aux_loss(frame->cams_host, frame->cams_dev, frame->n_views, depth, alpha,
                          normal, dist, lam_nm != 0.0f ? mdepth : nullptr, lam_tc, lam_n, lam_d,
                          lam_nm, loss, d_alpha, d_depth, d_normal, d_dist, stream),
         "aux_loss");
  return LV_OK;
}

float lv_gamma_schedule(float t, float total, float t0_frac, float t1_frac, float gamma_max) {
  const float t0 = t0_frac * total, t1 = t1_frac * total;
  if (t < t0) return 0.0f;
  if (t < t1) return gamma_max * (t - t0) / (t1 - t0);
  return gamma_max;
}

uint64_t lv_quantile_workspace_size(int64_t n, int32_t n_bins) {
  if (n < 0 || n_bins < 1 || n_bins > 64) return 0;
  return lv::quant_ws_bytes(n, n_bins);
}

lv_status lv_depth_bins(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                        int32_t n_bins, void* workspace, uint8_t* bins, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_voxels(ctx, vox, false);
  if (s != LV_OK) return s;
  if ((s = check_frame(ctx, frame)) != LV_OK) return s;
  if (n_bins < 1 || n_bins > 64) return fail(ctx, LV_ERR_ARG, "n_bins must be in [1, 64]");
  if (!workspace) return fail(ctx, LV_ERR_ARG, "workspace must be non-NULL");
  lv::Layout L;
  lv::RasterArgs a = make_args(L, workspace, nullptr, vox, frame, nullptr);
  LV_TRY(lv::run_depth_bins(a, n_bins, workspace, bins, stream), "depth_bins");
  return LV_OK;
}

lv_status lv_depth_cutoff(lv_context* ctx, const lv_voxels* vox, const float* wmax, int32_t n_bins,
                          double q, void* workspace, float* tau, uint8_t* prune, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_voxels(ctx, vox, false);
  if (s != LV_OK) return s;
  if (n_bins < 1 || n_bins > 64) return fail(ctx, LV_ERR_ARG, "n_bins must be in [1, 64]");
  if (!(q > 0.0 && q <= 1.0)) return fail(ctx, LV_ERR_ARG, "q must be in (0, 1]");
  if (!workspace || !tau || (vox->n > 0 && (!wmax || !prune)))
    return fail(ctx, LV_ERR_ARG, "workspace/tau/wmax/prune must be non-NULL");
  lv::Layout L;
  lv::RasterArgs a = make_args(L, workspace, nullptr, vox, nullptr, nullptr);
  a.wmax = const_cast<float*>(wmax);
  LV_TRY(lv::run_depth_cutoff(a, n_bins, q, workspace, tau, prune, stream), "depth_cutoff");
  return LV_OK;
}

lv_status lv_depth_quantile(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                            const float* wmax, int32_t n_bins, double q, void* workspace,
                            float* tau, uint8_t* prune, uint8_t* bins, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_voxels(ctx, vox, false);
  if (s != LV_OK) return s;
  if ((s = check_frame(ctx, frame)) != LV_OK) return s;
  if (n_bins < 1 || n_bins > 64) return fail(ctx, LV_ERR_ARG, "n_bins must be in [1, 64]");
  if (!(q > 0.0 && q <= 1.0)) return fail(ctx, LV_ERR_ARG, "q must be in (0, 1]");
  if (!workspace || !tau || (vox->n > 0 && (!wmax || !prune)))
    return fail(ctx, LV_ERR_ARG, "workspace/tau/wmax/prune must be non-NULL");
  if ((s = lv_depth_bins(ctx, vox, frame, n_bins, workspace, bins, stream)) != LV_OK) return s;
  return lv_depth_cutoff(ctx, vox, wmax, n_bins, q, workspace, tau, prune, stream);
}

void lv_default_guard(lv_guard_params* p) {
  if (!p) return;
  p->alpha = 0.3f;
  p->m_low = 0.3f;
  p->m_high = 0.7f;
  p->rho = 0.25f;
  p->w_keep = 0.5f;
  p->cap_frac = 0.05;
}

uint64_t lv_guard_workspace_size(int64_t n) {
  if (n < 0) return 0;
  return lv::guard_ws_bytes(n);
}

lv_status lv_prune_guard(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                         const float* wmax, const uint8_t* bins, const float* tau, int32_t n_bins,
                         const lv_guard_params* params, void* workspace, float* ema,
                         uint8_t* state, uint8_t* prune, uint32_t* n_pruned, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_voxels(ctx, vox, false);
  if (s != LV_OK) return s;
  if ((s = check_frame(ctx, frame)) != LV_OK) return s;
  if (!params) return fail(ctx, LV_ERR_ARG, "params must be non-NULL");
  const lv_guard_params& g = *params;
  if (n_bins < 1 || n_bins > 64) return fail(ctx, LV_ERR_ARG, "n_bins must be in [1, 64]");
  if (!(g.alpha > 0.0f && g.alpha <= 1.0f)) return fail(ctx, LV_ERR_ARG, "alpha must be in (0, 1]");
  if (!(g.m_low <= g.m_high)) return fail(ctx, LV_ERR_ARG, "m_low must not exceed m_high");
  if (!(g.rho >= 0.0f)) return fail(ctx, LV_ERR_ARG, "rho must be >= 0");
  if (!(g.cap_frac >= 0.0 && g.cap_frac <= 1.0)) return fail(ctx, LV_ERR_ARG, "cap_frac must be in [0, 1]");
  if (!workspace || (vox->n > 0 && (!wmax || !bins || !tau || !ema || !state || !prune)))
    return fail(ctx, LV_ERR_ARG, "workspace/wmax/bins/tau/ema/state/prune must be non-NULL");
  if (vox->n > int64_t(0x7FFFFFFF)) return fail(ctx, LV_ERR_ARG, "n must be below 2^31");
  lv::Layout L;
  lv::RasterArgs a = make_args(L, workspace, nullptr, vox, frame, nullptr);
  a.wmax = const_cast<float*>(wmax);
  lv::GuardParams p;
  p.alpha = g.alpha;
  p.m_low = g.m_low;
  p.m_high = g.m_high;
  p.rho = g.rho;
  p.w_keep = g.w_keep;
  p.cap = uint32_t(std::floor(g.cap_frac * double(vox->n)));
  LV_TRY(lv::run_prune_guard(a, bins, tau, n_bins, p, workspace, ema, state, prune, n_pruned, stream),
         "prune_guard");
  return LV_OK;
}

void lv_default_split(lv_split_params* p) {
  if (!p) return;
  p->kappa = 1.0f;
  p->beta = 0.2f;
  p->max_splits = 8192u;
}

uint64_t lv_split_workspace_size(int64_t n) {
  if (n < 0) return 0;
  return lv::split_ws_bytes(n);
}

lv_status lv_footprint_range(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                             void* workspace, float* range, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_voxels(ctx, vox, false);
  if (s != LV_OK) return s;
  if ((s = check_frame(ctx, frame)) != LV_OK) return s;
  if (!workspace || !range) return fail(ctx, LV_ERR_ARG, "workspace/range must be non-NULL");
  lv::Layout L;
  lv::RasterArgs a = make_args(L, workspace, nullptr, vox, frame, nullptr);
  LV_TRY(lv::run_footprint_range(a, workspace, range, stream), "footprint_range");
  return LV_OK;
}

lv_status lv_subdivide_select(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                              const float* score, const float* range, const lv_split_params* params,
                              void* workspace, uint8_t* split, float* priority, uint32_t* n_split,
                              hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_voxels(ctx, vox, false);
  if (s != LV_OK) return s;
  if ((s = check_frame(ctx, frame)) != LV_OK) return s;
  if (!params) return fail(ctx, LV_ERR_ARG, "params must be non-NULL");
  if (!(std::isfinite(params->kappa) && params->kappa >= 0.0f))
    return fail(ctx, LV_ERR_ARG, "kappa must be finite and >= 0");
  if (!(std::isfinite(params->beta) && params->beta >= 0.0f))
    return fail(ctx, LV_ERR_ARG, "beta must be finite and >= 0");
  if (!workspace || (vox->n > 0 && (!score || !range || !split)))
    return fail(ctx, LV_ERR_ARG, "workspace/score/range/split must be non-NULL");
  lv::Layout L;
  lv::RasterArgs a = make_args(L, workspace, nullptr, vox, frame, nullptr);
  lv::SplitParams p;
  p.kappa = params->kappa;
  p.beta = params->beta;
  p.max_splits = params->max_splits;
  LV_TRY(lv::run_split_select(a, score, range, p, workspace, split, priority, n_split, stream),
         "subdivide_select");
  return LV_OK;
}

lv_status lv_subdivide_apply(lv_context* ctx, const lv_voxels* vox, const uint8_t* split,
                             int64_t n_out, void* workspace, uint16_t* ijk, uint8_t* level,
                             float* density, float* sh, uint64_t* n_needed, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  lv_status s = check_voxels(ctx, vox, true);
  if (s != LV_OK) return s;
  if (vox->corner_idx)
    return fail(ctx, LV_ERR_UNSUPPORTED, "subdivision needs the dense corner layout");
  if (n_out < vox->n || n_out > 8 * vox->n)
    return fail(ctx, LV_ERR_ARG, "n_out must lie in [n, 8 n]");
  if (!workspace || (vox->n > 0 && (!split || !ijk || !level || !density || !sh)))
    return fail(ctx, LV_ERR_ARG, "workspace/split/ijk/level/density/sh must be non-NULL");
  lv::Layout L;
  lv::RasterArgs a = make_args(L, workspace, nullptr, vox, nullptr, nullptr);
  LV_TRY(lv::run_split_apply(a, split, n_out, workspace, ijk, level, density, sh, n_needed, stream),
         "subdivide_apply");
  return LV_OK;
}

lv_status lv_graph_begin(lv_context* ctx, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  if (ctx->capturing) return fail(ctx, LV_ERR_STATE, "already capturing");
  if (stream == nullptr) return fail(ctx, LV_ERR_ARG, "cannot capture the null stream");
  LV_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed), "begin capture");
  ctx->capturing = true;
  return LV_OK;
}

lv_status lv_graph_end(lv_context* ctx, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  if (!ctx->capturing) return fail(ctx, LV_ERR_STATE, "not capturing");
  ctx->capturing = false;
  hipGraph_t g = nullptr;
  LV_TRY(hipStreamEndCapture(stream, &g), "end capture");
  if (ctx->exec) { (void)hipGraphExecDestroy(ctx->exec); ctx->exec = nullptr; }
  if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
  ctx->graph = g;
  LV_TRY(hipGraphInstantiate(&ctx->exec, g, nullptr, nullptr, 0), "instantiate graph");
  return LV_OK;
}

lv_status lv_graph_launch(lv_context* ctx, hipStream_t stream) {
  if (!ctx) return LV_ERR_ARG;
  if (!ctx->exec) return fail(ctx, LV_ERR_STATE, "no captured graph");
  LV_TRY(hipGraphLaunch(ctx->exec, stream), "graph launch");
  return LV_OK;
}

lv_status lv_graph_reset(lv_context* ctx) {
  if (!ctx) return LV_ERR_ARG;
  if (ctx->exec) { (void)hipGraphExecDestroy(ctx->exec); ctx->exec = nullptr; }
  if (ctx->graph) { (void)hipGraphDestroy(ctx->graph); ctx->graph = nullptr; }
  return LV_OK;
}

lv_status lv_set_timing(lv_context* ctx, int32_t enable) {
  if (!ctx) return LV_ERR_ARG;
  ctx->timing = enable != 0;
  return LV_OK;
}

lv_status lv_read_timings(lv_context* ctx, double* ms, int64_t* calls) {
  if (!ctx) return LV_ERR_ARG;
  for (auto& p : ctx->pending) {
    if (hipEventSynchronize(p.b) != hipSuccess) return fail(ctx, LV_ERR_HIP, "event sync");
    float t = 0.0f;
    if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      ctx->ms[p.phase] += t;
      ctx->calls[p.phase] += 1;
    }
    ctx->pool.push_back(p.a);
    ctx->pool.push_back(p.b);
  }
  ctx->pending.clear();
  for (int k = 0; k < LV_PH_COUNT; ++k) {
    if (ms) ms[k] = ctx->ms[k];
    if (calls) calls[k] = ctx->calls[k];
    ctx->ms[k] = 0.0;
    ctx->calls[k] = 0;
  }
  return LV_OK;
}

lv_status lv_autotune(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame, int32_t reps,
                      lv_settings* best, float* ms_table, hipStream_t stream) {
  if (!ctx || !best) return LV_ERR_ARG;
  lv_settings probe;
  lv_default_settings(&probe);
  if (best->t_eps > 0.0f) probe.t_eps = best->t_eps;
  lv::Layout L0;
  lv_status s = validate_all(ctx, vox, frame, &probe, &L0);
  if (s != LV_OK) return s;
  if (reps < 1) reps = 1;
  const int tiles[3] = {8, 16, 32};
  const int chunks[3] = {64, 128, 256};
  const uint64_t P = L0.P;
  const int64_t n = vox->n;
  const int nb = 3 * (vox->sh_degree + 1) * (vox->sh_degree + 1);
  float *rgb = nullptr, *depth = nullptr, *alpha = nullptr, *wmax = nullptr, *drgb = nullptr,
        *dd = nullptr, *dsh = nullptr;
  void* ws = nullptr;
  void* sv = nullptr;
  size_t ws_bytes = 0, sv_bytes = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
  lv_status result = LV_OK;
  float best_ms = -1.0f;
  auto cleanup = [&]() {
    for (void* p : {static_cast<void*>(rgb), static_cast<void*>(depth), static_cast<void*>(alpha),
                    static_cast<void*>(wmax), static_cast<void*>(drgb), static_cast<void*>(dd),
                    static_cast<void*>(dsh), ws, sv})
      if (p) (void)hipFree(p);
    for (hipEvent_t e : {e0, e1, e2})
      if (e) (void)hipEventDestroy(e);
  };
  bool ok = hipMalloc(&rgb, 12 * P) == hipSuccess && hipMalloc(&depth, 4 * P) == hipSuccess &&
            hipMalloc(&alpha, 4 * P) == hipSuccess && hipMalloc(&drgb, 12 * P) == hipSuccess &&
            hipMalloc(&wmax, 4 * size_t(n > 0 ? n : 1)) == hipSuccess &&
            hipMalloc(&dd, 32 * size_t(n > 0 ? n : 1)) == hipSuccess &&
            hipMalloc(&dsh, 4 * size_t(nb) * size_t(n > 0 ? n : 1)) == hipSuccess &&
            hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
            hipEventCreate(&e2) == hipSuccess;
  if (!ok) { cleanup(); return fail(ctx, LV_ERR_HIP, "autotune: allocation failed"); }
  // a small non-zero upstream gradient so the backward does its full work
  if (lv::launch_fill_u32(reinterpret_cast<uint32_t*>(drgb), 3 * P, 0x358637bdu /* 1e-6f */, stream) != hipSuccess ||
      lv::launch_fill_u32(reinterpret_cast<uint32_t*>(wmax), uint64_t(n > 0 ? n : 1), 0u, stream) != hipSuccess) {
    cleanup();
    return fail(ctx, LV_ERR_HIP, "autotune: fill failed");
  }
  const bool was_timing = ctx->timing;
  ctx->timing = false;
  for (int ti = 0; ti < 3 && result == LV_OK; ++ti) {
    lv_settings st = probe;
    st.tile = tiles[ti];
    uint64_t cap = std::max<uint64_t>(1u << 20, 2ull * uint64_t(n) * uint64_t(frame->n_views));
    cap = std::min<uint64_t>(cap, 0xFFFFFFFFull);
    uint64_t needed = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
      st.pair_capacity = cap;
      lv::Layout L;
      validate_all(ctx, vox, frame, &st, &L);
      if (L.total > ws_bytes) {
        if (ws) (void)hipFree(ws);
        ws = nullptr;
        if (hipMalloc(&ws, L.total) != hipSuccess) { result = fail(ctx, LV_ERR_HIP, "autotune: workspace"); break; }
        ws_bytes = L.total;
      }
      if (L.total_saved > sv_bytes) {
        if (sv) (void)hipFree(sv);
        sv = nullptr;
        if (hipMalloc(&sv, L.total_saved) != hipSuccess) { result = fail(ctx, LV_ERR_HIP, "autotune: saved state"); break; }
        sv_bytes = L.total_saved;
      }
      if ((s = lv_forward(ctx, vox, frame, &st, ws, sv, rgb, depth, alpha, wmax, stream)) != LV_OK) { result = s; break; }
      s = lv_check_overflow(ctx, vox, frame, &st, sv, &needed, stream);
      if (s == LV_OK) break;
      if (s != LV_ERR_CAPACITY) { result = s; break; }
      cap = std::min<uint64_t>(needed + needed / 16 + 1024, 0xFFFFFFFFull);
    }
    if (result != LV_OK) break;
    // the forward's per-pixel results do not depend on the chunk, so the
    // backward can be repeated on any forward's workspace
    float fwd_ms[3], bwd_ms[3];
    for (int ci = 0; ci < 3; ++ci) {
      st.chunk = chunks[ci];
      st.chunk_bwd = chunks[ci];
      float mf = 0.0f, mb = 0.0f;
      bool run_ok = lv_forward(ctx, vox, frame, &st, ws, sv, rgb, depth, alpha, wmax, stream) == LV_OK &&
                    lv_backward(ctx, vox, frame, &st, ws, sv, drgb, nullptr, nullptr, dd, dsh, stream) == LV_OK &&
                    hipEventRecord(e0, stream) == hipSuccess;
      for (int r = 0; r < reps && run_ok; ++r)
        run_ok = lv_forward(ctx, vox, frame, &st, ws, sv, rgb, depth, alpha, wmax, stream) == LV_OK;
      run_ok = run_ok && hipEventRecord(e1, stream) == hipSuccess;
      for (int r = 0; r < reps && run_ok; ++r)
        run_ok = lv_backward(ctx, vox, frame, &st, ws, sv, drgb, nullptr, nullptr, dd, dsh, stream) == LV_OK;
      run_ok = run_ok && hipEventRecord(e2, stream) == hipSuccess && hipEventSynchronize(e2) == hipSuccess &&
               hipEventElapsedTime(&mf, e0, e1) == hipSuccess && hipEventElapsedTime(&mb, e1, e2) == hipSuccess;
      fwd_ms[ci] = run_ok ? mf / reps : -1.0f;
      bwd_ms[ci] = run_ok ? mb / reps : -1.0f;
      if (ms_table) {
        ms_table[ti * 3 + ci] = fwd_ms[ci];
        ms_table[9 + ti * 3 + ci] = bwd_ms[ci];
      }
    }
    int bf = -1, bb = -1;
    for (int ci = 0; ci < 3; ++ci) {
      if (fwd_ms[ci] >= 0.0f && (bf < 0 || fwd_ms[ci] < fwd_ms[bf])) bf = ci;
      if (bwd_ms[ci] >= 0.0f && (bb < 0 || bwd_ms[ci] < bwd_ms[bb])) bb = ci;
    }
    if (bf >= 0 && bb >= 0 && (best_ms < 0.0f || fwd_ms[bf] + bwd_ms[bb] < best_ms)) {
      best_ms = fwd_ms[bf] + bwd_ms[bb];
      *best = st;
      best->chunk = chunks[bf];
      best->chunk_bwd = chunks[bb];
      best->pair_capacity = std::min<uint64_t>(needed + needed / 16 + 1024, 0xFFFFFFFFull);
    }
  }
  ctx->timing = was_timing;
  cleanup();
  if (result == LV_OK && best_ms < 0.0f) result = fail(ctx, LV_ERR_HIP, "autotune: no configuration ran");
  return result;
}

}  // extern "C"

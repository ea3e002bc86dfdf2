/*
 * litevoxel.h -- C-ABI of the MI355X (gfx950) differentiable sparse-voxel tile
 * rasterizer: the hot path of the LiteVoxel training loop
 * (arXiv 2511.02510, "LiteVoxel: Low-memory Intelligent Thresholding for
 * Efficient Voxel Rasterization").
 *
 * The problem each call solves is the paper's Sec. III ("Preliminaries"):
 *   - a pinhole camera with centre o casts one ray r(t) = o + t d(x, y),
 *     t >= 0, through the centre of every pixel (eq. 1);
 *   - the scene is a set of non-overlapping cube voxels, leaves of an octree
 *     (Sec. III, "Sparse Voxel/Octree Indexing"); a leaf at level l with
 *     integer cell coordinates (i, j, k) is the cube
 *        [root_min + (i, j, k) e, root_min + (i + 1, j + 1, k + 1) e],
 *        e = root_size * 2^-l;
 *   - the voxels met by a ray are composited front to back (eq. 2-4):
 *        T_0 = 1, w_k = T_{k-1} alpha_k, T_k = T_{k-1}(1 - alpha_k),
 *        C = sum_k w_k c_k  (+ T_K * bg);
 *     alpha_k = 1 - exp(-tau_k), tau_k = the integral over the chord of the
 *     trilinear interpolation of the voxel's 8 corner densities;
 *     c_k = max(0, sh_0 + sum_{l>=1,m} Y_lm(dir) sh_lm), a real spherical
 *     harmonic expansion of degree <= 3 evaluated at the direction from the
 *     camera centre to the voxel centre (constant term in colour units);
 *     depth D = sum_k w_k (t_in + t_out)/2, alpha A = 1 - T_K;
 *   - the per-voxel maximum blending weight
 *        w_max(v) = max over rays hitting v of T_{k(v,r)-1} alpha_v   (eq. 5).
 * The backward pass gives the gradient of a loss with respect to the corner
 * densities and SH coefficients (densities and colours are the trainable
 * voxel parameters, Sec. II-B).  lv_lf_weight / lv_l1_grad implement the
 * inverse-Sobel reweighted L1 photometric term (Sec. IV-B, eq. 7-10) and
 * lv_depth_quantile the depth-binned w_max quantile cutoff
 * (Sec. IV-C, eq. 11-12 with the eq. 14 depth normalisation), also as the
 * pair lv_depth_bins / lv_depth_cutoff.
 *
 * Conventions for every call:
 *   - Device pointers point to memory of the context's device, owned by the
 *     caller; the library never frees or keeps them beyond the call.  The
 *     rasterizer takes two caller-owned buffers: `saved`, the state one
 *     lv_forward leaves for the lv_backward of the same pass (tile lists,
 *     voxel and view records, per-pixel state), and `workspace`, scratch
 *     that every call may overwrite.  Each pass that will be differentiated
 *     later keeps its own `saved`; one workspace serves them all.
 *   - All device work is enqueued on the given stream; no call below
 *     synchronises except lv_check_overflow, lv_pass_stats, lv_export_bins,
 *     lv_autotune and lv_read_timings, which say so.  The enqueuing calls
 *     allocate no device memory and can be captured into a HIP graph.
 *   - Errors: every call returns an lv_status.  Argument errors are detected
 *     on the host before anything is enqueued (LV_ERR_ARG); a HIP runtime or
 *     launch failure gives LV_ERR_HIP.  lv_last_error() returns a message for
 *     the last failure on a context.  No exception crosses the ABI.
 *   - A context is not thread-safe; use one context per host thread/stream.
 *   - Limits: n < 2^28 voxels, n_views <= LV_MAX_VIEWS, width and height
 *     <= 32767, levels <= 12, sh_degree <= 3, pair_capacity < 2^32.
 *   - Preconditions documented, not checked: corner densities >= 0, leaves do
 *     not overlap, cams_dev[i] has the width/height of cams_host[i], and
 *     wmax holds non-negative values (not -0.0).
 */
#ifndef LITEVOXEL_H
#define LITEVOXEL_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LV_MAX_VIEWS 256
#define LV_MAX_LEVEL 12

typedef enum {
  LV_OK = 0,
  LV_ERR_ARG = 1,          /* invalid argument (host-detected, nothing enqueued) */
  LV_ERR_HIP = 2,          /* HIP runtime / launch failure */
  LV_ERR_CAPACITY = 3,     /* pair buffer too small (see lv_check_overflow) */
  LV_ERR_UNSUPPORTED = 4,  /* unsupported setting or device */
  LV_ERR_STATE = 5         /* call out of order (e.g. graph replay without capture) */
} lv_status;

typedef struct lv_context lv_context;  /* opaque, library-owned */

/* Pinhole camera (eq. 1).  OpenCV axes: x right, y down, z forward;
 * x_cam = R (x_world - o); R row-major.  Pixel (px, py) has its centre at
 * (px + 0.5, py + 0.5); its ray direction is
 * normalize(R^T ((px + 0.5 - cx)/fx, (py + 0.5 - cy)/fy, 1)). */
typedef struct {
  float R[9];
  float o[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} lv_camera;

/* Density activations (applied to each stored value before the trilinear
 * interpolation, so a voxel's density stays trilinear). */
#define LV_ACT_NONE 0
#define LV_ACT_SOFTPLUS 1  /* log(1 + e^x) */
#define LV_ACT_EXP 2       /* e^x */

/* Sparse voxel leaves, structure of arrays in device memory.
 * Dense layout (corner_idx NULL): density [8][n] holds one value per voxel
 * corner.  Grid-point layout (the storage of the sparse-voxel rasterizer the
 * paper starts from, Sec. III): density [n_grid] holds values on shared
 * corner points and corner c of voxel v reads density[corner_idx[c n + v]];
 * an index outside [0, n_grid) reads a corner density of 0.  Either way
 * corner c of voxel v has density act(value), act = density_act. */
typedef struct {
  int64_t n;               /* number of leaves */
  int32_t sh_degree;       /* 0..3 */
  float root_min[3];       /* min corner of the cubic root cell */
  float root_size;         /* edge of the root cell */
  const uint16_t* ijk;     /* [3][n] integer cell coordinates at the leaf's level */
  const uint8_t* level;    /* [n] octree level (<= 12) */
  const float* density;    /* [8][n] corner values, corner c = x + 2y + 4z bits, or [n_grid] */
  const float* sh;         /* [3 (deg+1)^2][n], row (i*3 + channel), i = l*l + l + m */
  const int32_t* corner_idx;  /* [8][n] grid point of each corner, or NULL (dense layout) */
  int64_t n_grid;          /* grid points (grid-point layout only) */
  int32_t density_act;     /* LV_ACT_* */
} lv_voxels;

/* A batch of views rendered in one call.  Pixel buffers pack the views in
 * order: view v starts at pixel offset off[v] = sum_{u<v} W_u H_u; rgb is
 * [3][H][W] per view starting at 3*off[v]; depth/alpha are [H][W] per view
 * starting at off[v]. */
typedef struct {
  int32_t n_views;
  const lv_camera* cams_host;  /* host array [n_views] (sizes used for planning) */
  const lv_camera* cams_dev;   /* device array [n_views] read by the kernels */
  float bg[3];                 /* background colour added with weight T_K */
} lv_frame;

typedef struct {
  int32_t tile;            /* tile side in pixels: 8, 16 or 32 */
  int32_t chunk;           /* voxels staged in LDS per step of the forward: 64, 128 or 256 */
  int32_t chunk_bwd;       /* the same for the backward; 0 = chunk */
  float t_eps;             /* a ray stops once T < t_eps (0 < t_eps <= 1e-5) */
  uint64_t pair_capacity;  /* capacity of the (tile, voxel) pair buffers */
} lv_settings;

/* Execution phases timed by lv_set_timing / lv_read_timings. */
typedef enum {
  LV_PH_SETUP = 0, LV_PH_PREPROCESS, LV_PH_SCAN, LV_PH_EMIT, LV_PH_SORT, LV_PH_ORDER,
  LV_PH_COMPOSITE_FWD, LV_PH_BWD_SETUP, LV_PH_COMPOSITE_BWD, LV_PH_SH_BWD,
  LV_PH_COUNT
} lv_phase;

/* ---------------------------------------------------------------- context */
lv_status lv_create(lv_context** out, int hip_device);   /* sets the device current */
void lv_destroy(lv_context* ctx);
const char* lv_status_str(lv_status s);
const char* lv_last_error(const lv_context* ctx);        /* "" if none; ctx may be NULL */
void lv_default_settings(lv_settings* s);   /* tile 16, chunk 64, chunk_bwd 0, t_eps 1e-6 */

/* Host-only argument checks (no device access): LV_OK or LV_ERR_ARG. */
lv_status lv_validate(const lv_voxels* vox, const lv_frame* frame, const lv_settings* st);

/* Host-only planning: bytes of the device workspace (scratch) and of the
 * saved state that lv_forward/lv_backward need for these shapes and
 * settings (pair capacity included).  The saved state is
 * 48 n + 32 n V + 8 P + 4 pair_capacity + 68 T bytes (T tiles, P pixels,
 * V views) plus alignment.  ctx may be NULL. */
lv_status lv_query_sizes(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                         const lv_settings* st, uint64_t* workspace_bytes, uint64_t* saved_bytes);

/* ------------------------------------------------------------------ forward
 * Sec. III, eq. 1-5.  Projects and bins every (voxel, view) record into
 * tiles, sorts each tile's list front to back, composites every pixel and
 * max-accumulates w_max.  Outputs: rgb [3P] (layout above), depth [P],
 * alpha [P] (all overwritten), wmax [n] (max-combined with its contents: the
 * caller zeroes it at the start of an adaptation window).  `saved`
 * (>= saved_bytes of lv_query_sizes, 256-byte aligned, overwritten) receives
 * what lv_backward reads: the view table, voxel and per-view records, the
 * per-tile front-to-back voxel lists, the pair count and, per pixel, the
 * index of the last hit and the transmittance before it (8 bytes; no
 * per-sample state).  `workspace` (>= workspace_bytes, 256-byte aligned) is
 * scratch.  If the pairs exceed pair_capacity the outputs are invalid and
 * lv_check_overflow reports it. */
lv_status lv_forward(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                     const lv_settings* st, void* workspace, void* saved, float* rgb,
                     float* depth, float* alpha, float* wmax, hipStream_t stream);

/* ----------------------------------------------------------------- backward
 * Adjoint of eq. 2-4 (and of the trilinear opacity and SH colour models):
 * given dL/d(rgb) [3P] and optional dL/d(depth), dL/d(alpha) [P] (NULL =
 * zero), writes dL/d(density) and dL/d(sh) [3 (deg+1)^2][n] (overwritten).
 * dL/d(density) has the layout of vox->density: [8][n] for the dense layout,
 * [n_grid] for grid points (each point sums the gradients of the corners
 * that read it), with respect to the stored values (through the
 * activation).  Transmittance is recomputed back to front from the state
 * the forward pass left in `saved`, which is only read; vox, frame and
 * settings (pair capacity included) must be those of that forward, and
 * vox's parameter arrays must hold the values it rendered.  `workspace` is
 * scratch of workspace_bytes (any buffer, not necessarily the forward's). */
lv_status lv_backward(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                      const lv_settings* st, void* workspace, const void* saved,
                      const float* d_rgb, const float* d_depth, const float* d_alpha,
                      float* d_density, float* d_sh, hipStream_t stream);

/* ------------------------------------------------------- auxiliary channels
 * Render channels for the auxiliary terms of the training objective (eq. 6
 * and eq. 17 name ray-space distortion and depth-normal consistency among
 * them without defining them; readings used):
 *   dist [P]    per pixel  sum_i sum_j w_i w_j |tm_i - tm_j| + 1/3 sum_i w_i^2 l_i
 *               over the composited hits (tm = (t_in + t_out)/2, l = t_out - t_in);
 *   normal      per pixel  N = sum_k w_k n_k, rgb layout ([3][H][W] per view),
 *               n_v = -u/|u| with u the gradient of voxel v's trilinear
 *               density at the cell centre (n_v = 0 when u = 0);
 *   mdepth [P]  per pixel  the median depth that the median-based
 *               depth-normal term of eq. 17 reads: tm of the first hit after
 *               which the transmittance is at most 1/2, 0 when no hit takes
 *               it there.  Piecewise constant in the densities: no gradient.
 * lv_forward_aux is lv_forward that also writes dist, normal and mdepth (any
 * may be NULL; the rest as lv_forward, the same `saved` for the backward).
 * lv_backward_aux is lv_backward with the upstream gradients of the new
 * channels: d_dist [P] and d_normal (rgb layout), each nullable; d_dist
 * needs depth_fwd, the depth lv_forward_aux wrote for this pass (the
 * backward recovers the depth accumulated before each hit from it), else
 * LV_ERR_ARG.  With both NULL it equals lv_backward. */
lv_status lv_forward_aux(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                         const lv_settings* st, void* workspace, void* saved, float* rgb,
                         float* depth, float* alpha, float* wmax, float* dist, float* normal,
                         float* mdepth, hipStream_t stream);
lv_status lv_backward_aux(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                          const lv_settings* st, void* workspace, const void* saved,
                          const float* d_rgb, const float* d_depth, const float* d_alpha,
                          const float* depth_fwd, const float* d_dist, const float* d_normal,
                          float* d_density, float* d_sh, hipStream_t stream);

/* Image-space auxiliary terms per view (eq. 6 and 17; readings used):
 *   loss[4v + 0] = lam_tc / |P_v| sum_p A (1 - A)        (transmittance concentration)
 *   loss[4v + 1] = lam_n / |I_v| sum_{p in I_v} (A - N . m)  (depth-normal consistency)
 *   loss[4v + 2] = lam_d / |P_v| sum_p dist              (distortion)
 *   loss[4v + 3] = lam_nm / |I_v| sum_{p in I_v} (A - N . m') (median depth-normal)
 * with I_v the interior pixels (1 <= x <= W-2, 1 <= y <= H-2; none when W or
 * H < 3) and m the unit normal of the surface of the depth channel: X = o +
 * D d (d the pixel's unit ray), m = normalise((X(x,y+1) - X(x,y-1)) x
 * (X(x+1,y) - X(x-1,y))) (0 when the cross product's squared length is below
 * the smallest normal float), facing the camera; m' is the same on the
 * median-depth map mdepth (from lv_forward_aux), which passes no gradient.
 * Writes (overwrites) loss [4 n_views] (device; each term summed with float
 * atomics in no fixed order, so the last bits may vary between calls) and the
 * gradients of the summed losses: d_alpha, d_depth, d_dist [P] and d_normal
 * (rgb layout), which are deterministic.  Every pointer but mdepth must be
 * non-NULL; mdepth may be NULL when lam_nm is 0 (the median term is then 0),
 * else LV_ERR_ARG. */
lv_status lv_aux_loss(lv_context* ctx, const lv_frame* frame, const float* depth,
                      const float* alpha, const float* normal, const float* dist,
                      const float* mdepth, float lam_tc, float lam_n, float lam_d, float lam_nm,
                      float* loss, float* d_alpha, float* d_depth, float* d_normal, float* d_dist,
                      hipStream_t stream);

/* Synchronises the stream and reports the number of (tile, voxel) pairs the
 * forward pass that filled `saved` produced: LV_OK if it fitted,
 * LV_ERR_CAPACITY otherwise. */
lv_status lv_check_overflow(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                            const lv_settings* st, const void* saved,
                            uint64_t* pairs_needed, hipStream_t stream);

/* Synchronises the stream and reports the size of the forward pass that
 * filled `saved`: pairs = (tile, voxel) pairs it produced (as
 * lv_check_overflow), records = visible (view, voxel) records (voxels whose
 * projected box covers at least one pixel centre of the view), counted by
 * one pass over the view records when `records` is not NULL (that pass
 * allocates and frees 8 bytes of device memory).  Either pointer may be NULL.
 * For measurement (bytes moved per pass). */
lv_status lv_pass_stats(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                        const lv_settings* st, const void* saved, uint64_t* pairs,
                        uint64_t* records, hipStream_t stream);

/* Copies the binning state a forward pass left in `saved` to host buffers
 * (synchronises): tile_start [T+1] (T = total tiles, views in order,
 * row-major), ids [tile_start[T]] voxel ids in per-tile front-to-back order,
 * codes [n_views*n] 36-bit visibility codes, rects [n_views*n*4] pixel-centre
 * ranges (x0, x1, y0, y1) and vis [n_views*n] (1 = record binned).  Any
 * pointer may be NULL.  For tests and debugging. */
lv_status lv_export_bins(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                         const lv_settings* st, const void* saved, uint32_t* tile_start,
                         uint32_t* ids, uint64_t* codes, int32_t* rects, uint8_t* vis,
                         hipStream_t stream);

/* ------------------------------------------------------------- loss (eq. 7-10)
 * Inverse-Sobel weight of each view's target (stop-gradient, Sec. IV-B):
 * grey = mean RGB; g = |3x3 Sobel| with replicated borders; g99 = the
 * ceil(0.99 |P|)-th smallest g of the view; form 0 (eq. 7):
 * w = (eps + 1 - min(1, g/g99))^gamma; form 1: w = (1 + g/g99)^-gamma
 * (g/g99 := 0 when g99 = 0); then w~ = w / mean_view(w) (eq. 8).
 * target/weight use the pixel layout above.  workspace >= lv_lf_weight_workspace_size. */
uint64_t lv_lf_weight_workspace_size(int32_t n_views);
lv_status lv_lf_weight(lv_context* ctx, const lv_frame* frame, const float* target,
                       float gamma, int32_t form, float eps, float* weight, void* workspace,
                       hipStream_t stream);

/* lv_lf_weight for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same computation and results, with the workspace replaced by a static
 * scratch array of the library (544 KiB per GPU, held until the process
 * ends), so the caller passes only inputs and outputs.  At most
 * LV_NOALLOC_MAX_VIEWS views (more: LV_ERR_ARG); the context's device must
 * be current (else LV_ERR_STATE).  Every call on one GPU shares that GPU's
 * scratch: calls that overlap in time on one GPU (other streams, other
 * contexts, other host threads) race and give undefined weights; calls on
 * one stream are ordered and safe.  Allocates nothing; each call clears the
 * scratch it needs on the stream before using it. */
#define LV_NOALLOC_MAX_VIEWS 64
lv_status lv_lf_weight_noalloc(lv_context* ctx, const lv_frame* frame, const float* target,
                               float gamma, int32_t form, float eps, float* weight,
                               hipStream_t stream);

/* Weighted L1 (eq. 10 with rho = mean over channels of |r|): writes
 * loss[v] = (1/|P_v|) sum_p w~(p) (1/3) sum_ch |C - I| per view (device
 * [n_views], overwritten) and d_rgb = w~ sign(C - I) / (3 |P_v|). */
lv_status lv_l1_grad(lv_context* ctx, const lv_frame* frame, const float* rgb,
                     const float* target, const float* weight, float* loss, float* d_rgb,
                     hipStream_t stream);

/* Piecewise-linear LF emphasis ramp gamma(t) of eq. 9 (host function). */
float lv_gamma_schedule(float t, float total, float t0_frac, float t1_frac, float gamma_max);

/* ------------------------------------------------- depth quantile (eq. 11-12)
 * Per voxel: delta = min over views with z_c > 0 of z_c / fx (the inter-ray
 * spacing at the voxel centre, the depth proxy), +inf if no view has it in
 * front; z~ = clip((delta - p5)/(p95 - p5), 0, 1) with nearest-rank 5th/95th
 * percentiles over all voxels (eq. 14); bin = min(B-1, floor(B z~)) (+inf ->
 * B-1; all finite voxels in bin 0 if p95 <= p5 or p95 = +inf).  Binning
 * arithmetic is binary32 in the order written.  Per bin:
 * tau_b = the ceil(q |V_b|)-th smallest w_max (eq. 11-12; -inf if empty)
 * and prune_v = (w_max_v <= tau_{bin(v)}).  Outputs tau [n_bins], prune [n],
 * bins [n] (nullable).  workspace >= lv_quantile_workspace_size. */
uint64_t lv_quantile_workspace_size(int64_t n, int32_t n_bins);
lv_status lv_depth_quantile(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                            const float* wmax, int32_t n_bins, double q, void* workspace,
                            float* tau, uint8_t* prune, uint8_t* bins, hipStream_t stream);

/* The same in two calls.  lv_depth_bins does the part that does not read
 * w_max (delta, p5/p95, bins and per-bin counts, kept in the workspace;
 * bins [n] also written when non-NULL), so it can run before or beside the
 * forward pass; lv_depth_cutoff then computes tau and prune from w_max on
 * that workspace.  The cutoff requires a workspace filled by lv_depth_bins
 * for the same voxels and n_bins (it may be called again with other w_max
 * values; otherwise its results are unspecified, but every access stays
 * inside the workspace).  Results are identical to lv_depth_quantile's. */
lv_status lv_depth_bins(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                        int32_t n_bins, void* workspace, uint8_t* bins, hipStream_t stream);
lv_status lv_depth_cutoff(lv_context* ctx, const lv_voxels* vox, const float* wmax, int32_t n_bins,
                          double q, void* workspace, float* tau, uint8_t* prune,
                          hipStream_t stream);

/* ------------------------------------------- pruning stability guards
 * One adaptation step of the three guards on pruning (Sec. IV-C, guards
 * i-iii), applied on top of lv_depth_quantile (same vox/frame; its tau and
 * bins, with the same n_bins; bin values >= n_bins are read as n_bins - 1):
 *   x_v = 1 if w_max_v > tau[bin_v], else 0      (inside score)
 *   i.   ema_v <- (1 - alpha) ema_v + alpha x_v;  state_v <- 0 (out) if
 *        ema_v < m_low, 1 (in) if ema_v > m_high, else unchanged
 *   ii.  protected if delta_v is finite and h_v < rho delta_v (h_v = half
 *        edge, delta_v the footprint defined for lv_depth_quantile), or
 *        w_max_v >= w_keep                         (keep-halo)
 *   iii. candidates = out and not protected; the first min(cap, count) of
 *        them in the order (ema_v, v) get prune_v = 1, cap =
 *        floor(cap_frac n) in double; ema ordered as binary32 (-0 < +0).
 * All arithmetic binary32, one rounded operation at a time as written.
 * ema [n] (f32) and state [n] (u8) are caller-owned device arrays updated in
 * place (start new voxels at 1.0 and 1); prune [n] (u8) is written;
 * n_pruned (device u32, nullable) receives the number pruned.  Argument
 * errors (null pointers for n > 0, alpha outside (0, 1], m_low > m_high,
 * rho < 0, cap_frac outside [0, 1], n_bins outside [1, 64]) return
 * LV_ERR_ARG before anything is enqueued.  The paper fixes none of the
 * constants; lv_default_guard gives alpha 0.3, m_low 0.3, m_high 0.7,
 * rho 0.25, w_keep 0.5, cap_frac 0.05. */
typedef struct {
  float alpha;
  float m_low, m_high;
  float rho;
  float w_keep;
  double cap_frac;
} lv_guard_params;
void lv_default_guard(lv_guard_params* p);
uint64_t lv_guard_workspace_size(int64_t n);
lv_status lv_prune_guard(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                         const float* wmax, const uint8_t* bins, const float* tau, int32_t n_bins,
                         const lv_guard_params* params, void* workspace, float* ema,
                         uint8_t* state, uint8_t* prune, uint32_t* n_pruned, hipStream_t stream);

/* ------------------------------------- priority-driven subdivision (Sec. IV-D)
 * Three calls, one workspace (>= lv_split_workspace_size(n)):
 *  lv_footprint_range: range [2] (device f32) = nearest-rank 5th and 95th
 *    percentiles over all voxels of delta (the footprint defined for
 *    lv_depth_quantile); 0, 0 without voxels.  One way to keep the running
 *    percentiles of eq. 14.
 *  lv_subdivide_select (eq. 13-16): with h_v the half edge and
 *    z~_v = clip((delta_v - range[0]) / (range[1] - range[0]), 0, 1)
 *    (+inf -> 1; range[1] <= range[0] or +inf -> 0 for finite delta),
 *      eligible_v = l_v < LV_MAX_LEVEL and delta_v finite and h_v > kappa delta_v
 *      priority_v = score_v (1 + beta z~_v)
 *    split [n] (u8) marks the first min(max_splits, count) eligible voxels
 *    with priority > 0 in the order (priority descending, index ascending).
 *    score [n] (f32) is the caller's running usefulness score P_v (the paper
 *    leaves it open).  priority [n] (f32, nullable) and n_split (device u32,
 *    nullable) are optional outputs.
 *  lv_subdivide_apply: writes the refined set of n_out = n + 7 (#split)
 *    leaves into caller-owned arrays laid out like lv_voxels with n_out
 *    rows (ijk [3][n_out] u16, level [n_out] u8, density [8][n_out] f32,
 *    sh [3 (deg+1)^2][n_out] f32): input order kept, each split voxel
 *    replaced in place by its 8 children (child c = x + 2y + 4z bits,
 *    ijk = 2 ijk + bits, level + 1), whose corner densities are the parent's
 *    trilinear field at their corners (midpoints 0.5 a + 0.5 b along x,
 *    then y, then z: the density field is unchanged) and whose SH are the
 *    parent's.  Flags on leaves at LV_MAX_LEVEL are ignored.  Dense layout only
 *    (LV_ERR_UNSUPPORTED for grid points); the midpoints refine the stored
 *    values, so with a density activation other than LV_ACT_NONE the
 *    children's field approximates the parent's instead of reproducing it.  n_needed
 *    (device u64, nullable) receives n + 7 (#split); rows at or beyond n_out
 *    are not written, so a wrong n_out gives a truncated set, never a write
 *    out of bounds.  The output arrays must not alias the input.
 * Binary32, one rounded operation at a time as written.  Argument errors
 * (null pointers for n > 0, kappa or beta negative or not finite, n_out < n)
 * return LV_ERR_ARG before anything is enqueued.  The paper fixes kappa ~ 1
 * and beta in [0.1, 0.3]; lv_default_split gives kappa 1, beta 0.2,
 * max_splits 8192. */
typedef struct {
  float kappa;
  float beta;
  uint32_t max_splits;
} lv_split_params;
void lv_default_split(lv_split_params* p);
uint64_t lv_split_workspace_size(int64_t n);
lv_status lv_footprint_range(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                             void* workspace, float* range, hipStream_t stream);
lv_status lv_subdivide_select(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                              const float* score, const float* range, const lv_split_params* params,
                              void* workspace, uint8_t* split, float* priority, uint32_t* n_split,
                              hipStream_t stream);
lv_status lv_subdivide_apply(lv_context* ctx, const lv_voxels* vox, const uint8_t* split,
                             int64_t n_out, void* workspace, uint16_t* ijk, uint8_t* level,
                             float* density, float* sh, uint64_t* n_needed, hipStream_t stream);

/* ------------------------------------------------------ execution structure
 * Graph capture: between lv_graph_begin and lv_graph_end every call that
 * enqueues on `stream` is recorded instead of run; lv_graph_launch replays
 * the instantiated graph on a stream.  Buffers and sizes are frozen at
 * capture; camera poses may change between replays through cams_dev.
 * `stream` must not be the null stream. */
lv_status lv_graph_begin(lv_context* ctx, hipStream_t stream);
lv_status lv_graph_end(lv_context* ctx, hipStream_t stream);
lv_status lv_graph_launch(lv_context* ctx, hipStream_t stream);
lv_status lv_graph_reset(lv_context* ctx);

/* Autotuner: times the forward and the backward separately for every tile in
 * {8,16,32} x chunk in {64,128,256} on these inputs (device memory it needs
 * is allocated and freed inside; synchronises) and writes into *best the
 * tile whose fastest forward plus fastest backward is smallest, with those
 * two chunks as chunk and chunk_bwd (capacity sized for that tile).
 * ms_table (nullable) receives 18 times in ms: 9 forward times, tile-major
 * over the chunks, then the 9 backward times in the same order; a
 * configuration that cannot run gets a negative entry. */
lv_status lv_autotune(lv_context* ctx, const lv_voxels* vox, const lv_frame* frame,
                      int32_t reps, lv_settings* best, float* ms_table, hipStream_t stream);

/* Per-phase GPU timing with HIP events recorded on the call's stream.
 * lv_read_timings synchronises and adds the elapsed ms of every phase since
 * the last read into ms[LV_PH_COUNT] and launch counts into calls. */
lv_status lv_set_timing(lv_context* ctx, int32_t enable);
lv_status lv_read_timings(lv_context* ctx, double* ms, int64_t* calls);

#ifdef __cplusplus
}
#endif

#endif /* LITEVOXEL_H */

// Per-tile compositing, forward (eq. 1-5) and backward (adjoint of eq. 2-4).
//
// Work unit: one TS x TS tile per workgroup, one pixel per lane, each wave an
// 8 x 8 pixel block.  Workgroups are persistent and pop tiles from an atomic
// queue ordered longest list first.  A tile's front-to-back voxel list is
// staged in LDS `chunk` voxels at a time (geometry relative to the camera,
// trilinear density coefficients, colour, pixel-centre coverage).  Per 64
// staged voxels the workgroup builds, with ballots, one 64-bit mask per tile
// row and per tile column; a lane's candidate set is the AND of its row and
// column masks, so it visits only voxels whose projected box covers its pixel
// centre, in list order (lowest bit first; backward: highest first).  A lane stops once its transmittance falls below t_eps; the wave
// and the workgroup stop when every lane has.
//
// Optical depth: the trilinear density along a chord is a cubic in t, so the
// 2-point Gauss-Legendre rule on [t_in, t_out] integrates it exactly.
//
// w_max (eq. 5) is max-reduced per chunk in LDS (integer max on the bits of a
// non-negative float, exact and order-independent) and then flushed with one
// global atomic max per (tile, voxel).  Backward gradients (8 corner
// densities + 3 colour channels per voxel) are first summed over runs of
// lanes that hold the same voxel in the same step (DPP, each 16-lane row a
// 4 x 4 pixel block), then pre-reduced per chunk in LDS and flushed with one
// global atomic add per (tile, voxel, component).
//
// Auxiliary channels (the AUX instances; the training objective's eq. 6 and
// eq. 17 name the terms they serve without defining them): per pixel the
// ray-space distortion sum_i sum_j w_i w_j |tm_i - tm_j| + 1/3 sum_i w_i^2 l_i
// (tm chord midpoint, l chord length), the rendered normal sum_k w_k n_k
// with n_v = -u / |u|, u the gradient of the voxel's trilinear density at
// the cell centre, and the median depth (tm of the hit that takes T to 1/2
// or below, 0 if none does; no gradient passes through it).  Front to back, the sum of the earlier weights is 1 - T
// and their depth sum is the depth accumulated so far, so the distortion
// takes one multiply-add chain per hit; the backward recovers the earlier
// depth sum from the forward's depth.
#include "lv_common.h"

namespace lv {

constexpr float kGL = 0.57735026918962576f;  // 1/sqrt(3): 2-point Gauss-Legendre node
constexpr float kSmallTau = 0.03125f;

template <int CH>
struct Stage {
  float rlo[3][CH];   // b - o
  float edge[CH];     // e (the far planes are b - o + e)
  float inve[CH];
  float cf[8][CH];    // trilinear density as a polynomial in (ux, uy, uz)
  float col[3][CH];
  uint32_t xr[CH];    // pixel-centre range x0 | x1 << 16
  uint32_t yr[CH];
  uint32_t id[CH];    // voxel id | colour clamp mask (bit c: raw channel c > 0) << 28
};

struct Ray {
  float d[3];
  float inv[3];
};

// the voxel normal n = -u / |u| and 1 / |u| (0 when u = 0), for the AUX passes
template <int CH>
struct StageAux {
  float n[3][CH];
  float iu[CH];
};

// Error-free transformations (contraction is off, so these are evaluated as
// written): a + b = s + e and a * b = p + e exactly.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
  p = a * b;
  e = fmaf(a, b, -p);
}

// Unit ray direction through the centre of pixel (px, py) (eq. 1), each
// component with a small error relative to itself.  A chord's entry or exit
// through a face of axis a lies at t = (plane - o_a) / d_a, so an absolute
// error in a small d_a (a ray nearly parallel to that face) would move the
// crossing by error / d_a.  The camera-space direction ((px + .5 - cx) / fx,
// (py + .5 - cy) / fy, 1) is therefore carried as unevaluated float pairs
// and R^T applied in compensated arithmetic: each world component is the
// correctly rounded sum of its products up to a few ulps of itself, also
// where the products cancel.  The normalisation (hardware reciprocal square
// root) then scales all three components alike, and the inverse components
// are hardware reciprocals (about 1 ulp each); the forward and the backward
// both take their chords from this one function.  Per pixel, not per
// fragment.
__device__ __forceinline__ Ray pixel_ray(const lv_camera& c, int px, int py) {
  const float nx = (float(px) + 0.5f) - c.cx, ny = (float(py) + 0.5f) - c.cy;   // exact
  // hardware reciprocals (about 1 ulp): xh within a few ulps of nx / fx, and
  // xh + xl equal to it far below the binary32 rounding of the pair's sum
  const float rfx = __builtin_amdgcn_rcpf(c.fx), rfy = __builtin_amdgcn_rcpf(c.fy);
  const float xh = nx * rfx, yh = ny * rfy;
  const float xl = fmaf(-xh, c.fx, nx) * rfx, yl = fmaf(-yh, c.fy, ny) * rfy;
  float dd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float p1, e1, p2, e2, s1, e3, s2, e4;
    two_prod(c.R[a], xh, p1, e1);
    two_prod(c.R[3 + a], yh, p2, e2);
    two_sum(p1, p2, s1, e3);
    two_sum(s1, c.R[6 + a], s2, e4);
    const float low = ((e1 + e2) + (e3 + e4)) + (c.R[a] * xl + c.R[3 + a] * yl);
    dd[a] = s2 + low;
  }
  const float in = __builtin_amdgcn_rsqf(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  Ray r;
  r.d[0] = dd[0] * in; r.d[1] = dd[1] * in; r.d[2] = dd[2] * in;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float x = r.d[a];
    if (fabsf(x) < 1e-30f) x = x < 0.0f ? -1e-30f : 1e-30f;
    r.inv[a] = __builtin_amdgcn_rcpf(x);
  }
  return r;
}

// Stage voxels [cb, cb + nc) of the tile list into LDS (with AUX also the
// voxel normals into SA).
template <int CH, int NT, bool AUX>
__device__ __forceinline__ void stage_chunk(Stage<CH>& S, StageAux<CH>* SA, const RasterArgs& a,
                                            const uint32_t* ids, uint32_t cb, uint32_t nc,
                                            int view, const float o[3]) {
  for (uint32_t k = threadIdx.x; k < uint32_t(CH); k += NT) {
    if (k < nc) {
      const uint32_t id = ids[cb + k];
      const VoxRec vr = a.ws.vox[id];
      const uint4 r0 = reinterpret_cast<const uint4*>(&a.ws.rec[size_t(view) * size_t(a.n) + id])[0];
      const uint4 r1 = reinterpret_cast<const uint4*>(&a.ws.rec[size_t(view) * size_t(a.n) + id])[1];
      const float e = vr.be.w;
      const float ie = 1.0f / e;
      const float bl[3] = {vr.be.x - o[0], vr.be.y - o[1], vr.be.z - o[2]};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        S.rlo[ax][k] = bl[ax];
      }
      S.edge[k] = e;
      S.inve[k] = ie;
      const float s000 = vr.s0.x, s100 = vr.s0.y, s010 = vr.s0.z, s110 = vr.s0.w;
      const float s001 = vr.s1.x, s101 = vr.s1.y, s011 = vr.s1.z, s111 = vr.s1.w;
      S.cf[0][k] = s000;
      S.cf[1][k] = s100 - s000;
      S.cf[2][k] = s010 - s000;
      S.cf[3][k] = s001 - s000;
      S.cf[4][k] = (s110 - s100) - (s010 - s000);
      S.cf[5][k] = (s101 - s100) - (s001 - s000);
      S.cf[6][k] = (s011 - s010) - (s001 - s000);
      S.cf[7][k] = ((s111 - s110) - (s101 - s100)) - ((s011 - s010) - (s001 - s000));
      if (AUX) {
        // u_a: a quarter of the summed corner differences along axis a
        const float ux = 0.25f * (((s100 - s000) + (s110 - s010)) + ((s101 - s001) + (s111 - s011)));
        const float uy = 0.25f * (((s010 - s000) + (s110 - s100)) + ((s011 - s001) + (s111 - s101)));
        const float uz = 0.25f * (((s001 - s000) + (s101 - s100)) + ((s011 - s010) + (s111 - s110)));
        const float ul = sqrtf(ux * ux + uy * uy + uz * uz);
        const float iu = ul > 0.0f ? 1.0f / ul : 0.0f;
        SA->n[0][k] = -ux * iu;
        SA->n[1][k] = -uy * iu;
        SA->n[2][k] = -uz * iu;
        SA->iu[k] = iu;
      }
      S.col[0][k] = __uint_as_float(r0.x);
      S.col[1][k] = __uint_as_float(r0.y);
      S.col[2][k] = __uint_as_float(r0.z);
      S.xr[k] = r1.x;
      S.yr[k] = r1.y;
      S.id[k] = id | ((r0.w & 7u) << kIdBits);
    } else {
      S.xr[k] = 1u;   // empty range (x0 = 1 > x1 = 0)
      S.yr[k] = 1u;
      S.id[k] = 0u;
    }
  }
}

// Coverage masks of a staged chunk, built once per tile: for every 64-voxel
// word w and every tile row r (column c), a 64-bit mask of the voxels whose
// pixel-centre range covers that row (column).  The waves share the 2 TS
// ballots per word; a lane's candidate set is rows[w][its row] &
// cols[w][its column].  Needs a barrier before the masks are read.
template <int TS, int CH>
struct Masks {
  unsigned long long rows[CH / 64][TS];
  unsigned long long cols[CH / 64][TS];
};

template <int TS, int CH>
__device__ __forceinline__ void build_masks(const Stage<CH>& S, Masks<TS, CH>& M, uint32_t nc,
                                            int tox, int toy) {
  constexpr int NWAVES = TS * TS / 64;
  constexpr int RPW = TS / NWAVES;   // rows (and columns) per wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwords = int((nc + 63) / 64);
  for (int w = 0; w < nwords; ++w) {
    const int j = w * 64 + lane;
    int ylo = int(S.yr[j] & 0xFFFFu) - toy, yhi = int(S.yr[j] >> 16) - toy;
    int xlo = int(S.xr[j] & 0xFFFFu) - tox, xhi = int(S.xr[j] >> 16) - tox;
    const uint32_t ys = yhi >= ylo ? uint32_t(yhi - ylo) : 0u;
    const uint32_t xs = xhi >= xlo ? uint32_t(xhi - xlo) : 0u;
    ylo = yhi >= ylo ? ylo : -0x10000;
    xlo = xhi >= xlo ? xlo : -0x10000;
    unsigned long long br = 0, bc = 0;
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = wave * RPW + k;
      const unsigned long long yb = __builtin_amdgcn_ballot_w64(uint32_t(r - ylo) <= ys);
      const unsigned long long xb = __builtin_amdgcn_ballot_w64(uint32_t(r - xlo) <= xs);
      br = lane == k ? yb : br;
      bc = lane == k ? xb : bc;
    }
    if (lane < RPW) {
      M.rows[w][wave * RPW + lane] = br;
      M.cols[w][wave * RPW + lane] = bc;
    }
  }
}

struct Seg {
  bool hit;
  float tn, tf;
};

template <int CH>
__device__ __forceinline__ Seg slab(const Stage<CH>& S, int j, const Ray& ray) {
  const float e = S.edge[j];
  const float l0 = S.rlo[0][j], l1 = S.rlo[1][j], l2 = S.rlo[2][j];
  const float a0 = l0 * ray.inv[0], b0 = (l0 + e) * ray.inv[0];
  const float a1 = l1 * ray.inv[1], b1 = (l1 + e) * ray.inv[1];
  const float a2 = l2 * ray.inv[2], b2 = (l2 + e) * ray.inv[2];
  Seg s;
  s.tn = fmaxf(fmaxf(fminf(a0, b0), fminf(a1, b1)), fmaxf(fminf(a2, b2), 0.0f));
  s.tf = fminf(fminf(fmaxf(a0, b0), fmaxf(a1, b1)), fmaxf(a2, b2));
  s.hit = s.tf > s.tn;
  return s;
}

struct Quad {
  float tm, hl;
  float ua[3], ub[3];
  float tau;
};

template <int CH>
__device__ __forceinline__ float trilin(const Stage<CH>& S, int j, const float u[3]) {
  float t = fmaf(u[2], S.cf[7][j], S.cf[4][j]);
  t = fmaf(u[1], t, S.cf[1][j]);
  t = fmaf(u[2], S.cf[5][j], t);
  const float q = fmaf(u[2], S.cf[6][j], S.cf[2][j]);
  float s = fmaf(u[0], t, S.cf[0][j]);
  s = fmaf(u[1], q, s);
  s = fmaf(u[2], S.cf[3][j], s);
  return s;
}

template <int CH>
__device__ __forceinline__ Quad quad(const Stage<CH>& S, int j, const Ray& ray, const Seg& sg) {
  Quad q;
  q.tm = 0.5f * (sg.tn + sg.tf);
  q.hl = 0.5f * (sg.tf - sg.tn);
  const float ta = fmaf(-q.hl, kGL, q.tm), tb = fmaf(q.hl, kGL, q.tm);
  const float ie = S.inve[j];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const float du = ray.d[ax] * ie;
    const float su = S.rlo[ax][j] * ie;   // (b - o) / e, recomputed: LDS is the occupancy limit
    q.ua[ax] = fmaf(ta, du, -su);
    q.ub[ax] = fmaf(tb, du, -su);
  }
  const float sa = trilin(S, j, q.ua), sb = trilin(S, j, q.ub);
  q.tau = fmaxf(q.hl * (sa + sb), 0.0f);
  return q;
}

// alpha = 1 - exp(-tau) without cancellation for small tau: below 1/32 the
// Taylor series to tau^4 (Horner form, relative truncation error < 8e-9)
// (both forms are evaluated and one is selected: lanes of a wave disagree)
__device__ __forceinline__ float opacity(float tau, float ex) {
  float t = fmaf(tau, -0.041666667f, 0.16666667f);
  t = fmaf(tau, t, -0.5f);
  t = fmaf(tau, t, 1.0f);
  return tau < kSmallTau ? tau * t : 1.0f - ex;
}


// ------------------------------------------------ run-combined LDS updates
// Neighbouring pixels walk nearly the same voxel lists in lockstep, so in one
// step many lanes of a wave update the same voxel, and LDS atomics on one
// address are executed one lane at a time.  Each 16-lane DPP row covers a
// 4 x 4 pixel block; runs of consecutive lanes of a row that hold the same
// voxel are summed by a segmented inclusive scan (row shifts by 1, 2, 4, 8)
// and only the last lane of a run updates LDS.  The LDS accumulators are
// doubles: on gfx950 an LDS add on f64 costs about a tenth of one on f32 per
// lane (and rounds less).  Must be called with every lane of the wave active.
__device__ __forceinline__ int pix_x_of_lane(int lane) { return ((lane >> 4) & 1) * 4 + (lane & 3); }
__device__ __forceinline__ int pix_y_of_lane(int lane) { return (lane >> 5) * 4 + ((lane >> 2) & 3); }

// One step of the scan over 11 values: v += v' * f, where v' is the value
// of lane - K in the same 16-lane row and f = 1 when that lane lies in this
// lane's run, 0 otherwise; one fused multiply-add per value that reads v'
// through DPP (a lane with no source in its row keeps v).  The leading and trailing s_nop
// give the two wait states a DPP read needs after a VALU write of its
// operand, on both sides of the block.  Every lane of the wave must be active.
#define LV_SEG_FMAC(K, R) "v_fmac_f32_dpp %" #R ", %" #R ", %11 row_shr:" #K " row_mask:0xf bank_mask:0xf\n"
#define LV_SEG_BLOCK(K)                                                                     \
  "s_nop 1\n" LV_SEG_FMAC(K, 0) LV_SEG_FMAC(K, 1) LV_SEG_FMAC(K, 2) LV_SEG_FMAC(K, 3)         \
      LV_SEG_FMAC(K, 4) LV_SEG_FMAC(K, 5) LV_SEG_FMAC(K, 6) LV_SEG_FMAC(K, 7) LV_SEG_FMAC(K, 8) \
          LV_SEG_FMAC(K, 9) LV_SEG_FMAC(K, 10) "s_nop 1"

#define LV_SEG_FMAC3(K, R) "v_fmac_f32_dpp %" #R ", %" #R ", %3 row_shr:" #K " row_mask:0xf bank_mask:0xf\n"
#define LV_SEG_BLOCK3(K)                                                              \
  "s_nop 1\n" LV_SEG_FMAC3(K, 0) LV_SEG_FMAC3(K, 1) LV_SEG_FMAC3(K, 2) "s_nop 1"

// the same step over 3 further values (the normal gradient of the AUX pass)
template <int K>
__device__ __forceinline__ void seg_step3(float* v, float f) {
#define LV_SEG_ASM3(K)                                                                           \
  asm volatile(LV_SEG_BLOCK3(K) : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]) : "v"(f))
  if constexpr (K == 1) LV_SEG_ASM3(1);
  else if constexpr (K == 2) LV_SEG_ASM3(2);
  else if constexpr (K == 4) LV_SEG_ASM3(4);
  else LV_SEG_ASM3(8);
#undef LV_SEG_ASM3
}

template <int K, int NV>
__device__ __forceinline__ void seg_step(float* v, int dist) {
  if (__ballot(dist >= K) == 0) return;
  const float f = dist >= K ? 1.0f : 0.0f;
#define LV_SEG_ASM(K)                                                                          \
  asm volatile(LV_SEG_BLOCK(K)                                                                 \
               : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]),       \
                 "+v"(v[6]), "+v"(v[7]), "+v"(v[8]), "+v"(v[9]), "+v"(v[10])                   \
               : "v"(f))
  if constexpr (K == 1) LV_SEG_ASM(1);
  else if constexpr (K == 2) LV_SEG_ASM(2);
  else if constexpr (K == 4) LV_SEG_ASM(4);
  else LV_SEG_ASM(8);
#undef LV_SEG_ASM
  if constexpr (NV > 11) seg_step3<K>(v + 11, f);
}
#undef LV_SEG_BLOCK
#undef LV_SEG_FMAC
#undef LV_SEG_BLOCK3
#undef LV_SEG_FMAC3

// After the call, a lane with `last` set holds in v the sum over its run of
// lanes with the same key (pend lanes only; others form runs of their own).
template <int NV>
__device__ __forceinline__ bool seg_reduce_rows(float (&v)[NV], int jj, bool pend) {
  const int lane = threadIdx.x & 63;
  const int key = pend ? jj : -1 - lane;
  const int prev = __builtin_amdgcn_update_dpp(0x7FFFFFFF, key, 0x111, 0xF, 0xF, false);
  const bool head = (lane & 15) == 0 || prev != key;
  const unsigned long long H = __ballot(head);
  const bool last = (lane & 15) == 15 || (((H >> lane) >> 1) & 1ull);
  if (H != ~0ull) {
    const unsigned long long le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int dist = lane - (63 - __builtin_clzll(H & le));
    seg_step<1, NV>(v, dist);
    seg_step<2, NV>(v, dist);
    seg_step<4, NV>(v, dist);
    seg_step<8, NV>(v, dist);
  }
  return last;
}

// ------------------------------------------------------------ tile queues
// The longest-first tile order is dealt round-robin to nq = min(kQueues,
// blocks) queues; block b pops queue b mod nq, whose j-th entry is order
// position q + j nq.  Every queue has at least one block (the grid has at
// least nq blocks), so every tile is taken exactly once.  pop() returns an
// order position, or T once the block's queue is exhausted.
struct TileQueue {
  uint32_t* head;
  uint32_t q, nq, len, T;
  __device__ uint32_t pop() const {
    const uint32_t j = atomicAdd(head, 1u);
    return j < len ? q + j * nq : T;
  }
};

__device__ __forceinline__ TileQueue tile_queue(uint32_t T, uint32_t* heads) {
  TileQueue tq;
  tq.nq = gridDim.x < uint32_t(kQueues) ? gridDim.x : uint32_t(kQueues);
  tq.q = blockIdx.x % tq.nq;
  tq.len = T > tq.q ? (T - tq.q + tq.nq - 1) / tq.nq : 0u;
  tq.head = heads + tq.q * kQueueStride;
  tq.T = T;
  return tq;
}

// ======================================================================
// forward
// A pixel is done once T < t_eps; pixels outside the image start with T = 0.
struct FwdState {
  float T, C0, C1, C2, D, Tpre;
  uint32_t nlast;
  float N0, N1, N2, L;   // AUX: rendered normal, distortion
  float M;               // AUX: median depth
};

// one hit fragment (this lane's pixel, voxel jj at list position pos, chord
// sg); returns w_k
template <int CH, bool AUX>
__device__ __forceinline__ float fwd_fragment(const Stage<CH>& S, const StageAux<CH>* SA, int jj,
                                              uint32_t pos, const Ray& ray, const Seg& sg,
                                              FwdState& st) {
  const Quad q = quad(S, jj, ray, sg);
  const float ex = __expf(-q.tau);
  const float al = opacity(q.tau, ex);
  const float wk = st.T * al;
  if (AUX) {
    // earlier weights sum to 1 - T and their depths to D: the pairs of this
    // hit with the earlier ones add 2 wk (tm (1 - T) - D), its own segment
    // wk^2 l / 3 with l = 2 hl
    const float pair = fmaf(q.tm, 1.0f - st.T, -st.D);
    st.L = fmaf(2.0f * wk, pair, st.L);
    st.L = fmaf(wk * wk, q.hl * (2.0f / 3.0f), st.L);
    st.N0 = fmaf(wk, SA->n[0][jj], st.N0);
    st.N1 = fmaf(wk, SA->n[1][jj], st.N1);
    st.N2 = fmaf(wk, SA->n[2][jj], st.N2);
    // median depth: the hit that takes the transmittance to 1/2 or below
    // (T only decreases, so this happens at most once)
    if (st.T > 0.5f && st.T * ex <= 0.5f) st.M = q.tm;
  }
  st.C0 = fmaf(wk, S.col[0][jj], st.C0);
  st.C1 = fmaf(wk, S.col[1][jj], st.C1);
  st.C2 = fmaf(wk, S.col[2][jj], st.C2);
  st.D = fmaf(wk, q.tm, st.D);
  st.Tpre = st.T;
  st.nlast = pos + 1u;
  st.T = st.T * ex;
  return wk;
}

// Occupancy targets: 7 waves per SIMD for the AUX instances (at most 72
// registers, no spills; 84 registers and 5 waves with no target: 0.56 ms on the ring
// workload, 0.513 at 6 waves, 0.490 at 7), 8 for the plain ones (64
// registers with a few spilled outside the candidate loop; 72 and 7 waves
// otherwise, 0.458 against 0.424 ms)
template <int TS, int NW, bool AUX>
__global__ __launch_bounds__(TS* TS) __attribute__((amdgpu_waves_per_eu(AUX ? 7 : 8))) void k_composite_fwd(
    RasterArgs a) {
  constexpr int NT = TS * TS;
  constexpr int CH = 64 * NW;
  constexpr int BPR = TS / 8;
  __shared__ Stage<CH> S;
  __shared__ StageAux<AUX ? CH : 64> s_aux;
  StageAux<CH>* SA = AUX ? reinterpret_cast<StageAux<CH>*>(&s_aux) : nullptr;
  __shared__ Masks<TS, CH> MK;
  __shared__ uint32_t s_wmax[CH];
  __shared__ uint32_t s_tile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = lane & 7, ly = lane >> 3;
  const int wbx = (wave % BPR) * 8, wby = (wave / BPR) * 8;

  // the next queue slot is taken while the current tile is processed; a
  // block stops at the first slot past the end of its queue
  const TileQueue tq = tile_queue(a.T, a.ws.counters + C_QFWD);
  uint32_t next = 0;
  if (threadIdx.x == 0) next = tq.pop();
  for (;;) {
    if (threadIdx.x == 0) {
      s_tile = next;
      next = tq.pop();
    }
    __syncthreads();
    const uint32_t qi = s_tile;
    __syncthreads();
    if (qi >= a.T) break;
    const uint32_t gt = a.ws.torder[qi];
    const int v = view_of_tile(a.ws.views, a.V, gt);
    const ViewTab vt = a.ws.views[v];
    const uint32_t lt = gt - vt.tile_base;
    const int tx = int(lt % vt.tiles_x), ty = int(lt / vt.tiles_x);
    const int bx = tx * TS + wbx, by = ty * TS + wby;   // wave block origin (pixels)
    const int px = bx + lx, py = by + ly;
    const bool inimg = px < vt.W && py < vt.H;
    const lv_camera& cam = a.cams[v];
    const float o[3] = {cam.o[0], cam.o[1], cam.o[2]};
    const Ray ray = pixel_ray(cam, px, py);
    const uint64_t s0 = tile_begin(a, gt);
    const uint64_t s1 = tile_begin(a, gt + 1);
    const uint32_t count = uint32_t(s1 - s0);
    const uint32_t* ids = a.ws.ids + s0;

    FwdState st;
    st.T = inimg ? 1.0f : 0.0f; st.C0 = st.C1 = st.C2 = 0.0f; st.D = 0.0f; st.Tpre = 1.0f;
    st.nlast = 0;
    st.N0 = st.N1 = st.N2 = st.L = st.M = 0.0f;
    for (uint32_t cb = 0; cb < count; cb += CH) {
      const uint32_t nc = (count - cb) < uint32_t(CH) ? (count - cb) : uint32_t(CH);
      stage_chunk<CH, NT, AUX>(S, SA, a, ids, cb, nc, v, o);
      for (int k = threadIdx.x; k < CH; k += NT) s_wmax[k] = 0u;
      __syncthreads();
      build_masks<TS, CH>(S, MK, nc, tx * TS, ty * TS);
      __syncthreads();
#pragma unroll 1
      for (int w = 0; w < NW; ++w) {
        if (uint32_t(w * 64) >= nc) break;
        unsigned long long m = MK.rows[w][wby + ly] & MK.cols[w][wbx + lx];
        if (!(st.T >= a.t_eps)) m = 0;
        while (m) {
          const int jj = w * 64 + __builtin_ctzll(m);
          m &= m - 1;
          const Seg sg = slab(S, jj, ray);
          if (sg.hit) {
            const float wk = fwd_fragment<CH, AUX>(S, SA, jj, cb + uint32_t(jj), ray, sg, st);
            if (wk > 0.0f) atomicMax(&s_wmax[jj], __float_as_uint(wk));
            if (st.T < a.t_eps) break;
          }
        }
      }
      __syncthreads();
      for (uint32_t k = threadIdx.x; k < nc; k += NT) {
        const uint32_t u = s_wmax[k];
        if (u) atomicMax(reinterpret_cast<unsigned int*>(a.wmax) + (S.id[k] & kIdMask), u);
      }
      if (__syncthreads_and(st.T < a.t_eps ? 1 : 0)) break;
    }
    if (inimg) {
      const uint64_t local = uint64_t(py) * uint64_t(vt.W) + uint64_t(px);
      const uint64_t npv = uint64_t(vt.W) * uint64_t(vt.H);
      const uint64_t g = vt.pix_base + local;
      float* rgb = a.rgb + 3 * vt.pix_base + local;
      rgb[0] = fmaf(st.T, a.bg[0], st.C0);
      rgb[npv] = fmaf(st.T, a.bg[1], st.C1);
      rgb[2 * npv] = fmaf(st.T, a.bg[2], st.C2);
      a.depth[g] = st.D;
      a.alpha[g] = 1.0f - st.T;
      a.ws.nlast[g] = st.nlast;
      a.ws.tpre[g] = st.Tpre;
      if (AUX) {
        if (a.dist) a.dist[g] = st.L;
        if (a.mdepth) a.mdepth[g] = st.M;
        if (a.normal) {
          float* nm = a.normal + 3 * vt.pix_base + local;
          nm[0] = st.N0;
          nm[npv] = st.N1;
          nm[2 * npv] = st.N2;
        }
      }
    }
  }
}

// ======================================================================
// backward: back-to-front adjoint sweep.  With T_k the transmittance after
// hit k and S_k^C = sum_{j>k} w_j c_j (likewise S^D for depth):
//   dL/dtau_k = g_C . (T_k c_k - S_k^C - T_K bg) + g_D (T_k tm_k - S_k^D) + g_A T_K
//   dL/dsigma_corner += dL/dtau_k * integral of the corner's trilinear weight
//   dL/dcolour_k     += w_k g_C
// T_{k-1} = T_k exp(tau_k), starting from the transmittance saved before the
// last hit, so no per-sample state is stored.
//
// Accumulation: the sweep queues each hit (voxel, pixel, dL/dtau, weight,
// chord) in a per-wave LDS ring; 64 queued hits at a time are expanded by
// the whole wave into their 11 contributions, summed over runs of lanes on
// the same voxel (seg_reduce_rows) and added to the voxel's LDS accumulator
// by the run's last lane; each chunk is flushed with one global atomic per
// (voxel, component).
struct BwdState {
  float Tb;            // transmittance before the hit processed last
  float gC0, gC1, gC2, gD, gA;
  float base, SC0, SC1, SC2, SD;
  bool first;
  // AUX: upstream of the distortion and normal channels, the pixel's depth,
  // suffix sums of w n, of w and of w times the distortion's dL/dw
  float gL, Dt, gN0, gN1, gN2, SN0, SN1, SN2, SW, SG;
};

// Sequential part of one fragment (this lane's pixel, voxel jj), in the
// pixel's back-to-front sweep: transmittance, weight and dL/dtau.  Returns
// hit and, for a hit, what the deferred part needs: gh = dL/dtau * half
// chord, the weight wk and the chord's midpoint and half length.
template <int CH, bool AUX>
__device__ __forceinline__ bool bwd_sweep(const Stage<CH>& S, const StageAux<CH>* SA, int jj,
                                          const Ray& ray, BwdState& st, const float bg[3],
                                          float& gh, float& wk, float& tm, float& hl) {
  const Seg sg = slab(S, jj, ray);
  if (!sg.hit) return false;
  const Quad q = quad(S, jj, ray, sg);
  const float ex = __expf(-q.tau);
  const float al = opacity(q.tau, ex);
  float Tafter, Tbefore;
  if (st.first) {
    Tbefore = st.Tb;
    Tafter = st.Tb * ex;
    st.base = Tafter * (st.gA - (st.gC0 * bg[0] + st.gC1 * bg[1] + st.gC2 * bg[2]));
    st.first = false;
  } else {
    Tafter = st.Tb;
    Tbefore = st.Tb * __expf(q.tau);
  }
  wk = Tbefore * al;
  const float c0 = S.col[0][jj], c1 = S.col[1][jj], c2 = S.col[2][jj];
  float dtau = st.base + st.gD * (Tafter * q.tm - st.SD);
  dtau = fmaf(st.gC0, Tafter * c0 - st.SC0, dtau);
  dtau = fmaf(st.gC1, Tafter * c1 - st.SC1, dtau);
  dtau = fmaf(st.gC2, Tafter * c2 - st.SC2, dtau);
  if (AUX) {
    // distortion: dL/dw_k = gL (2 (tm W - S) + 2 (S' - tm W') + (4/3) w_k hl), with
    // W = 1 - T before the hit, S = D - w_k tm - S' the earlier sums, S' = SD
    // and W' = SW the later ones
    const float pre = fmaf(q.tm, 1.0f - Tbefore, -((st.Dt - wk * q.tm) - st.SD));
    const float post = fmaf(-q.tm, st.SW, st.SD);
    const float Gd = st.gL * (2.0f * (pre + post) + (4.0f / 3.0f) * wk * q.hl);
    dtau += fmaf(Gd, Tafter, -st.SG);
    st.SG = fmaf(wk, Gd, st.SG);
    st.SW += wk;
    // normal: like a colour without background
    const float n0 = SA->n[0][jj], n1 = SA->n[1][jj], n2 = SA->n[2][jj];
    dtau = fmaf(st.gN0, Tafter * n0 - st.SN0, dtau);
    dtau = fmaf(st.gN1, Tafter * n1 - st.SN1, dtau);
    dtau = fmaf(st.gN2, Tafter * n2 - st.SN2, dtau);
    st.SN0 = fmaf(wk, n0, st.SN0);
    st.SN1 = fmaf(wk, n1, st.SN1);
    st.SN2 = fmaf(wk, n2, st.SN2);
  }
  gh = dtau * q.hl;
  tm = q.tm;
  hl = q.hl;
  st.SC0 = fmaf(wk, c0, st.SC0);
  st.SC1 = fmaf(wk, c1, st.SC1);
  st.SC2 = fmaf(wk, c2, st.SC2);
  st.SD = fmaf(wk, q.tm, st.SD);
  st.Tb = Tbefore;
  return true;
}

// Deferred part of a fragment: the 8 corner-density contributions (gh times
// the trilinear corner weights summed over the two Gauss points, recomputed
// from the chord exactly as the sweep computed them) and the 3 colour
// contributions wk * dL/dC.
template <int CH>
__device__ __forceinline__ void bwd_spread(const Stage<CH>& S, int jj, const float d[3], float gh,
                                           float wk, const float gc[3], float tm, float hl,
                                           float* g) {
  const float ta = fmaf(-hl, kGL, tm), tb = fmaf(hl, kGL, tm);
  const float ie = S.inve[jj];
  float ua[3], ub[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const float du = d[ax] * ie;
    const float su = S.rlo[ax][jj] * ie;
    ua[ax] = fmaf(ta, du, -su);
    ub[ax] = fmaf(tb, du, -su);
  }
  {
    const float x1 = ua[0], y1 = ua[1], z1 = ua[2];
    const float x0 = 1.0f - x1, y0 = 1.0f - y1, z0 = 1.0f - z1;
    const float y0z0 = y0 * z0, y1z0 = y1 * z0, y0z1 = y0 * z1, y1z1 = y1 * z1;
    g[0] = x0 * y0z0; g[1] = x1 * y0z0; g[2] = x0 * y1z0; g[3] = x1 * y1z0;
    g[4] = x0 * y0z1; g[5] = x1 * y0z1; g[6] = x0 * y1z1; g[7] = x1 * y1z1;
  }
  {
    const float x1 = ub[0], y1 = ub[1], z1 = ub[2];
    const float x0 = 1.0f - x1, y0 = 1.0f - y1, z0 = 1.0f - z1;
    const float y0z0 = y0 * z0, y1z0 = y1 * z0, y0z1 = y0 * z1, y1z1 = y1 * z1;
    g[0] = gh * (g[0] + x0 * y0z0); g[1] = gh * (g[1] + x1 * y0z0);
    g[2] = gh * (g[2] + x0 * y1z0); g[3] = gh * (g[3] + x1 * y1z0);
    g[4] = gh * (g[4] + x0 * y0z1); g[5] = gh * (g[5] + x1 * y0z1);
    g[6] = gh * (g[6] + x0 * y1z1); g[7] = gh * (g[7] + x1 * y1z1);
  }
  g[8] = wk * gc[0];
  g[9] = wk * gc[1];
  g[10] = wk * gc[2];
}

// Per-wave ring of deferred fragments (kRing entries; the sweep appends at
// most 64 per step and the wave drains 64 whenever that many are queued, so
// fewer than kRing are ever pending).
constexpr int kRing = 128;

template <int CH, bool AUX>
struct BwdRing {
  uint16_t key[kRing];   // jj | pixel lane << 8 (jj < 256)
  float gh[kRing], wk[kRing], tm[kRing], hl[kRing];
  // plain instances: the unit ray direction and dL/dC of each pixel of the
  // wave; the AUX instances read those (and dL/dN) from the pixel's own lane
  // instead, which leaves them the LDS for one more wave per SIMD
  float d[AUX ? 1 : 64][3];
  float gc[AUX ? 1 : 64][3];
};

// Processes the `count` (<= 64) oldest entries of the ring with one entry per
// lane: corner and colour contributions, summed over runs of lanes on the
// same voxel, added to the chunk's LDS accumulators.  Every lane of the
// wave must call it.
// own (AUX): this lane's pixel values (unit ray direction, dL/dC, dL/dN),
// read by the entries of that pixel through a cross-lane permute.
template <int CH, bool AUX>
__device__ __forceinline__ void bwd_drain(const Stage<CH>& S, const BwdRing<CH, AUX>& R,
                                          double (*s_g)[CH], uint32_t head, uint32_t count,
                                          const float (&own)[9]) {
  constexpr int NV = AUX ? 14 : 11;
  const uint32_t lane = threadIdx.x & 63u;
  const bool valid = lane < count;
  int jj = 0;
  uint32_t p = lane, e = 0u;
  if (valid) {
    e = (head + lane) & uint32_t(kRing - 1);
    const uint32_t key = R.key[e];
    p = key >> 8;
    jj = int(key & 0xFFu);
  }
  float pv[9];
  if constexpr (AUX) {   // every lane takes part in the permute
#pragma unroll
    for (int c = 0; c < 9; ++c)
      pv[c] = __int_as_float(__builtin_amdgcn_ds_bpermute(int(p << 2), __float_as_int(own[c])));
  }
  float g[NV];
#pragma unroll
  for (int c = 0; c < NV; ++c) g[c] = 0.0f;
  if (valid) {
    if constexpr (AUX) {
      const float d[3] = {pv[0], pv[1], pv[2]};
      const float gc[3] = {pv[3], pv[4], pv[5]};
      bwd_spread(S, jj, d, R.gh[e], R.wk[e], gc, R.tm[e], R.hl[e], g);
      // dL/dn of the voxel: w times the pixel's dL/dN
      g[NV - 3] = R.wk[e] * pv[6];
      g[NV - 2] = R.wk[e] * pv[7];
      g[NV - 1] = R.wk[e] * pv[8];
    } else {
      const float d[3] = {R.d[p][0], R.d[p][1], R.d[p][2]};
      const float gc[3] = {R.gc[p][0], R.gc[p][1], R.gc[p][2]};
      bwd_spread(S, jj, d, R.gh[e], R.wk[e], gc, R.tm[e], R.hl[e], g);
    }
  }
  const bool last = seg_reduce_rows<NV>(g, jj, valid);
  if (valid && last) {
#pragma unroll
    for (int c = 0; c < NV; ++c) atomicAdd(&s_g[c][jj], double(g[c]));
  }
}

// 6 waves per SIMD where the LDS allows it (the plain chunk-64 instances: 80
// registers, a few spilled outside the sweep; 94 and 5 waves otherwise, 1.255
// against 1.19 ms on the ring workload), 5 for the AUX ones (96 registers, no
// spills; with the pixel values taken from the owning lanes their chunk-64
// LDS fits 5 workgroups: 1.60 against 1.52 ms)
template <int TS, int NW, bool AUX>
__global__ __launch_bounds__(TS* TS) __attribute__((amdgpu_waves_per_eu(AUX ? 5 : 6))) void k_composite_bwd(RasterArgs a) {
  constexpr int NT = TS * TS;
  constexpr int CH = 64 * NW;
  constexpr int BPR = TS / 8;
  constexpr int NV = AUX ? 14 : 11;   // accumulated values per voxel
  static_assert(CH <= 256, "ring keys hold the chunk position in 8 bits");
  __shared__ Stage<CH> S;
  __shared__ StageAux<AUX ? CH : 64> s_aux;
  StageAux<CH>* SA = AUX ? reinterpret_cast<StageAux<CH>*>(&s_aux) : nullptr;
  __shared__ Masks<TS, CH> MK;
  __shared__ double s_g[NV][CH];
  __shared__ BwdRing<CH, AUX> s_ring[NT / 64];
  __shared__ uint32_t s_tile, s_maxn;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lx = pix_x_of_lane(lane), ly = pix_y_of_lane(lane);
  BwdRing<CH, AUX>& ring = s_ring[wave];
  const int wbx = (wave % BPR) * 8, wby = (wave / BPR) * 8;
  const float bg[3] = {a.bg[0], a.bg[1], a.bg[2]};

  const TileQueue tq = tile_queue(a.T, a.ws.counters + C_QBWD);
  uint32_t next = 0;
  if (threadIdx.x == 0) next = tq.pop();
  for (;;) {
    if (threadIdx.x == 0) {
      s_tile = next;
      next = tq.pop();
      s_maxn = 0u;
    }
    __syncthreads();
    const uint32_t qi = s_tile;
    if (qi >= a.T) break;
    const uint32_t gt = a.ws.torder[qi];
    const int v = view_of_tile(a.ws.views, a.V, gt);
    const ViewTab vt = a.ws.views[v];
    const uint32_t lt = gt - vt.tile_base;
    const int tx = int(lt % vt.tiles_x), ty = int(lt / vt.tiles_x);
    const int bx = tx * TS + wbx, by = ty * TS + wby;
    const int px = bx + lx, py = by + ly;
    const bool inimg = px < vt.W && py < vt.H;
    const lv_camera& cam = a.cams[v];
    const float o[3] = {cam.o[0], cam.o[1], cam.o[2]};
    const Ray ray = pixel_ray(cam, px, py);
    const uint64_t s0 = tile_begin(a, gt);
    const uint32_t* ids = a.ws.ids + s0;
    float* const dden = a.ws.dden;
    float* const dcol_v = a.ws.dcol + size_t(v) * size_t(a.n) * 3u;   // this view's colour rows

    uint32_t nlast = 0;
    BwdState st;
    st.Tb = 1.0f; st.gC0 = st.gC1 = st.gC2 = st.gD = st.gA = 0.0f;
    st.base = st.SC0 = st.SC1 = st.SC2 = st.SD = 0.0f;
    st.first = true;
    st.gL = st.Dt = st.gN0 = st.gN1 = st.gN2 = 0.0f;
    st.SN0 = st.SN1 = st.SN2 = st.SW = st.SG = 0.0f;
    if (inimg) {
      const uint64_t local = uint64_t(py) * uint64_t(vt.W) + uint64_t(px);
      const uint64_t npv = uint64_t(vt.W) * uint64_t(vt.H);
      const uint64_t gp = vt.pix_base + local;
      nlast = a.ws.nlast[gp];
      st.Tb = a.ws.tpre[gp];
      const float* dr = a.d_rgb + 3 * vt.pix_base + local;
      st.gC0 = dr[0]; st.gC1 = dr[npv]; st.gC2 = dr[2 * npv];
      st.gD = a.d_depth ? a.d_depth[gp] : 0.0f;
      st.gA = a.d_alpha ? a.d_alpha[gp] : 0.0f;
      if (AUX) {
        if (a.d_dist) {
          st.gL = a.d_dist[gp];
          st.Dt = a.depth_fwd[gp];
        }
        if (a.d_normal) {
          const float* dn = a.d_normal + 3 * vt.pix_base + local;
          st.gN0 = dn[0]; st.gN1 = dn[npv]; st.gN2 = dn[2 * npv];
        }
      }
    }
    // the pixel's values the deferred part reads: in the wave's LDS (plain
    // instances) or from this lane's registers (AUX)
    float own[9];
    if constexpr (AUX) {
      own[0] = ray.d[0]; own[1] = ray.d[1]; own[2] = ray.d[2];
      own[3] = st.gC0; own[4] = st.gC1; own[5] = st.gC2;
      own[6] = st.gN0; own[7] = st.gN1; own[8] = st.gN2;
    } else {
      ring.d[lane][0] = ray.d[0]; ring.d[lane][1] = ray.d[1]; ring.d[lane][2] = ray.d[2];
      ring.gc[lane][0] = st.gC0; ring.gc[lane][1] = st.gC1; ring.gc[lane][2] = st.gC2;
    }
    if (nlast) atomicMax(&s_maxn, nlast);
    __syncthreads();
    const uint32_t maxn = s_maxn;
    __syncthreads();

    uint32_t rhead = 0u, rcount = 0u;   // the wave's ring (wave-uniform)
    const int nch = int((maxn + CH - 1) / CH);
    for (int ci = nch - 1; ci >= 0; --ci) {
      const uint32_t cb = uint32_t(ci) * CH;
      const uint32_t nc = (maxn - cb) < uint32_t(CH) ? (maxn - cb) : uint32_t(CH);
      stage_chunk<CH, NT, AUX>(S, SA, a, ids, cb, nc, v, o);
      {
        double* z = &s_g[0][0];
        for (int k = threadIdx.x; k < NV * CH; k += NT) z[k] = 0.0;
      }
      __syncthreads();
      build_masks<TS, CH>(S, MK, nc, tx * TS, ty * TS);
      __syncthreads();
#pragma unroll 1
      for (int w = NW - 1; w >= 0; --w) {
        if (uint32_t(w * 64) >= nc) continue;
        unsigned long long m = MK.rows[w][wby + ly] & MK.cols[w][wbx + lx];
        const int lim = int(nlast) - int(cb) - w * 64;
        if (lim <= 0) m = 0;
        else if (lim < 64) m &= (1ull << lim) - 1ull;
        // wave-uniform loop: each lane takes its next candidate (back to
        // front); hits are queued in the wave's ring in lane order, and the
        // wave drains 64 of them whenever that many are pending
        for (;;) {
          const bool act = m != 0;
          if (__ballot(act) == 0) break;
          // jj and the fragment values are read only where hit is set
          bool hit = false;
          int jj;
          float gh, wk, tm, hl;
          if (act) {
            const int jbit = 63 - __builtin_clzll(m);
            m &= ~(1ull << jbit);
            jj = w * 64 + jbit;
            hit = bwd_sweep<CH, AUX>(S, SA, jj, ray, st, bg, gh, wk, tm, hl);
          }
          const unsigned long long hb = __ballot(hit);
          if (hb) {
            if (hit) {
              const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                  uint32_t(hb >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(hb), 0u));
              const uint32_t e = (rhead + rcount + below) & uint32_t(kRing - 1);
              ring.key[e] = uint16_t(uint32_t(jj) | (uint32_t(lane) << 8));
              ring.gh[e] = gh;
              ring.wk[e] = wk;
              ring.tm[e] = tm;
              ring.hl[e] = hl;
            }
            rcount += uint32_t(__popcll(hb));
            if (rcount >= 64u) {
              bwd_drain(S, ring, s_g, rhead, 64u, own);
              rhead = (rhead + 64u) & uint32_t(kRing - 1);
              rcount -= 64u;
            }
          }
        }
      }
      if (rcount) {   // the rest of this chunk's fragments
        bwd_drain(S, ring, s_g, rhead, rcount, own);
        rhead = (rhead + rcount) & uint32_t(kRing - 1);
        rcount = 0u;
      }
      __syncthreads();
      if (AUX) {
        // the chunk's dL/dn of each voxel through n = -u / |u|: dL/du =
        // -(g - (g . n) n) / |u|, and du_a/dsigma_c = +-1/4 (corner bit a)
        for (uint32_t k = threadIdx.x; k < nc; k += NT) {
          const double g0 = s_g[11][k], g1 = s_g[12][k], g2 = s_g[13][k];
          const double n0 = SA->n[0][k], n1 = SA->n[1][k], n2 = SA->n[2][k];
          const double gn = g0 * n0 + g1 * n1 + g2 * n2;
          const double iu = SA->iu[k];
          s_g[11][k] = -0.25 * (g0 - gn * n0) * iu;
          s_g[12][k] = -0.25 * (g1 - gn * n1) * iu;
          s_g[13][k] = -0.25 * (g2 - gn * n2) * iu;
        }
        __syncthreads();
      }
      // flush: consecutive lanes take consecutive components of a voxel, so
      // its 8 density and 3 colour sums go out as two contiguous groups
      for (uint32_t e = threadIdx.x; e < 11u * nc; e += NT) {
        const uint32_t k = e / 11u, c = e - 11u * k;
        double sd = s_g[c][k];
        if (AUX && c < 8u)
          sd += ((c & 1u) ? s_g[11][k] : -s_g[11][k]) + ((c & 2u) ? s_g[12][k] : -s_g[12][k]) +
                ((c & 4u) ? s_g[13][k] : -s_g[13][k]);
        const float s = float(sd);
        // colour gradients stop at the clamp (channels whose raw value <= 0)
        const bool pass = c < 8u || ((S.id[k] >> (kIdBits + (c - 8u))) & 1u);
        if (s != 0.0f && pass) {
          // 32-bit offsets: ids are below 2^28
          const uint32_t id = S.id[k] & kIdMask;
          float* dst = c < 8u ? dden + (8u * id + c) : dcol_v + (3u * id + (c - 8u));
          unsafeAtomicAdd(dst, s);
        }
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------- launchers
template <typename K>
static int persistent_grid(K kernel, int nt, uint32_t T, int grid_cap) {
  int dev = 0, cus = 256, per = 1;
  if (hipGetDevice(&dev) == hipSuccess) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, nt, 0) != hipSuccess || per < 1) per = 1;
  long g = long(cus) * per;
  if (grid_cap > 0 && g > grid_cap) g = grid_cap;
  if (g > long(T)) g = long(T);
  if (g < 1) g = 1;
  return int(g);
}

template <int TS, int NW, bool AUX>
static hipError_t fwd_inst(const RasterArgs& a, int grid_cap, hipStream_t s) {
  auto k = k_composite_fwd<TS, NW, AUX>;
  const int g = persistent_grid(k, TS * TS, a.T, grid_cap);
  hipLaunchKernelGGL(k, dim3(g), dim3(TS * TS), 0, s, a);
  return hipGetLastError();
}

template <int TS, int NW, bool AUX>
static hipError_t bwd_inst(const RasterArgs& a, int grid_cap, hipStream_t s) {
  auto k = k_composite_bwd<TS, NW, AUX>;
  const int g = persistent_grid(k, TS * TS, a.T, grid_cap);
  hipLaunchKernelGGL(k, dim3(g), dim3(TS * TS), 0, s, a);
  return hipGetLastError();
}

#define LV_DISPATCH(FN, AUX, a, chunk, cap, s)                         \
  switch (a.TS * 1000 + chunk) {                                       \
    case 8064: return FN<8, 1, AUX>(a, cap, s);                        \
    case 8128: return FN<8, 2, AUX>(a, cap, s);                        \
    case 8256: return FN<8, 4, AUX>(a, cap, s);                        \
    case 16064: return FN<16, 1, AUX>(a, cap, s);                      \
    case 16128: return FN<16, 2, AUX>(a, cap, s);                      \
    case 16256: return FN<16, 4, AUX>(a, cap, s);                      \
    case 32064: return FN<32, 1, AUX>(a, cap, s);                      \
    case 32128: return FN<32, 2, AUX>(a, cap, s);                      \
    case 32256: return FN<32, 4, AUX>(a, cap, s);                      \
    default: return hipErrorInvalidValue;                              \
  }

hipError_t launch_composite_fwd(const RasterArgs& a, int chunk, int grid_cap, hipStream_t s,
                                bool aux) {
  if (a.T == 0) return hipSuccess;
  if (aux) {
    LV_DISPATCH(fwd_inst, true, a, chunk, grid_cap, s);
  }
  LV_DISPATCH(fwd_inst, false, a, chunk, grid_cap, s);
}

hipError_t launch_composite_bwd(const RasterArgs& a, int chunk, int grid_cap, hipStream_t s,
                                bool aux) {
  if (a.T == 0) return hipSuccess;
  if (aux) {
    LV_DISPATCH(bwd_inst, true, a, chunk, grid_cap, s);
  }
  LV_DISPATCH(bwd_inst, false, a, chunk, grid_cap, s);
}

}  // namespace lv

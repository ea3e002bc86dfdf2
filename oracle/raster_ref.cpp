// Reference (oracle) implementation of the differentiable sparse-voxel
// rasterizer: plain, slow, FP64.  TEST INFRASTRUCTURE ONLY: it is called by the
// tests, by the smoke check and by the CPU-baseline leg of the benchmark, never
// by the product path.  It shares no code with the HIP library.
//
// What it computes (LiteVoxel, Sec. III "Preliminaries"):
//   * rays r(t) = o + t d, t >= 0, one per pixel centre (eq. 1);
//   * voxels are axis-aligned cubes of an octree (Sec. III, "Sparse
//     Voxel/Octree Indexing"); level l has edge root_size * 2^-l;
//   * front-to-back alpha compositing T_0 = 1, w_k = T_{k-1} alpha_k,
//     T_k = T_{k-1}(1 - alpha_k), C = sum_k w_k c_k (eq. 2-4);
//   * the per-voxel maximum blending weight w_max (eq. 5).
// Opacity of a voxel along a ray is alpha = 1 - exp(-tau) with tau the exact
// integral of the trilinear density of the voxel's 8 corner values over the
// chord (the trilinear field restricted to a line is a cubic; its integral
// is taken from the expanded polynomial, not by quadrature).
// Colour is a real spherical-harmonic expansion (degree <= 3) evaluated at the
// direction from the camera centre to the voxel centre, with the constant
// term in colour units, clamped below at zero.
//
// The image path bins voxels conservatively (FP64 projected box dilated by one
// pixel) and, per pixel, sorts the intersected voxels by entry distance; the
// result is the plain definition of eq. 2-4 over every voxel the ray meets.
// The key path (ref_project_keys) reproduces the binary32 binning and the
// visibility code used to order per-tile lists.
//
// Build: g++ -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

constexpr int kLMax = 12;

struct Cam {
  double R[9];
  double o[3];
  double fx, fy, cx, cy;
  int W, H;
};

struct Scene {
  int64_t n;
  int deg;
  double root_min[3];
  double root_size;
  const uint16_t* ijk;   // [3][n]
  const uint8_t* level;  // [n]
  const double* density; // [8][n]
  const double* sh;      // [3(deg+1)^2][n]
  double edge(int64_t v) const { return std::ldexp(root_size, -int(level[v])); }
  void box(int64_t v, double b[3], double& e) const {
    e = edge(v);
    for (int a = 0; a < 3; ++a) b[a] = root_min[a] + double(ijk[a * n + v]) * e;
  }
};

std::vector<Cam> load_cams(int nv, const float* cams, const int32_t* wh) {
  // cams: 17 floats per view: R (row-major 3x3), o (3), fx, fy, cx, cy
  std::vector<Cam> out(nv);
  for (int i = 0; i < nv; ++i) {
    const float* c = cams + 17 * i;
    for (int k = 0; k < 9; ++k) out[i].R[k] = c[k];
    for (int k = 0; k < 3; ++k) out[i].o[k] = c[9 + k];
    out[i].fx = c[12]; out[i].fy = c[13]; out[i].cx = c[14]; out[i].cy = c[15];
    out[i].W = wh[2 * i]; out[i].H = wh[2 * i + 1];
  }
  return out;
}

// ---------------------------------------------------------------- SH basis
// Real orthonormal spherical harmonics with the Condon-Shortley phase, polar
// axis z, azimuth measured from x towards y, index i = l*l + l + m.  Built
// from associated Legendre functions (recurrence in l) rather than Cartesian
// polynomials.
double fact(int k) { double r = 1.0; for (int i = 2; i <= k; ++i) r *= i; return r; }

double assoc_legendre(int l, int m, double x) {  // m >= 0, includes (-1)^m
  double pmm = 1.0;
  double s = std::sqrt(std::max(0.0, 1.0 - x * x));
  for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s;
  if (l == m) return pmm;
  double pm1 = x * (2.0 * m + 1.0) * pmm;
  if (l == m + 1) return pm1;
  double pl = 0.0;
  for (int ll = m + 2; ll <= l; ++ll) {
    pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
    pmm = pm1; pm1 = pl;
  }
  return pl;
}

void sh_basis(int deg, const double d[3], double* Y) {
  const double kPi = 3.14159265358979323846;
  double ct = d[2];
  double phi = std::atan2(d[1], d[0]);
  for (int l = 0; l <= deg; ++l) {
    for (int m = -l; m <= l; ++m) {
      int am = std::abs(m);
      double K = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * fact(l - am) / fact(l + am));
      double P = assoc_legendre(l, am, ct);
      double y;
      if (m > 0) y = std::sqrt(2.0) * K * std::cos(am * phi) * P;
      else if (m < 0) y = std::sqrt(2.0) * K * std::sin(am * phi) * P;
      else y = K * P;
      Y[l * l + l + m] = y;
    }
  }
}

// colour of voxel v seen from camera centre o (DC term in colour units)
void voxel_colour(const Scene& sc, int64_t v, const double o[3], double c[3],
                  double raw[3], double Y[16]) {
  double b[3], e;
  sc.box(v, b, e);
  double d[3], nrm = 0.0;
  for (int a = 0; a < 3; ++a) { d[a] = b[a] + 0.5 * e - o[a]; nrm += d[a] * d[a]; }
  nrm = std::sqrt(nrm);
  for (int a = 0; a < 3; ++a) d[a] /= nrm;
  sh_basis(sc.deg, d, Y);
  Y[0] = 1.0;  // constant term carries the colour directly
  int nb = (sc.deg + 1) * (sc.deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += Y[i] * sc.sh[(i * 3 + ch) * sc.n + v];
    raw[ch] = s;
    c[ch] = s > 0.0 ? s : 0.0;
  }
}

// ------------------------------------------------------------- ray / voxel
void pixel_ray(const Cam& c, int px, int py, double d[3]) {
  double dc[3] = {(px + 0.5 - c.cx) / c.fx, (py + 0.5 - c.cy) / c.fy, 1.0};
  double n = 0.0;
  for (int a = 0; a < 3; ++a) {
    // world direction = R^T d_cam
    d[a] = c.R[0 * 3 + a] * dc[0] + c.R[1 * 3 + a] * dc[1] + c.R[2 * 3 + a] * dc[2];
    n += d[a] * d[a];
  }
  n = std::sqrt(n);
  for (int a = 0; a < 3; ++a) d[a] /= n;
}

// slab test against the closed box [b, b+e]; returns true and the entry/exit
// distances (t_in clamped to the ray origin) when the chord has positive length
bool slab(const double o[3], const double d[3], const double b[3], double e,
          double& tin, double& tout) {
  double lo = 0.0, hi = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < b[a] || o[a] > b[a] + e) return false;
      continue;
    }
    double t1 = (b[a] - o[a]) / d[a], t2 = (b[a] + e - o[a]) / d[a];
    lo = std::max(lo, std::min(t1, t2));
    hi = std::min(hi, std::max(t1, t2));
  }
  tin = lo; tout = hi;
  return tout > tin;
}

// beta[c] = integral over the chord of the trilinear weight of corner c
// (corner c = x + 2y + 4z); tau = sum_c sigma_c beta[c].
void corner_integrals(const double o[3], const double d[3], const double b[3], double e,
                      double tin, double tout, double beta[8]) {
  double len = tout - tin;
  double A[3], B[3];
  for (int a = 0; a < 3; ++a) {
    A[a] = (o[a] + tin * d[a] - b[a]) / e;  // u_a at s = 0
    B[a] = len * d[a] / e;                 // du_a / ds
  }
  for (int c = 0; c < 8; ++c) {
    // product of three linear factors f_a(s) = p_a + q_a s
    double poly[4] = {1.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) {
      int bit = (c >> a) & 1;
      double p = bit ? A[a] : 1.0 - A[a];
      double q = bit ? B[a] : -B[a];
      double np[4] = {0, 0, 0, 0};
      for (int k = 0; k < 3; ++k) { np[k] += poly[k] * p; np[k + 1] += poly[k] * q; }
      for (int k = 0; k < 4; ++k) poly[k] = np[k];
    }
    beta[c] = len * (poly[0] + poly[1] / 2.0 + poly[2] / 3.0 + poly[3] / 4.0);
  }
}

// -------------------------------------------------- conservative binning
constexpr int kRefTile = 16;

struct ViewBins {
  int tx, ty;
  std::vector<std::vector<int64_t>> lists;  // per tile: candidate voxel ids
};

void project_box_fp64(const Cam& c, const double b[3], double e, bool& cull,
                      bool& whole, double& u0, double& u1, double& v0, double& v1) {
  cull = false; whole = false;
  u0 = v0 = INFINITY; u1 = v1 = -INFINITY;
  int behind = 0;
  for (int k = 0; k < 8; ++k) {
    double p[3] = {b[0] + ((k >> 0) & 1) * e, b[1] + ((k >> 1) & 1) * e, b[2] + ((k >> 2) & 1) * e};
    double q[3] = {p[0] - c.o[0], p[1] - c.o[1], p[2] - c.o[2]};
    double xc = c.R[0] * q[0] + c.R[1] * q[1] + c.R[2] * q[2];
    double yc = c.R[3] * q[0] + c.R[4] * q[1] + c.R[5] * q[2];
    double zc = c.R[6] * q[0] + c.R[7] * q[1] + c.R[8] * q[2];
    if (zc <= 0.0) { ++behind; continue; }
    double u = c.fx * xc / zc + c.cx, v = c.fy * yc / zc + c.cy;
    u0 = std::min(u0, u); u1 = std::max(u1, u); v0 = std::min(v0, v); v1 = std::max(v1, v);
  }
  if (behind == 8) { cull = true; return; }
  if (behind > 0) { whole = true; }
}

ViewBins bin_view(const Scene& sc, const Cam& c) {
  ViewBins vb;
  vb.tx = (c.W + kRefTile - 1) / kRefTile;
  vb.ty = (c.H + kRefTile - 1) / kRefTile;
  vb.lists.assign(size_t(vb.tx) * vb.ty, {});
  for (int64_t v = 0; v < sc.n; ++v) {
    double b[3], e;
    sc.box(v, b, e);
    bool cull, whole;
    double u0, u1, v0, v1;
    project_box_fp64(c, b, e, cull, whole, u0, u1, v0, v1);
    if (cull) continue;
    int x0, x1, y0, y1;
    if (whole) { x0 = 0; x1 = c.W - 1; y0 = 0; y1 = c.H - 1; }
    else {
      // pixels whose centre lies within the box dilated by one pixel
      double fx0 = std::ceil(u0 - 1.5), fx1 = std::floor(u1 + 0.5);
      double fy0 = std::ceil(v0 - 1.5), fy1 = std::floor(v1 + 0.5);
      fx0 = std::max(fx0, 0.0); fy0 = std::max(fy0, 0.0);
      fx1 = std::min(fx1, double(c.W - 1)); fy1 = std::min(fy1, double(c.H - 1));
      if (fx0 > fx1 || fy0 > fy1) continue;
      x0 = int(fx0); x1 = int(fx1); y0 = int(fy0); y1 = int(fy1);
    }
    for (int ty = y0 / kRefTile; ty <= y1 / kRefTile; ++ty)
      for (int tx = x0 / kRefTile; tx <= x1 / kRefTile; ++tx)
        vb.lists[size_t(ty) * vb.tx + tx].push_back(v);
  }
  return vb;
}

struct Hit {
  int64_t v;
  double tin, tout, tau, alpha;
  double beta[8];
};

// all voxels met by the ray of pixel (px, py), sorted front to back
void trace(const Scene& sc, const Cam& c, const ViewBins& vb, int px, int py,
           std::vector<Hit>& hits, bool want_beta) {
  hits.clear();
  double d[3];
  pixel_ray(c, px, py, d);
  const auto& lst = vb.lists[size_t(py / kRefTile) * vb.tx + px / kRefTile];
  for (int64_t v : lst) {
    double b[3], e, tin, tout;
    sc.box(v, b, e);
    if (!slab(c.o, d, b, e, tin, tout)) continue;
    Hit h;
    h.v = v; h.tin = tin; h.tout = tout;
    corner_integrals(c.o, d, b, e, tin, tout, h.beta);
    double tau = 0.0;
    for (int k = 0; k < 8; ++k) tau += sc.density[k * sc.n + v] * h.beta[k];
    h.tau = tau;
    h.alpha = -std::expm1(-tau);
    if (!want_beta) std::memset(h.beta, 0, sizeof(h.beta));
    hits.push_back(h);
  }
  std::sort(hits.begin(), hits.end(), [](const Hit& a, const Hit& b) { return a.tin < b.tin; });
}

void atomic_max_double(double* p, double val) {
  auto* ap = reinterpret_cast<std::atomic<uint64_t>*>(p);
  uint64_t cur = ap->load();
  for (;;) {
    double cd;
    std::memcpy(&cd, &cur, 8);
    if (!(val > cd)) return;
    uint64_t nv;
    std::memcpy(&nv, &val, 8);
    if (ap->compare_exchange_weak(cur, nv)) return;
  }
}

Scene make_scene(int64_t n, int deg, const float* root_min, double root_size,
                 const uint16_t* ijk, const uint8_t* level, const double* density,
                 const double* sh) {
  Scene sc;
  sc.n = n; sc.deg = deg;
  for (int a = 0; a < 3; ++a) sc.root_min[a] = root_min[a];
  sc.root_size = root_size;
  sc.ijk = ijk; sc.level = level; sc.density = density; sc.sh = sh;
  return sc;
}

// pixel list helper: global pixel index -> (view, px, py)
struct PixLoc { int view, px, py; };

std::vector<int64_t> pix_offsets(const std::vector<Cam>& cams) {
  std::vector<int64_t> off(cams.size() + 1, 0);
  for (size_t i = 0; i < cams.size(); ++i) off[i + 1] = off[i] + int64_t(cams[i].W) * cams[i].H;
  return off;
}

PixLoc locate(const std::vector<int64_t>& off, const std::vector<Cam>& cams, int64_t g) {
  int v = int(std::upper_bound(off.begin(), off.end(), g) - off.begin()) - 1;
  int64_t r = g - off[v];
  return PixLoc{v, int(r % cams[v].W), int(r / cams[v].W)};
}

// ------------------------------------------------------- auxiliary channels
// Render channels behind the auxiliary terms of the training objective that
// the paper names (eq. 6 and eq. 17: ray-space distortion, depth-normal
// consistency; transmittance concentration acts on alpha and needs none).
// The paper defines none of them; readings used here:
//   distortion  Ld = sum_i sum_j w_i w_j |tm_i - tm_j| + (1/3) sum_i w_i^2 l_i
//               over the hits of the ray, tm the chord midpoint, l the chord
//               length (the segment-based distortion of Mip-NeRF 360 with
//               ray distance as the coordinate);
//   normal      N = sum_k w_k n_k, n_v = -g / |g| with g the gradient of the
//               voxel's trilinear density at the cell centre (0 when g = 0).

// u = gradient of the trilinear density at the cell centre in cell units:
// u_a = 1/4 sum over the cell's 4 edges along axis a of (upper - lower corner
// value), the exact derivative there.  n = -u / |u| (0 if u = 0).
void voxel_normal(const Scene& sc, int64_t v, double u[3], double& ulen, double nrm[3]) {
  double q = 0.0;
  for (int a = 0; a < 3; ++a) {
    double s = 0.0;
    for (int c = 0; c < 8; ++c) s += (((c >> a) & 1) ? 1.0 : -1.0) * sc.density[c * sc.n + v];
    u[a] = 0.25 * s;
    q += u[a] * u[a];
  }
  ulen = std::sqrt(q);
  for (int a = 0; a < 3; ++a) nrm[a] = ulen > 0.0 ? -u[a] / ulen : 0.0;
}

// weights, chord midpoints and lengths of a pixel's hits (front to back),
// and the transmittance after each hit
void hit_weights(const std::vector<Hit>& hits, std::vector<double>& w, std::vector<double>& tm,
                 std::vector<double>& len, std::vector<double>& Ta) {
  size_t K = hits.size();
  w.assign(K, 0.0); tm.assign(K, 0.0); len.assign(K, 0.0); Ta.assign(K, 0.0);
  double T = 1.0;
  for (size_t k = 0; k < K; ++k) {
    w[k] = T * hits[k].alpha;
    tm[k] = 0.5 * (hits[k].tin + hits[k].tout);
    len[k] = hits[k].tout - hits[k].tin;
    T *= std::exp(-hits[k].tau);
    Ta[k] = T;
  }
}

}  // namespace

extern "C" {

// Real SH basis (degree deg, orthonormal, Condon-Shortley) at n unit directions.
void ref_sh_basis(int64_t n, int deg, const double* dirs, double* out) {
  int nb = (deg + 1) * (deg + 1);
  for (int64_t i = 0; i < n; ++i) sh_basis(deg, dirs + 3 * i, out + nb * i);
}

// Forward render, eq. 1-5.  Pixels: all (pix_list == nullptr) or the listed
// global indices (views packed in order, row-major within a view).
// Outputs: rgb [3][P] per view block (view v at 3*off[v]), depth [P], alpha [P],
// n_hits [P] (nullable); wmax [n] is max-combined with its input.
int ref_render(int64_t n, int deg, const float* root_min, double root_size,
               const uint16_t* ijk, const uint8_t* level, const double* density,
               const double* sh, int n_views, const float* cams, const int32_t* wh,
               const double* bg, const int64_t* pix_list, int64_t n_list,
               double* rgb, double* depth, double* alpha, int32_t* n_hits,
               double* wmax, int n_threads) {
  Scene sc = make_scene(n, deg, root_min, root_size, ijk, level, density, sh);
  auto C = load_cams(n_views, cams, wh);
  auto off = pix_offsets(C);
  std::vector<ViewBins> bins(n_views);
  for (int i = 0; i < n_views; ++i) bins[i] = bin_view(sc, C[i]);
  int64_t total = pix_list ? n_list : off[n_views];
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
  {
    std::vector<Hit> hits;
    std::vector<std::vector<double>> col_cache;  // unused: colours are recomputed
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < total; ++k) {
      int64_t g = pix_list ? pix_list[k] : k;
      PixLoc pl = locate(off, C, g);
      const Cam& cam = C[pl.view];
      trace(sc, cam, bins[pl.view], pl.px, pl.py, hits, false);
      double d[3];
      pixel_ray(cam, pl.px, pl.py, d);
      double T = 1.0, acc[3] = {0, 0, 0}, dep = 0.0;
      for (const Hit& h : hits) {
        double c[3], raw[3], Y[16];
        voxel_colour(sc, h.v, cam.o, c, raw, Y);
        double w = T * h.alpha;
        for (int ch = 0; ch < 3; ++ch) acc[ch] += w * c[ch];
        dep += w * 0.5 * (h.tin + h.tout);
        if (wmax) atomic_max_double(&wmax[h.v], w);
        T *= std::exp(-h.tau);
      }
      int64_t local = g - off[pl.view];
      int64_t npv = int64_t(cam.W) * cam.H;
      for (int ch = 0; ch < 3; ++ch)
        rgb[3 * off[pl.view] + ch * npv + local] = acc[ch] + T * bg[ch];
      depth[g] = dep;
      alpha[g] = 1.0 - T;
      if (n_hits) n_hits[g] = int32_t(hits.size());
    }
  }
  return 0;
}

// Forward render with the auxiliary channels: everything ref_render writes
// (rgb, depth, alpha, wmax) plus dist [P] (the distortion Ld of each pixel)
// and normal (the rendered normal N, per view [3][H][W] at 3*off[v]).
int ref_render_aux(int64_t n, int deg, const float* root_min, double root_size,
                   const uint16_t* ijk, const uint8_t* level, const double* density,
                   const double* sh, int n_views, const float* cams, const int32_t* wh,
                   const double* bg, double* rgb, double* depth, double* alpha, double* dist,
                   double* normal, double* wmax, int n_threads) {
  Scene sc = make_scene(n, deg, root_min, root_size, ijk, level, density, sh);
  auto C = load_cams(n_views, cams, wh);
  auto off = pix_offsets(C);
  std::vector<ViewBins> bins(n_views);
  for (int i = 0; i < n_views; ++i) bins[i] = bin_view(sc, C[i]);
  int64_t total = off[n_views];
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
  {
    std::vector<Hit> hits;
    std::vector<double> w, tm, len, Ta;
#pragma omp for schedule(dynamic, 256)
    for (int64_t g = 0; g < total; ++g) {
      PixLoc pl = locate(off, C, g);
      const Cam& cam = C[pl.view];
      trace(sc, cam, bins[pl.view], pl.px, pl.py, hits, false);
      hit_weights(hits, w, tm, len, Ta);
      size_t K = hits.size();
      double TK = K ? Ta[K - 1] : 1.0;
      double acc[3] = {0, 0, 0}, dep = 0.0, nr[3] = {0, 0, 0}, ld = 0.0;
      for (size_t k = 0; k < K; ++k) {
        double c[3], raw[3], Y[16], u[3], ul, nv[3];
        voxel_colour(sc, hits[k].v, cam.o, c, raw, Y);
        voxel_normal(sc, hits[k].v, u, ul, nv);
        for (int ch = 0; ch < 3; ++ch) { acc[ch] += w[k] * c[ch]; nr[ch] += w[k] * nv[ch]; }
        dep += w[k] * tm[k];
        if (wmax) atomic_max_double(&wmax[hits[k].v], w[k]);
        for (size_t j = 0; j < K; ++j) ld += w[k] * w[j] * std::fabs(tm[k] - tm[j]);
        ld += w[k] * w[k] * len[k] / 3.0;
      }
      int64_t local = g - off[pl.view];
      int64_t npv = int64_t(cam.W) * cam.H;
      for (int ch = 0; ch < 3; ++ch) {
        rgb[3 * off[pl.view] + ch * npv + local] = acc[ch] + TK * bg[ch];
        normal[3 * off[pl.view] + ch * npv + local] = nr[ch];
      }
      depth[g] = dep;
      alpha[g] = 1.0 - TK;
      dist[g] = ld;
    }
  }
  return 0;
}

// Median depth per pixel (the depth the median-based depth-normal term of
// eq. 17 reads; reading): the chord midpoint of the first hit after which the
// transmittance is at most t_half (1/2: half the opacity accumulated), 0 when
// no hit takes it there.  It moves only when the crossing jumps to another
// hit, so it passes no gradient to the densities.
int ref_median_depth(int64_t n, int deg, const float* root_min, double root_size,
                     const uint16_t* ijk, const uint8_t* level, const double* density,
                     const double* sh, int n_views, const float* cams, const int32_t* wh,
                     double t_half, double* mdepth, int n_threads) {
  Scene sc = make_scene(n, deg, root_min, root_size, ijk, level, density, sh);
  auto C = load_cams(n_views, cams, wh);
  auto off = pix_offsets(C);
  std::vector<ViewBins> bins(n_views);
  for (int i = 0; i < n_views; ++i) bins[i] = bin_view(sc, C[i]);
  int64_t total = off[n_views];
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
  {
    std::vector<Hit> hits;
    std::vector<double> w, tm, len, Ta;
#pragma omp for schedule(dynamic, 256)
    for (int64_t g = 0; g < total; ++g) {
      PixLoc pl = locate(off, C, g);
      trace(sc, C[pl.view], bins[pl.view], pl.px, pl.py, hits, false);
      hit_weights(hits, w, tm, len, Ta);
      double md = 0.0;
      for (size_t k = 0; k < hits.size(); ++k)
        if (Ta[k] <= t_half) {
          md = tm[k];
          break;
        }
      mdepth[g] = md;
    }
  }
  return 0;
}

// Analytic gradient with the auxiliary channels.  Upstream per pixel:
// g_rgb (rgb layout), g_depth, g_alpha, g_dist [P], g_normal (rgb layout);
// every pointer but g_rgb may be NULL.  With G_k = dL/dw_k (colour, depth,
// distortion and normal terms),
//   dL/dtau_k = T_k G_k - sum_{j>k} w_j G_j + T_K (g_A - g_C . bg)
// (dw_k/dtau_k = T_k, dw_j/dtau_k = -w_j for j > k), spread over the corner
// densities by the chord integrals of their trilinear weights; the normal
// term adds w_k g_N to dL/dn_v, carried through n = -u/|u| and u (linear in
// the corner values) to the densities.  Outputs overwritten: d_density
// [8][n], d_sh [3(deg+1)^2][n].
int ref_backward_aux(int64_t n, int deg, const float* root_min, double root_size,
                     const uint16_t* ijk, const uint8_t* level, const double* density,
                     const double* sh, int n_views, const float* cams, const int32_t* wh,
                     const double* bg, const double* g_rgb, const double* g_depth,
                     const double* g_alpha, const double* g_dist, const double* g_normal,
                     double* d_density, double* d_sh, int n_threads) {
  Scene sc = make_scene(n, deg, root_min, root_size, ijk, level, density, sh);
  auto C = load_cams(n_views, cams, wh);
  auto off = pix_offsets(C);
  std::vector<ViewBins> bins(n_views);
  for (int i = 0; i < n_views; ++i) bins[i] = bin_view(sc, C[i]);
  int nb = (deg + 1) * (deg + 1);
  std::memset(d_density, 0, sizeof(double) * 8 * n);
  std::memset(d_sh, 0, sizeof(double) * 3 * nb * n);
  std::vector<double> d_col(size_t(n_views) * n * 3, 0.0);
  std::vector<double> d_nrm(size_t(n) * 3, 0.0);
  int64_t total = off[n_views];
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
  {
    std::vector<Hit> hits;
    std::vector<double> w, tm, len, Ta, G;
#pragma omp for schedule(dynamic, 256)
    for (int64_t g = 0; g < total; ++g) {
      PixLoc pl = locate(off, C, g);
      const Cam& cam = C[pl.view];
      int64_t local = g - off[pl.view];
      int64_t npv = int64_t(cam.W) * cam.H;
      double gC[3], gN[3] = {0, 0, 0};
      for (int ch = 0; ch < 3; ++ch) {
        gC[ch] = g_rgb[3 * off[pl.view] + ch * npv + local];
        if (g_normal) gN[ch] = g_normal[3 * off[pl.view] + ch * npv + local];
      }
      double gD = g_depth ? g_depth[g] : 0.0;
      double gA = g_alpha ? g_alpha[g] : 0.0;
      double gL = g_dist ? g_dist[g] : 0.0;
      trace(sc, cam, bins[pl.view], pl.px, pl.py, hits, true);
      hit_weights(hits, w, tm, len, Ta);
      size_t K = hits.size();
      double TK = K ? Ta[K - 1] : 1.0;
      G.assign(K, 0.0);
      for (size_t k = 0; k < K; ++k) {
        double c[3], raw[3], Y[16], u[3], ul, nv[3];
        voxel_colour(sc, hits[k].v, cam.o, c, raw, Y);
        voxel_normal(sc, hits[k].v, u, ul, nv);
        double Gk = gD * tm[k];
        for (int ch = 0; ch < 3; ++ch) Gk += gC[ch] * c[ch] + gN[ch] * nv[ch];
        double dd = 0.0;
        for (size_t j = 0; j < K; ++j) dd += w[j] * std::fabs(tm[k] - tm[j]);
        Gk += gL * (2.0 * dd + 2.0 * w[k] * len[k] / 3.0);
        G[k] = Gk;
        for (int ch = 0; ch < 3; ++ch) {
#pragma omp atomic
          d_col[(size_t(pl.view) * n + hits[k].v) * 3 + ch] += w[k] * gC[ch];
#pragma omp atomic
          d_nrm[size_t(hits[k].v) * 3 + ch] += w[k] * gN[ch];
        }
      }
      double base = TK * (gA - (gC[0] * bg[0] + gC[1] * bg[1] + gC[2] * bg[2]));
      for (size_t k = 0; k < K; ++k) {
        double later = 0.0;
        for (size_t j = k + 1; j < K; ++j) later += w[j] * G[j];
        double dtau = Ta[k] * G[k] - later + base;
        for (int c = 0; c < 8; ++c) {
#pragma omp atomic
          d_density[c * n + hits[k].v] += dtau * hits[k].beta[c];
        }
      }
    }
  }
  // normal -> corner densities: dn/du = -(I - u u^T / |u|^2) / |u|,
  // du_a/dsigma_c = +1/4 (corner bit a set) or -1/4
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    const double* gn = &d_nrm[size_t(v) * 3];
    if (gn[0] == 0.0 && gn[1] == 0.0 && gn[2] == 0.0) continue;
    double u[3], ul, nv[3];
    voxel_normal(sc, v, u, ul, nv);
    if (!(ul > 0.0)) continue;
    double ug = (u[0] * gn[0] + u[1] * gn[1] + u[2] * gn[2]) / (ul * ul);
    double gu[3];
    for (int a = 0; a < 3; ++a) gu[a] = -(gn[a] - u[a] * ug) / ul;
    for (int c = 0; c < 8; ++c)
      for (int a = 0; a < 3; ++a) d_density[c * n + v] += 0.25 * (((c >> a) & 1) ? 1.0 : -1.0) * gu[a];
  }
  // colour -> SH coefficients (through the clamp at zero)
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    for (int vi = 0; vi < n_views; ++vi) {
      const double* dc = &d_col[(size_t(vi) * n + v) * 3];
      if (dc[0] == 0.0 && dc[1] == 0.0 && dc[2] == 0.0) continue;
      double c[3], raw[3], Y[16];
      voxel_colour(sc, v, C[vi].o, c, raw, Y);
      for (int ch = 0; ch < 3; ++ch) {
        if (!(raw[ch] > 0.0)) continue;
        for (int i = 0; i < nb; ++i) d_sh[(i * 3 + ch) * n + v] += Y[i] * dc[ch];
      }
    }
  }
  return 0;
}

// Per-hit trace of one pixel ray, front to back (for invariants and the
// visibility-order pin).  Returns the number of hits (<= cap written).
int ref_trace_pixel(int64_t n, int deg, const float* root_min, double root_size,
                    const uint16_t* ijk, const uint8_t* level, const double* density,
                    const double* sh, const float* cam, const int32_t* wh, int px, int py,
                    int cap, int64_t* vid, double* tin, double* tout, double* tau,
                    double* w, double* T_after) {
  Scene sc = make_scene(n, deg, root_min, root_size, ijk, level, density, sh);
  auto C = load_cams(1, cam, wh);
  ViewBins vb = bin_view(sc, C[0]);
  std::vector<Hit> hits;
  trace(sc, C[0], vb, px, py, hits, false);
  double T = 1.0;
  int k = 0;
  for (const Hit& h : hits) {
    double wk = T * h.alpha;
    T *= std::exp(-h.tau);
    if (k < cap) {
      vid[k] = h.v; tin[k] = h.tin; tout[k] = h.tout; tau[k] = h.tau; w[k] = wk; T_after[k] = T;
    }
    ++k;
  }
  return k;
}

// Analytic gradient of a loss L given dL/d(rgb), dL/d(depth), dL/d(alpha) per
// pixel (the adjoint of eq. 2-4 with the colour and opacity models above).
// Only pixels in pix_list (or all) contribute.  Outputs (overwritten):
// d_density [8][n], d_sh [3(deg+1)^2][n].
int ref_backward(int64_t n, int deg, const float* root_min, double root_size,
                 const uint16_t* ijk, const uint8_t* level, const double* density,
                 const double* sh, int n_views, const float* cams, const int32_t* wh,
                 const double* bg, const int64_t* pix_list, int64_t n_list,
                 const double* g_rgb, const double* g_depth, const double* g_alpha,
                 double* d_density, double* d_sh, int n_threads) {
  Scene sc = make_scene(n, deg, root_min, root_size, ijk, level, density, sh);
  auto C = load_cams(n_views, cams, wh);
  auto off = pix_offsets(C);
  std::vector<ViewBins> bins(n_views);
  for (int i = 0; i < n_views; ++i) bins[i] = bin_view(sc, C[i]);
  int nb = (deg + 1) * (deg + 1);
  std::memset(d_density, 0, sizeof(double) * 8 * n);
  std::memset(d_sh, 0, sizeof(double) * 3 * nb * n);
  // dL/d(colour) per (view, voxel)
  std::vector<double> d_col(size_t(n_views) * n * 3, 0.0);
  int64_t total = pix_list ? n_list : off[n_views];
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel
  {
    std::vector<Hit> hits;
    std::vector<double> Tb, wv, cv, tm;
#pragma omp for schedule(dynamic, 256)
    for (int64_t k = 0; k < total; ++k) {
      int64_t g = pix_list ? pix_list[k] : k;
      PixLoc pl = locate(off, C, g);
      const Cam& cam = C[pl.view];
      int64_t local = g - off[pl.view];
      int64_t npv = int64_t(cam.W) * cam.H;
      double gC[3];
      for (int ch = 0; ch < 3; ++ch) gC[ch] = g_rgb[3 * off[pl.view] + ch * npv + local];
      double gD = g_depth ? g_depth[g] : 0.0;
      double gA = g_alpha ? g_alpha[g] : 0.0;
      trace(sc, cam, bins[pl.view], pl.px, pl.py, hits, true);
      size_t K = hits.size();
      Tb.assign(K + 1, 1.0); wv.assign(K, 0.0); cv.assign(3 * K, 0.0); tm.assign(K, 0.0);
      for (size_t j = 0; j < K; ++j) {
        double raw[3], Y[16];
        voxel_colour(sc, hits[j].v, cam.o, &cv[3 * j], raw, Y);
        wv[j] = Tb[j] * hits[j].alpha;
        Tb[j + 1] = Tb[j] * std::exp(-hits[j].tau);
        tm[j] = 0.5 * (hits[j].tin + hits[j].tout);
      }
      double TK = Tb[K];
      double SC[3] = {0, 0, 0}, SD = 0.0;
      for (size_t jj = K; jj-- > 0;) {
        const Hit& h = hits[jj];
        double Tk = Tb[jj + 1];
        double dtau = gD * (Tk * tm[jj] - SD) + gA * TK;
        for (int ch = 0; ch < 3; ++ch) dtau += gC[ch] * (Tk * cv[3 * jj + ch] - SC[ch] - TK * bg[ch]);
        for (int c = 0; c < 8; ++c) {
#pragma omp atomic
          d_density[c * n + h.v] += dtau * h.beta[c];
        }
        for (int ch = 0; ch < 3; ++ch) {
#pragma omp atomic
          d_col[(size_t(pl.view) * n + h.v) * 3 + ch] += wv[jj] * gC[ch];
        }
        for (int ch = 0; ch < 3; ++ch) SC[ch] += wv[jj] * cv[3 * jj + ch];
        SD += wv[jj] * tm[jj];
      }
    }
  }
  // colour -> SH coefficients (through the clamp at zero)
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) {
    for (int vi = 0; vi < n_views; ++vi) {
      const double* dc = &d_col[(size_t(vi) * n + v) * 3];
      if (dc[0] == 0.0 && dc[1] == 0.0 && dc[2] == 0.0) continue;
      double c[3], raw[3], Y[16];
      voxel_colour(sc, v, C[vi].o, c, raw, Y);
      for (int ch = 0; ch < 3; ++ch) {
        if (!(raw[ch] > 0.0)) continue;
        for (int i = 0; i < nb; ++i) d_sh[(i * 3 + ch) * n + v] += Y[i] * dc[ch];
      }
    }
  }
  return 0;
}

// Pixels whose centre lies within the conservatively projected box of the
// listed voxels (every pixel whose ray can hit them), as global indices into
// out (cap entries); returns the count (may exceed cap).
int64_t ref_footprint_pixels(int64_t n, const float* root_min, double root_size,
                             const uint16_t* ijk, const uint8_t* level, int n_views,
                             const float* cams, const int32_t* wh, const int64_t* vox,
                             int64_t n_vox, int64_t* out, int64_t cap) {
  Scene sc = make_scene(n, 0, root_min, root_size, ijk, level, nullptr, nullptr);
  auto C = load_cams(n_views, cams, wh);
  auto off = pix_offsets(C);
  int64_t cnt = 0;
  for (int vi = 0; vi < n_views; ++vi) {
    const Cam& c = C[vi];
    for (int64_t k = 0; k < n_vox; ++k) {
      double b[3], e;
      sc.box(vox[k], b, e);
      bool cull, whole;
      double u0, u1, v0, v1;
      project_box_fp64(c, b, e, cull, whole, u0, u1, v0, v1);
      if (cull) continue;
      int x0 = 0, x1 = c.W - 1, y0 = 0, y1 = c.H - 1;
      if (!whole) {
        double fx0 = std::max(std::ceil(u0 - 1.5), 0.0), fx1 = std::min(std::floor(u1 + 0.5), double(c.W - 1));
        double fy0 = std::max(std::ceil(v0 - 1.5), 0.0), fy1 = std::min(std::floor(v1 + 0.5), double(c.H - 1));
        if (fx0 > fx1 || fy0 > fy1) continue;
        x0 = int(fx0); x1 = int(fx1); y0 = int(fy0); y1 = int(fy1);
      }
      for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x) {
          if (cnt < cap) out[cnt] = off[vi] + int64_t(y) * c.W + x;
          ++cnt;
        }
    }
  }
  return cnt;
}

// Colour model per (view, voxel): raw SH sum and clamped colour, [V][n][3].
int ref_voxel_colours(int64_t n, int deg, const float* root_min, double root_size,
                      const uint16_t* ijk, const uint8_t* level, const double* sh,
                      int n_views, const float* cams, const int32_t* wh,
                      double* raw_out, double* col_out) {
  Scene sc = make_scene(n, deg, root_min, root_size, ijk, level, nullptr, sh);
  auto C = load_cams(n_views, cams, wh);
  for (int vi = 0; vi < n_views; ++vi)
    for (int64_t v = 0; v < n; ++v) {
      double c[3], raw[3], Y[16];
      voxel_colour(sc, v, C[vi].o, c, raw, Y);
      for (int ch = 0; ch < 3; ++ch) {
        raw_out[(size_t(vi) * n + v) * 3 + ch] = raw[ch];
        col_out[(size_t(vi) * n + v) * 3 + ch] = c[ch];
      }
    }
  return 0;
}

// ------------------------------------------------------------------ key path
// Binary32 binning and visibility code per (view, voxel).  Every arithmetic
// step is a separately rounded IEEE binary32 operation in the order written
// (built with -ffp-contract=off): corner p = b + bit*e, q = p - o,
// x_c = (R00 q0 + R01 q1) + R02 q2 (likewise y_c, z_c), u = fx (x_c / z_c) + cx.
// A record is culled when every corner has z_c <= z_near, covers the whole
// image when some corner does, and otherwise covers the pixels whose centre
// px + 0.5 lies in [min u, max u] (likewise rows).  Tiles are TS x TS pixel
// blocks.  The visibility code orders the leaves of any octree front to back
// for rays leaving the camera centre: at each split level m (1..l) and axis a
// the child bit is flipped when the eye lies above the split plane, and the
// three flipped bits (z, y, x) of level m sit at bit 3 (12 - m) of a 36-bit code.
int ref_project_keys(int64_t n, const float* root_min, float root_size,
                     const uint16_t* ijk, const uint8_t* level, int n_views,
                     const float* cams, const int32_t* wh, float z_near,
                     uint8_t* vis, int32_t* rect /* [V][n][4]: x0,x1,y0,y1 */,
                     uint64_t* code /* [V][n] */) {
  for (int vi = 0; vi < n_views; ++vi) {
    const float* c = cams + 17 * vi;
    const int W = wh[2 * vi], H = wh[2 * vi + 1];
    float R[9], o[3], fx = c[12], fy = c[13], cx = c[14], cy = c[15];
    for (int k = 0; k < 9; ++k) R[k] = c[k];
    for (int k = 0; k < 3; ++k) o[k] = c[9 + k];
    // records are independent: one per (view, voxel)
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
      size_t r = size_t(vi) * n + v;
      int l = level[v];
      float e = std::ldexp(root_size, -l);
      float b[3];
      for (int a = 0; a < 3; ++a) b[a] = root_min[a] + float(ijk[a * n + v]) * e;
      float u0 = INFINITY, u1 = -INFINITY, v0 = INFINITY, v1 = -INFINITY;
      int near_cnt = 0;
      for (int k = 0; k < 8; ++k) {
        float p0 = (k & 1) ? b[0] + e : b[0];
        float p1 = (k & 2) ? b[1] + e : b[1];
        float p2 = (k & 4) ? b[2] + e : b[2];
        float q0 = p0 - o[0], q1 = p1 - o[1], q2 = p2 - o[2];
        float t0, t1;
        t0 = R[0] * q0; t1 = R[1] * q1; float xc = t0 + t1; t0 = R[2] * q2; xc = xc + t0;
        t0 = R[3] * q0; t1 = R[4] * q1; float yc = t0 + t1; t0 = R[5] * q2; yc = yc + t0;
        t0 = R[6] * q0; t1 = R[7] * q1; float zc = t0 + t1; t0 = R[8] * q2; zc = zc + t0;
        if (zc <= z_near) { ++near_cnt; continue; }
        float qx = xc / zc, qy = yc / zc;
        float uu = fx * qx; uu = uu + cx;
        float vv = fy * qy; vv = vv + cy;
        u0 = std::min(u0, uu); u1 = std::max(u1, uu);
        v0 = std::min(v0, vv); v1 = std::max(v1, vv);
      }
      int32_t* rr = rect + 4 * r;
      vis[r] = 0;
      rr[0] = rr[1] = rr[2] = rr[3] = 0;
      code[r] = 0;
      if (near_cnt == 8) continue;
      float fx0, fx1, fy0, fy1;
      if (near_cnt > 0) {
        fx0 = 0.0f; fx1 = float(W - 1); fy0 = 0.0f; fy1 = float(H - 1);
      } else {
        fx0 = std::ceil(u0 - 0.5f); fx1 = std::floor(u1 - 0.5f);
        fy0 = std::ceil(v0 - 0.5f); fy1 = std::floor(v1 - 0.5f);
        fx0 = std::max(fx0, 0.0f); fy0 = std::max(fy0, 0.0f);
        fx1 = std::min(fx1, float(W - 1)); fy1 = std::min(fy1, float(H - 1));
        if (fx0 > fx1 || fy0 > fy1) continue;
      }
      vis[r] = 1;
      rr[0] = int32_t(fx0); rr[1] = int32_t(fx1); rr[2] = int32_t(fy0); rr[3] = int32_t(fy1);
      uint64_t cd = 0;
      for (int m = 1; m <= l; ++m) {
        float half = std::ldexp(root_size, -m);  // child edge at split level m
        uint64_t bits = 0;
        for (int a = 0; a < 3; ++a) {
          uint32_t idx = uint32_t(ijk[a * n + v]) >> (l - m);  // index at level m
          uint32_t child = idx & 1u;
          uint32_t parent = idx >> 1;
          float plane = float(2u * parent + 1u) * half;
          plane = root_min[a] + plane;
          uint32_t flip = o[a] > plane ? 1u : 0u;
          bits |= uint64_t(child ^ flip) << a;
        }
        cd |= bits << (3 * (kLMax - m));
      }
      code[r] = cd;
    }
  }
  return 0;
}

}  // extern "C"

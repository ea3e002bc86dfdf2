// Backward tail: colour gradients of every (view, voxel) record (already
// stopped at the clamp at zero by the composite pass) are taken through the
// SH expansion to the SH coefficients, summed over views, and the
// voxel-major corner-density gradient the composite pass accumulated is
// taken through the density activation to the stored values: transposed
// into the caller's [8][n] rows (dense layout), or added to the shared grid
// points the corners read (grid-point layout, one atomic per corner).  One
// thread per voxel; the dense rows are written coalesced and fully
// overwritten.
#include "lv_common.h"

namespace lv {

hipError_t launch_bwd_setup(const RasterArgs& a, hipStream_t s) {
  FillSet f;
  f.count = 0;
  auto add = [&f](void* p, uint64_t n) {
    f.p[f.count] = static_cast<uint32_t*>(p);
    f.n[f.count] = n;
    f.v[f.count] = 0u;
    ++f.count;
  };
  add(a.ws.dden, 8ull * uint64_t(a.n));
  add(a.ws.dcol, 3ull * uint64_t(a.n) * uint64_t(a.V));
  add(a.ws.counters + C_QBWD, uint64_t(kQueues) * kQueueStride);
  // grid points accumulate the gradients of the corners that read them
  if (a.corner_idx) add(a.d_density, uint64_t(a.n_grid));
  return launch_fill_set(f, s);
}

// GENERIC: grid-point layout or a density activation
template <int DEG, bool GENERIC>
__global__ __launch_bounds__(256) void k_sh_bwd(RasterArgs a) {
  constexpr int NB = (DEG + 1) * (DEG + 1);
  const int64_t n = a.n;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  {
    const float4 d0 = reinterpret_cast<const float4*>(a.ws.dden)[2 * i];
    const float4 d1 = reinterpret_cast<const float4*>(a.ws.dden)[2 * i + 1];
    const float dd[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
    if (!GENERIC) {
#pragma unroll
      for (int c = 0; c < 8; ++c) a.d_density[size_t(c) * size_t(n) + size_t(i)] = dd[c];
    } else if (!a.corner_idx) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const size_t k = size_t(c) * size_t(n) + size_t(i);
        a.d_density[k] = dd[c] * density_act_grad(a.density[k], a.act);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int64_t k = corner_slot(a, c, i);
        if (k >= 0 && dd[c] != 0.0f)
          unsafeAtomicAdd(&a.d_density[k], dd[c] * density_act_grad(a.density[k], a.act));
      }
    }
  }
  float acc[NB][3];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0f;
  const VoxRec vr = a.ws.vox[i];
  const float he = 0.5f * vr.be.w;
  const float xv0 = vr.be.x + he, xv1 = vr.be.y + he, xv2 = vr.be.z + he;
  for (int v = 0; v < a.V; ++v) {
    // the composite backward zeroed the clamped channels (and never wrote
    // the records of views that do not see the voxel)
    const float* dcp = a.ws.dcol + 3 * (size_t(v) * size_t(n) + size_t(i));
    const float g0 = dcp[0], g1 = dcp[1], g2 = dcp[2];
    if (g0 == 0.0f && g1 == 0.0f && g2 == 0.0f) continue;
    const lv_camera& cam = a.cams[v];
    float dx = xv0 - cam.o[0], dy = xv1 - cam.o[1], dz = xv2 - cam.o[2];
    const float inv = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= inv; dy *= inv; dz *= inv;
    float Y[16];
    sh_basis<DEG>(dx, dy, dz, Y);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      acc[j][0] = fmaf(Y[j], g0, acc[j][0]);
      acc[j][1] = fmaf(Y[j], g1, acc[j][1]);
      acc[j][2] = fmaf(Y[j], g2, acc[j][2]);
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) a.d_sh[size_t(j * 3 + ch) * size_t(n) + size_t(i)] = acc[j][ch];
}

hipError_t launch_sh_bwd(const RasterArgs& a, hipStream_t s) {
  const uint32_t blocks = uint32_t((a.n + 255) / 256);
  if (blocks == 0) return hipSuccess;
  const bool generic = a.corner_idx != nullptr || a.act != LV_ACT_NONE;
#define LV_SHB(D) (generic ? k_sh_bwd<D, true> : k_sh_bwd<D, false>)
  switch (a.deg) {
    case 0: hipLaunchKernelGGL(LV_SHB(0), dim3(blocks), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL(LV_SHB(1), dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(LV_SHB(2), dim3(blocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(LV_SHB(3), dim3(blocks), dim3(256), 0, s, a); break;
  }
#undef LV_SHB
  return hipGetLastError();
}

}  // namespace lv

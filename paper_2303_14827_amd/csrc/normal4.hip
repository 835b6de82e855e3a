// normal4.hip -- the four-neighbour normal (paragraph "Lighting/Illumination": the
// points above, below, left and right of a hit are examined to build the surrounding
// surface, whose normal shades the hit).
//
// After a frame is rendered (the render kernels skip their own normal stencil in this
// mode), each hit pixel takes the hit points P = eye + t d of itself and of the pixels
// left, right, above and below (row 0 is the top; a miss or a pixel outside the image
// has no hit). Along each image axis the tangent is the central difference of the two
// neighbours' hits when both hit, else the one-sided difference with the pixel's own
// hit; the normal is the normalised cross product of the horizontal tangent (towards
// the right) and the vertical one (towards the top), turned to face the eye. A missing
// tangent or a vanishing product gives -d (flagged as a fallback). The shade is then
// Eq. phong (phong_shade). One thread per pixel; it reads five depths and writes the
// pixel's shade and optional normal, 8-bit image and flags.
#include <hip/hip_runtime.h>

#include "dq_device.h"
#include "kparams.h"
#include "launch.h"

namespace dqj {

namespace {

__device__ __forceinline__ bool hit_point(const KParams &P, const KOut &out, int i, int j, float p[3],
                                          float d[3]) {
  if (i < 0 || j < 0 || i >= P.W || j >= P.H) return false;
  const float t = out.depth[(int64_t)j * P.W + i];
  if (!isfinite(t)) return false;
  pixel_dir(P, i, j, d);
#pragma unroll
  for (int k = 0; k < 3; ++k) p[k] = fmaf(t, d[k], P.eye[k]);
  return true;
}

__global__ __launch_bounds__(256) void neighbour_normal_kernel(KParams P, KOut out) {
  const int i = blockIdx.x * 16 + (threadIdx.x & 15);
  const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= P.W || j >= P.H) return;
  const int64_t idx = (int64_t)j * P.W + i;
  if (!out.mask[idx]) return;
  float pc[3] = {0.0f, 0.0f, 0.0f}, dc[3] = {0.0f, 0.0f, -1.0f}, dn[3];
  float pl[3] = {0.0f, 0.0f, 0.0f}, pr[3] = {0.0f, 0.0f, 0.0f};
  float pu[3] = {0.0f, 0.0f, 0.0f}, pd[3] = {0.0f, 0.0f, 0.0f};
  hit_point(P, out, i, j, pc, dc);
  const bool hl = hit_point(P, out, i - 1, j, pl, dn);
  const bool hr = hit_point(P, out, i + 1, j, pr, dn);
  const bool hu = hit_point(P, out, i, j - 1, pu, dn);
  const bool hd = hit_point(P, out, i, j + 1, pd, dn);
  float tx[3], ty[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    tx[k] = (hl && hr) ? pr[k] - pl[k] : (hr ? pr[k] - pc[k] : pc[k] - pl[k]);
    ty[k] = (hu && hd) ? pu[k] - pd[k] : (hu ? pu[k] - pc[k] : pc[k] - pd[k]);
  }
  const float c[3] = {tx[1] * ty[2] - tx[2] * ty[1], tx[2] * ty[0] - tx[0] * ty[2],
                      tx[0] * ty[1] - tx[1] * ty[0]};
  const float len = sqrtf(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  float n[3];
  bool fallback = !((hl || hr) && (hu || hd) && len > 0.0f && isfinite(len));
  if (!fallback) {
    const float sg = (c[0] * dc[0] + c[1] * dc[1] + c[2] * dc[2]) > 0.0f ? -1.0f : 1.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) n[k] = sg * c[k] / len;
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) n[k] = -dc[k];
  }
  const float s = phong_shade(P, n, dc);
  out.shade[idx] = s;
  if (out.image8) out.image8[idx] = (uint8_t)floorf(fmaf(255.0f, s, 0.5f));
  if (out.normal) {
    out.normal[3 * idx + 0] = n[0];
    out.normal[3 * idx + 1] = n[1];
    out.normal[3 * idx + 2] = n[2];
  }
  if (out.flags)
    out.flags[idx] = (uint8_t)((out.flags[idx] & ~DQJ_FLAG_FALLBACK) | (fallback ? DQJ_FLAG_FALLBACK : 0));
}

}  // namespace

hipError_t launch_neighbour_normal(const KParams &P, const KOut &out, hipStream_t s) {
  const dim3 grid((P.W + 15) / 16, (P.H + 15) / 16);
  hipLaunchKernelGGL(neighbour_normal_kernel, grid, dim3(256), 0, s, P, out);
  return hipGetLastError();
}

}  // namespace dqj

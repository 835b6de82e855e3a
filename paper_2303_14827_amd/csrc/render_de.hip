// render_de.hip -- distance-estimate ray march (section "Ray-Marching", Eq. distfract2).
//
// One thread per pixel. From the box entry the ray is stepped by the distance estimate
// 0.5 |z_m| ln|z_m| / |z'_m| of the current point, clamped to [de_min_step, de_max_step],
// until the estimate falls below de_hit_eps (hit there), a step lands inside the set
// (the step is bisected B times), the ray leaves the box, or S steps were taken (miss).
// The derivative norm follows |z'_{n+1}| = 2 |z_n| |z'_n| from |z'_0| = 1 (Eq. distfract;
// norms are the escape norm). Normal and shade are those of the fixed-step path.
//
// FP32 range: |z'_n|^2 grows like (4 R^2)^n, beyond FP32 for n >= 22 at R = 4, so the
// kernel carries D_n = |z'_n|^2 / (4 R^2)^n, which obeys D_{n+1} = D_n |z_n|^2 / R^2 and
// stays <= 1 while the orbit has not escaped. The estimate is formed in base-2 logs:
//   log2(|z_m| / |z'_m|) = (log2 |z_m|^2 - log2 D_m - m log2(4 R^2)) / 2.
// D_m may underflow to 0 on orbits that stay very small for a long time; the estimate is
// then +inf and the step is clamped to de_max_step, as a huge estimate would be.
#include "dq_device.h"
#include "launch.h"

namespace dqj {

namespace {

// Classify with the scaled derivative: returns the escape index m (0 when inside) and,
// for an escaping point, the distance estimate in *de.
template <int NORM>
__device__ __forceinline__ int classify_de(const KParams &P, DQ<float> z, float *de, float *n2out) {
  float s = vec_s(z);
  float n2prev = fmaf(z.a0, z.a0, s);
  if (NORM == 0) n2prev = fmaf(z.b3, z.b3, fmaf(z.b2, z.b2, fmaf(z.b1, z.b1, fmaf(z.b0, z.b0, n2prev))));
  float D = 1.0f;
  for (int n = 1; n <= P.N; ++n) {
    D = D * (n2prev * P.de_inv_r2);
    const float n2 = dq_update<NORM>(z, s, P.c);
    if (n2 > P.R2) {
      const float l2n = __builtin_amdgcn_logf(n2);     // log2 |z_m|^2
      const float q = 0.5f * (l2n - __builtin_amdgcn_logf(D) - (float)n * P.de_log2_4r2);
      // 0.5 |z| ln|z| / |z'| = 0.5 * 2^q * (ln 2 / 2) * log2 |z|^2
      *de = 0.25f * 0.69314718f * l2n * __builtin_amdgcn_exp2f(q);
      *n2out = n2;
      return n;
    }
    n2prev = n2;
  }
  *n2out = n2prev;
  return 0;
}

template <int NORM>
__device__ void render_pixel_de(const KParams &P, int i, int j, PixelOut &r,
                                unsigned long long &iters) {
  float d[3];
  pixel_dir(P, i, j, d);
  float t0, t1;
  if (!clip_box(P, d, t0, t1)) {
    r = miss_pixel(0);
    return;
  }
  int kstar = -1;
  float thit = t0, lo = t0, hi = t0;
  bool bisect = false;
  float t = t0, tprev = t0;
  for (int k = 0; k < P.S; ++k) {
    DQ<float> z = slice_map<float>(P, fmaf(t, d[0], P.eye[0]), fmaf(t, d[1], P.eye[1]),
                                   fmaf(t, d[2], P.eye[2]));
    float de = 0.0f, n2;
    const int m = classify_de<NORM>(P, z, &de, &n2);
    iters += m ? m : P.N;
    if (m == 0) {   // inside: the hit is t0 on the first point, else bisect the last step
      kstar = k;
      if (k > 0) {
        lo = tprev;
        hi = t;
        bisect = true;
      }
      break;
    }
    if (de < P.de_eps) {
      kstar = k;
      thit = t;
      break;
    }
    const float step = fminf(fmaxf(de, P.de_min_step), P.de_max_step);
    tprev = t;
    t = t + step;
    if (t > t1) break;
  }
  if (kstar < 0) {
    r = miss_pixel(DQJ_FLAG_BOX);
    return;
  }
  const float *c = P.c;
  if (bisect) {
    for (int b = 0; b < P.B; ++b) {
      const float tm = 0.5f * (lo + hi);
      DQ<float> z = slice_map<float>(P, fmaf(tm, d[0], P.eye[0]), fmaf(tm, d[1], P.eye[1]),
                                     fmaf(tm, d[2], P.eye[2]));
      float n2;
      const int m = dq_classify<NORM>(z, c, P.N, P.R2, &n2);
      iters += m ? m : P.N;
      if (m == 0)
        hi = tm;
      else
        lo = tm;
    }
    thit = 0.5f * (lo + hi);
  }
  const float ph[3] = {fmaf(thit, d[0], P.eye[0]), fmaf(thit, d[1], P.eye[1]),
                       fmaf(thit, d[2], P.eye[2])};
  float g[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float gp = 0.0f;
#pragma unroll
    for (int sgn = 0; sgn < 2; ++sgn) {
      float x[3] = {ph[0], ph[1], ph[2]};
      x[a] = sgn == 0 ? ph[a] + P.h : ph[a] - P.h;
      DQ<float> z = slice_map<float>(P, x[0], x[1], x[2]);
      float n2;
      int m = dq_classify<NORM>(z, c, P.N, P.R2, &n2);
      m = m ? m : P.N;
      iters += m;
      const float G = potential(n2, m);
      gp = sgn == 0 ? G : gp - G;
    }
    g[a] = gp;
  }
  finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
}

template <int NORM>
__global__ __launch_bounds__(256) void render_de_kernel(KParams P, KOut out) {
  const int i = blockIdx.x * 16 + (threadIdx.x & 15);
  const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
  unsigned long long iters = 0;
  if (i < P.W && j < P.H) {
    PixelOut r;
    render_pixel_de<NORM>(P, i, j, r, iters);
    write_pixel(out, (int64_t)j * P.W + i, r);
  }
  if (out.iters) wave_add_u64(out.iters, iters);
}

}  // namespace

hipError_t launch_render_de(const KParams &P, const KOut &out, hipStream_t s) {
  dim3 grid((P.W + 15) / 16, (P.H + 15) / 16);
  if (P.norm == 0)
    hipLaunchKernelGGL(render_de_kernel<0>, grid, dim3(256), 0, s, P, out);
  else
    hipLaunchKernelGGL(render_de_kernel<1>, grid, dim3(256), 0, s, P, out);
  return hipGetLastError();
}

}  // namespace dqj

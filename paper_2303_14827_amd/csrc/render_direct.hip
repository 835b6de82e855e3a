// render_direct.hip -- the straightforward per-pixel ray marcher and the point
// classifier.
//
// One thread per pixel walks the whole method in order: camera ray, box clip,
// fixed-step march, bisection of the first crossing, central-difference normal of
// the escape potential, ambient + diffuse shade. Lanes of a wave stay on their
// own ray to the end, so a wave runs as long as its slowest ray; the refill kernel
// in render_refill.hip removes that cost. This kernel is the simplest complete
// form of the path and the yardstick the faster kernels are compared with.
#include "dq_device.h"
#include "launch.h"

namespace dqj {

template <int NORM>
__device__ void render_pixel_f32(const KParams &P, int i, int j, PixelOut &r,
                                 unsigned long long &iters) {
  float d[3];
  pixel_dir(P, i, j, d);
  float t0, t1;
  if (!clip_box(P, d, t0, t1)) {
    r = miss_pixel(0);
    return;
  }
  const float *c = P.c;
  const float dt = (t1 - t0) / (float)P.S;
  int kstar = -1;
  for (int k = 0; k <= P.S; ++k) {
    const float t = fmaf((float)k, dt, t0);
    DQ<float> z = slice_map<float>(P, fmaf(t, d[0], P.eye[0]), fmaf(t, d[1], P.eye[1]),
                                   fmaf(t, d[2], P.eye[2]));
    float n2;
    const int m = dq_classify<NORM>(z, c, P.N, P.R2, &n2);
    iters += m ? m : P.N;
    if (m == 0) {
      kstar = k;
      break;
    }
  }
  if (kstar < 0) {
    r = miss_pixel(DQJ_FLAG_BOX);
    return;
  }
  float thit;
  if (kstar == 0) {
    thit = t0;
  } else {
    float lo = fmaf((float)(kstar - 1), dt, t0);
    float hi = fmaf((float)kstar, dt, t0);
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
  float g[3] = {0.0f, 0.0f, 0.0f};
  int m0 = 0;
  // (the four-neighbour normal is formed after the frame: no stencil here)
  if (P.normal_mode == 0)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int sgn = 0; sgn < 2; ++sgn) {
      float x[3] = {ph[0], ph[1], ph[2]};
      x[a] = sgn == 0 ? ph[a] + P.h : ph[a] - P.h;
      DQ<float> z = slice_map<float>(P, x[0], x[1], x[2]);
      float n2;
      int m = dq_classify<NORM>(z, c, P.N, P.R2, &n2);
      m = m ? m : P.N;
      iters += m;
      stencil_add(g[0], g[1], g[2], m0, 2 * a + sgn, pot_log(n2), m);
    }
  }
  finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
}

template <int NORM>
__global__ __launch_bounds__(256) void render_direct_kernel(KParams P, KOut out) {
  const int i = blockIdx.x * 16 + (threadIdx.x & 15);
  const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
  unsigned long long iters = 0;
  if (i < P.W && j < P.H) {
    PixelOut r;
    render_pixel_f32<NORM>(P, i, j, r, iters);
    write_pixel(out, (int64_t)j * P.W + i, r);
  }
  if (out.iters) wave_add_u64(out.iters, iters);
}

hipError_t launch_render_direct(const KParams &P, const KOut &out, hipStream_t s) {
  dim3 grid((P.W + 15) / 16, (P.H + 15) / 16);
  if (P.norm == 0)
    hipLaunchKernelGGL(render_direct_kernel<0>, grid, dim3(256), 0, s, P, out);
  else
    hipLaunchKernelGGL(render_direct_kernel<1>, grid, dim3(256), 0, s, P, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Point classifier (test and debugging entry point).
// ---------------------------------------------------------------------------

template <int NORM>
__global__ __launch_bounds__(256) void classify_f32_kernel(const float *pts, int n, KParams P,
                                                           int32_t *esc, float *n2out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float *p = pts + 8 * (int64_t)q;
  DQ<float> z{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]};
  float n2;
  esc[q] = dq_classify<NORM>(z, P.c, P.N, P.R2, &n2);
  if (n2out) n2out[q] = n2;
}

template <int NORM>
__global__ __launch_bounds__(256) void classify_f64_kernel(const double *pts, int n, KIter64 P,
                                                           int32_t *esc, float *n2out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double *p = pts + 8 * (int64_t)q;
  DQ<double> z{p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7]};
  double n2;
  esc[q] = dq_classify<NORM>(z, P.c, P.N, P.R2, &n2);
  if (n2out) n2out[q] = (float)n2;
}

hipError_t launch_classify_f32(const float *pts, int n, const KParams &P, int32_t *esc,
                               float *n2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (n + 255) / 256;
  if (P.norm == 0)
    hipLaunchKernelGGL(classify_f32_kernel<0>, dim3(blocks), dim3(256), 0, s, pts, n, P, esc, n2);
  else
    hipLaunchKernelGGL(classify_f32_kernel<1>, dim3(blocks), dim3(256), 0, s, pts, n, P, esc, n2);
  return hipGetLastError();
}

hipError_t launch_classify_f64(const double *pts, int n, const KIter64 &P, int32_t *esc,
                               float *n2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (n + 255) / 256;
  if (P.norm == 0)
    hipLaunchKernelGGL(classify_f64_kernel<0>, dim3(blocks), dim3(256), 0, s, pts, n, P, esc, n2);
  else
    hipLaunchKernelGGL(classify_f64_kernel<1>, dim3(blocks), dim3(256), 0, s, pts, n, P, esc, n2);
  return hipGetLastError();
}

}  // namespace dqj

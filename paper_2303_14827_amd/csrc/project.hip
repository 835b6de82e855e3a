// project.hip -- projection ("shadow") rendering, the second dimension reduction of
// paragraph "Dimension Reduction": the set of R^8 seen through its projection onto the
// slice's 3D space. A world point x is inside when some point of R^8 that projects onto
// it is inside; that fibre is sampled by F offsets (o_f, given by the caller), so the
// test is: some o_f has O + x U + y V + z W + o_f inside (N updates without escape). The
// march, bisection and shade are those of the slice render; the potential of the normal
// is the least potential over the F points (the potential of the union of the fibre's
// sets). One thread per pixel: a sample costs up to F classifications and stops at the
// first inside fibre point, and the fibre loop index is wave-uniform, so the offsets are
// read as scalars from the kernel argument.
#include "dq_device.h"
#include "launch.h"
#include "qform.h"

namespace dqj {

namespace {

// Per-lane constants of the q-form update: h (c0 and c_i / 2) and R^2 - c0.
struct QC {
  float h[8];
  float R2c;
};

// Escape index of zeta_0 = z (0 when it stays inside for N updates), with the q-form
// update; *n2 receives ||z_m||^2 (||z_N||^2 when inside). Two updates per loop trip, each
// tested: the per-lane loop's control (exit mask, counter, branch) is paid once per two
// updates. A point escaping on the first of the pair has its index and norm from that
// update; the second runs on the escaped state (a norm of at most about R^4) and is
// discarded.
template <int NORM>
__device__ __forceinline__ int classify_q(DQ<float> z, const QC &K, int N, float *n2) {
  float q = q_of(z, K.h[0]);
  float m2 = 0.0f;
  int n = 1;
  for (; n + 1 <= N; n += 2) {
    const float a = dq_update_q<NORM>(z, q, K.h);
    const float b = dq_update_q<NORM>(z, q, K.h);
    const bool ea = a > K.R2c;
    if (ea || b > K.R2c) {
      *n2 = (ea ? a : b) + K.h[0];
      return ea ? n : n + 1;
    }
    m2 = b;
  }
  if (n == N) {   // odd N: the last update alone
    m2 = dq_update_q<NORM>(z, q, K.h);
    if (m2 > K.R2c) {
      *n2 = m2 + K.h[0];
      return n;
    }
  }
  *n2 = m2 + K.h[0];
  return 0;
}

// 1 when some fibre point over world point (x, y, w) is inside; counts the updates.
template <int NORM>
__device__ __forceinline__ bool inside_union(const KParams &P, const QC &K, const FiberTable &fb, int F,
                                             float x, float y, float w,
                                             unsigned long long &iters) {
  const DQ<float> z0 = slice_map<float>(P, x, y, w);
  for (int f = 0; f < F; ++f) {
    DQ<float> z{z0.a0 + fb.off[f][0], z0.a1 + fb.off[f][1], z0.a2 + fb.off[f][2],
                z0.a3 + fb.off[f][3], z0.b0 + fb.off[f][4], z0.b1 + fb.off[f][5],
                z0.b2 + fb.off[f][6], z0.b3 + fb.off[f][7]};
    float n2;
    const int m = classify_q<NORM>(z, K, P.N, &n2);
    iters += m ? m : P.N;
    if (m == 0) return true;
  }
  return false;
}

// Least escape potential over the fibre points of world point (x, y, w).
template <int NORM>
__device__ __forceinline__ float potential_union(const KParams &P, const QC &K, const FiberTable &fb,
                                                 int F,
                                                 float x, float y, float w,
                                                 unsigned long long &iters) {
  const DQ<float> z0 = slice_map<float>(P, x, y, w);
  float best = 0.0f;
  for (int f = 0; f < F; ++f) {
    DQ<float> z{z0.a0 + fb.off[f][0], z0.a1 + fb.off[f][1], z0.a2 + fb.off[f][2],
                z0.a3 + fb.off[f][3], z0.b0 + fb.off[f][4], z0.b1 + fb.off[f][5],
                z0.b2 + fb.off[f][6], z0.b3 + fb.off[f][7]};
    float n2;
    int m = classify_q<NORM>(z, K, P.N, &n2);
    m = m ? m : P.N;
    iters += m;
    const float G = potential(n2, m);
    best = (f == 0 || G < best) ? G : best;
  }
  return best;
}

template <int NORM>
__device__ void render_pixel_project(const KParams &P, const QC &K, const FiberTable &fb, int F,
                                     int i, int j, PixelOut &r, unsigned long long &iters) {
  float d[3];
  pixel_dir(P, i, j, d);
  float t0, t1;
  if (!clip_box(P, d, t0, t1)) {
    r = miss_pixel(0);
    return;
  }
  const float dt = (t1 - t0) / (float)P.S;
  int kstar = -1;
  for (int k = 0; k <= P.S; ++k) {
    const float t = fmaf((float)k, dt, t0);
    if (inside_union<NORM>(P, K, fb, F, fmaf(t, d[0], P.eye[0]), fmaf(t, d[1], P.eye[1]),
                           fmaf(t, d[2], P.eye[2]), iters)) {
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
      if (inside_union<NORM>(P, K, fb, F, fmaf(tm, d[0], P.eye[0]), fmaf(tm, d[1], P.eye[1]),
                             fmaf(tm, d[2], P.eye[2]), iters))
        hi = tm;
      else
        lo = tm;
    }
    thit = 0.5f * (lo + hi);
  }
  const float ph[3] = {fmaf(thit, d[0], P.eye[0]), fmaf(thit, d[1], P.eye[1]),
                       fmaf(thit, d[2], P.eye[2])};
  float g[3] = {0.0f, 0.0f, 0.0f};
  // (the four-neighbour normal is formed after the frame: no stencil here)
  if (P.normal_mode == 0) {
    for (int a = 0; a < 3; ++a) {
      float x[3] = {ph[0], ph[1], ph[2]};
      x[a] = ph[a] + P.h;
      const float gp = potential_union<NORM>(P, K, fb, F, x[0], x[1], x[2], iters);
      x[a] = ph[a] - P.h;
      const float gm = potential_union<NORM>(P, K, fb, F, x[0], x[1], x[2], iters);
      g[a] = gp - gm;
    }
  }
  finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
}

template <int NORM>
__global__ __launch_bounds__(256) void render_project_kernel(KParams P, FiberTable fb, int F,
                                                             KOut out) {
  const int i = blockIdx.x * 16 + (threadIdx.x & 15);
  const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
  unsigned long long iters = 0;
  enter_update_mode();
  QC K;
  K.h[0] = to_vgpr(P.c[0]);
#pragma unroll
  for (int q = 1; q < 8; ++q) K.h[q] = to_vgpr(0.5f * P.c[q]);
  K.R2c = to_vgpr(P.R2 - P.c[0]);
  if (i < P.W && j < P.H) {
    PixelOut r;
    render_pixel_project<NORM>(P, K, fb, F, i, j, r, iters);
    write_pixel(out, (int64_t)j * P.W + i, r);
  }
  if (out.iters) wave_add_u64(out.iters, iters);
}

}  // namespace

hipError_t launch_render_project(const KParams &P, const FiberTable &fb, int F, const KOut &out,
                                 hipStream_t s) {
  if (F < 1 || F > kMaxFiber) return hipErrorInvalidValue;
  const dim3 grid((P.W + 15) / 16, (P.H + 15) / 16);
  if (P.norm == 0)
    hipLaunchKernelGGL(render_project_kernel<0>, grid, dim3(256), 0, s, P, fb, F, out);
  else
    hipLaunchKernelGGL(render_project_kernel<1>, grid, dim3(256), 0, s, P, fb, F, out);
  return hipGetLastError();
}

}  // namespace dqj

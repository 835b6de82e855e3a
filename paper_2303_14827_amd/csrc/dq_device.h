// dq_device.h -- device building blocks of the ray-march path (library-internal).
//
// The dual-quaternion square uses the cross-product-free form of the product
// rule: for zeta = a + e b,
//   a^2      = (a0^2 - |a_v|^2, 2 a0 a_v)                         (Eq. quatsq)
//   a b + b a = (2 (a0 b0 - a_v . b_v), 2 (a0 b_v + b0 a_v))       (the cross
//   products of the two Hamilton products cancel)
// so one update zeta <- zeta^2 + c (Eq. dqjulia2) is 37 flops and the 8-square
// escape norm 15 more.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dqj.h"
#include "kparams.h"

namespace dqj {

// 8-component state held in registers.
template <typename T>
struct DQ {
  T a0, a1, a2, a3, b0, b1, b2, b3;
};

// One update z <- z^2 + c given s = |a_v|^2 of the current z. Leaves z at z',
// s at |a'_v|^2 (which the next update needs, so the escape norm reuses it) and
// returns ||z'||^2 under NORM (0: all 8 squares, 1: the real quaternion's 4).
// 26 VALU operations, 13 of them fused multiply-adds.
template <int NORM, typename T>
__device__ __forceinline__ T dq_update(DQ<T> &z, T &s, const T *c) {
  const T ta = z.a0 + z.a0;
  const T tb = z.b0 + z.b0;
  const T dot = fma(z.a3, z.b3, fma(z.a2, z.b2, z.a1 * z.b1));
  DQ<T> r;
  r.a0 = fma(z.a0, z.a0, c[0] - s);
  r.a1 = fma(ta, z.a1, c[1]);
  r.a2 = fma(ta, z.a2, c[2]);
  r.a3 = fma(ta, z.a3, c[3]);
  r.b0 = fma(ta, z.b0, fma(T(-2), dot, c[4]));
  r.b1 = fma(ta, z.b1, fma(tb, z.a1, c[5]));
  r.b2 = fma(ta, z.b2, fma(tb, z.a2, c[6]));
  r.b3 = fma(ta, z.b3, fma(tb, z.a3, c[7]));
  const T s2 = fma(r.a3, r.a3, fma(r.a2, r.a2, r.a1 * r.a1));
  T n2 = fma(r.a0, r.a0, s2);
  if (NORM == 0) n2 = fma(r.b3, r.b3, fma(r.b2, r.b2, fma(r.b1, r.b1, fma(r.b0, r.b0, n2))));
  z = r;
  s = s2;
  return n2;
}

// The same update in FP32 with the 8-square norm, written so every state register
// is overwritten in place (the compiler's version of the loop rotates the state
// through fresh registers and pays 5-9 copies per update). VALU only: no memory
// operands. The leading s_nop gives any preceding transcendental result the wait
// states a dependent VALU read needs.
__device__ __forceinline__ float dq_update_inplace(DQ<float> &z, float &s, const float *c) {
  float ta, tb, dot, n2;
  asm("s_nop 1\n\t"
      "v_add_f32_e32 %[ta], %[a0], %[a0]\n\t"
      "v_add_f32_e32 %[tb], %[b0], %[b0]\n\t"
      "v_mul_f32_e32 %[dot], %[a1], %[b1]\n\t"
      "v_fmac_f32_e32 %[dot], %[a2], %[b2]\n\t"
      "v_fmac_f32_e32 %[dot], %[a3], %[b3]\n\t"
      "v_fma_f32 %[b1], %[ta], %[b1], %[c5]\n\t"
      "v_fmac_f32_e32 %[b1], %[tb], %[a1]\n\t"
      "v_fma_f32 %[b2], %[ta], %[b2], %[c6]\n\t"
      "v_fmac_f32_e32 %[b2], %[tb], %[a2]\n\t"
      "v_fma_f32 %[b3], %[ta], %[b3], %[c7]\n\t"
      "v_fmac_f32_e32 %[b3], %[tb], %[a3]\n\t"
      "v_fma_f32 %[b0], %[ta], %[b0], %[c4]\n\t"
      "v_fmac_f32_e32 %[b0], -2.0, %[dot]\n\t"
      "v_fma_f32 %[a1], %[ta], %[a1], %[c1]\n\t"
      "v_fma_f32 %[a2], %[ta], %[a2], %[c2]\n\t"
      "v_fma_f32 %[a3], %[ta], %[a3], %[c3]\n\t"
      "v_fma_f32 %[a0], %[a0], %[a0], %[c0]\n\t"
      "v_sub_f32_e32 %[a0], %[a0], %[s]\n\t"
      "v_mul_f32_e32 %[s], %[a1], %[a1]\n\t"
      "v_fmac_f32_e32 %[s], %[a2], %[a2]\n\t"
      "v_fmac_f32_e32 %[s], %[a3], %[a3]\n\t"
      "v_fma_f32 %[n2], %[a0], %[a0], %[s]\n\t"
      "v_fmac_f32_e32 %[n2], %[b0], %[b0]\n\t"
      "v_fmac_f32_e32 %[n2], %[b1], %[b1]\n\t"
      "v_fmac_f32_e32 %[n2], %[b2], %[b2]\n\t"
      "v_fmac_f32_e32 %[n2], %[b3], %[b3]"
      : [a0] "+v"(z.a0), [a1] "+v"(z.a1), [a2] "+v"(z.a2), [a3] "+v"(z.a3), [b0] "+v"(z.b0),
        [b1] "+v"(z.b1), [b2] "+v"(z.b2), [b3] "+v"(z.b3), [s] "+v"(s), [ta] "=&v"(ta),
        [tb] "=&v"(tb), [dot] "=&v"(dot), [n2] "=&v"(n2)
      : [c0] "s"(c[0]), [c1] "s"(c[1]), [c2] "s"(c[2]), [c3] "s"(c[3]), [c4] "s"(c[4]),
        [c5] "s"(c[5]), [c6] "s"(c[6]), [c7] "s"(c[7]));
  return n2;
}


// The same update with the Julia constant in vector registers. On gfx950 an FP32
// operation that reads a scalar register issues at about 1.6x the cost of one whose
// operands are all vector registers, so the hot loop keeps per-lane copies of c.
__device__ __forceinline__ float dq_update_inplace_v(DQ<float> &z, float &s, const float *c) {
  float ta, tb, dot, n2;
  asm("s_nop 1\n\t"
      "v_add_f32_e32 %[ta], %[a0], %[a0]\n\t"
      "v_add_f32_e32 %[tb], %[b0], %[b0]\n\t"
      "v_mul_f32_e32 %[dot], %[a1], %[b1]\n\t"
      "v_fmac_f32_e32 %[dot], %[a2], %[b2]\n\t"
      "v_fmac_f32_e32 %[dot], %[a3], %[b3]\n\t"
      "v_fma_f32 %[b1], %[ta], %[b1], %[c5]\n\t"
      "v_fmac_f32_e32 %[b1], %[tb], %[a1]\n\t"
      "v_fma_f32 %[b2], %[ta], %[b2], %[c6]\n\t"
      "v_fmac_f32_e32 %[b2], %[tb], %[a2]\n\t"
      "v_fma_f32 %[b3], %[ta], %[b3], %[c7]\n\t"
      "v_fmac_f32_e32 %[b3], %[tb], %[a3]\n\t"
      "v_fma_f32 %[b0], %[ta], %[b0], %[c4]\n\t"
      "v_fmac_f32_e32 %[b0], -2.0, %[dot]\n\t"
      "v_fma_f32 %[a1], %[ta], %[a1], %[c1]\n\t"
      "v_fma_f32 %[a2], %[ta], %[a2], %[c2]\n\t"
      "v_fma_f32 %[a3], %[ta], %[a3], %[c3]\n\t"
      "v_fma_f32 %[a0], %[a0], %[a0], %[c0]\n\t"
      "v_sub_f32_e32 %[a0], %[a0], %[s]\n\t"
      "v_mul_f32_e32 %[s], %[a1], %[a1]\n\t"
      "v_fmac_f32_e32 %[s], %[a2], %[a2]\n\t"
      "v_fmac_f32_e32 %[s], %[a3], %[a3]\n\t"
      "v_fma_f32 %[n2], %[a0], %[a0], %[s]\n\t"
      "v_fmac_f32_e32 %[n2], %[b0], %[b0]\n\t"
      "v_fmac_f32_e32 %[n2], %[b1], %[b1]\n\t"
      "v_fmac_f32_e32 %[n2], %[b2], %[b2]\n\t"
      "v_fmac_f32_e32 %[n2], %[b3], %[b3]"
      : [a0] "+v"(z.a0), [a1] "+v"(z.a1), [a2] "+v"(z.a2), [a3] "+v"(z.a3), [b0] "+v"(z.b0),
        [b1] "+v"(z.b1), [b2] "+v"(z.b2), [b3] "+v"(z.b3), [s] "+v"(s), [ta] "=&v"(ta),
        [tb] "=&v"(tb), [dot] "=&v"(dot), [n2] "=&v"(n2)
      : [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3]), [c4] "v"(c[4]),
        [c5] "v"(c[5]), [c6] "v"(c[6]), [c7] "v"(c[7]));
  return n2;
}
// A wave-uniform value copied into a vector register (opaque to the compiler, which
// would otherwise keep a uniform value in a scalar register).
__device__ __forceinline__ float to_vgpr(float x) {
  float r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}
// Hot-loop update: the in-place form for FP32 with the 8-square norm.
template <int NORM, typename T>
__device__ __forceinline__ T dq_update_hot(DQ<T> &z, T &s, const T *c) {
  if constexpr (NORM == 0 && sizeof(T) == 4) {
    return dq_update_inplace(z, s, c);
  } else {
    return dq_update<NORM>(z, s, c);
  }
}

template <typename T>
__device__ __forceinline__ T vec_s(const DQ<T> &z) {
  return fma(z.a3, z.a3, fma(z.a2, z.a2, z.a1 * z.a1));
}

// Iterate up to N updates, testing after each (strict > R2). Returns the escape
// index m in 1..N, or 0 if the point stayed inside; z is left at z_m (z_N when
// inside) and *n2 at its norm.
template <int NORM, typename T>
__device__ __forceinline__ int dq_classify(DQ<T> &z, const T *c, int N, T R2, T *n2) {
  T s = vec_s(z);
  T nn = T(0);
  for (int n = 1; n <= N; ++n) {
    nn = dq_update<NORM>(z, s, c);
    if (nn > R2) {
      *n2 = nn;
      return n;
    }
  }
  *n2 = nn;
  return 0;
}

// World point -> R^8 through the slice zeta_0 = O + X U + Y V + Z W.
template <typename T>
__device__ __forceinline__ DQ<T> slice_map(const KParams &P, T x, T y, T z) {
  T v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    v[k] = fma(z, T(P.sw[k]), fma(y, T(P.sv[k]), fma(x, T(P.su[k]), T(P.so[k]))));
  return DQ<T>{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
}

// Camera ray through the centre of pixel (i, j), row 0 at the top.
__device__ __forceinline__ void pixel_dir(const KParams &P, int i, int j, float d[3]) {
  const float sx = fmaf((float)(2 * i + 1), P.inv_w, -1.0f) * P.sx_scale;
  const float sy = fmaf(-(float)(2 * j + 1), P.inv_h, 1.0f) * P.sy_scale;
  float v[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = fmaf(sy, P.up[k], fmaf(sx, P.right[k], P.fwd[k]));
  const float inv = 1.0f / sqrtf(fmaf(v[2], v[2], fmaf(v[1], v[1], v[0] * v[0])));
  d[0] = v[0] * inv;
  d[1] = v[1] * inv;
  d[2] = v[2] * inv;
}

// Bounding sphere about the origin (section "Ray-Marching"): narrows [tn, tf] to the
// roots -b -+ sqrt(b^2 - (|eye|^2 - r^2)) of |eye + t d|^2 = r^2, b = eye.d; false when
// the ray misses the sphere or the intervals do not meet. cull_r2 = 0: no sphere.
// P_T is the FP32 or the FP64 record.
template <typename P_T, typename T>
__device__ __forceinline__ bool clip_sphere(const P_T &P, const T d[3], T &tn, T &tf) {
  if (!(P.cull_r2 > 0)) return true;
  const T ex = T(P.eye[0]), ey = T(P.eye[1]), ez = T(P.eye[2]);
  const T b = ex * d[0] + ey * d[1] + ez * d[2];
  const T q = b * b - ((ex * ex + ey * ey + ez * ez) - T(P.cull_r2));
  if (q < T(0)) return false;
  const T sq = sqrt(q);
  const T sa = -b - sq, sb = -b + sq;
  tn = sa > tn ? sa : tn;
  tf = sb < tf ? sb : tf;
  return !(tn > tf);
}

// x^s for 0 < x <= 1 as exp2(s log2 x) on the hardware transcendental units: relative
// error a few ulp times s |log2 x|, far inside a shade quantum (shades are stored in
// FP32 and compared to 1/255). The FP64 path takes it in FP32 too: an FP64 pow would
// raise that kernel's register count by a quarter for one term of the shade.
__device__ __forceinline__ float spec_pow(float x, float s) {
  return __builtin_amdgcn_exp2f(s * __builtin_amdgcn_logf(x));
}
__device__ __forceinline__ double spec_pow(double x, double s) {
  return (double)spec_pow((float)x, (float)s);
}

// Eq. phong with one directional light of unit intensity: k_a + k_d max(0, n.l), plus
// k_s max(0, r.v)^s with r = 2 n (n.l) - l and v = -d where the light reaches the surface
// (n.l > 0); clamped to [0, 1]. P_T is the FP32 or the FP64 record.
template <typename P_T, typename T>
__device__ __forceinline__ T phong_shade(const P_T &P, const T n[3], const T d[3]) {
  const T l0 = T(P.light[0]), l1 = T(P.light[1]), l2 = T(P.light[2]);
  const T ndl = n[0] * l0 + n[1] * l1 + n[2] * l2;
  T s = T(P.ka) + T(P.kd) * (ndl > T(0) ? ndl : T(0));
  if (P.ks > 0 && ndl > T(0)) {
    const T tn = ndl + ndl;
    const T rv = (n[0] * tn - l0) * (-d[0]) + (n[1] * tn - l1) * (-d[1]) + (n[2] * tn - l2) * (-d[2]);
    if (rv > T(0)) s = s + T(P.ks) * spec_pow(rv < T(1) ? rv : T(1), T(P.shininess));
  }
  return s < T(0) ? T(0) : (s > T(1) ? T(1) : s);
}

// Slab clip of the ray eye + t d against the box (and the bounding sphere, if any);
// t0 >= 0. False if it misses.
template <typename T>
__device__ __forceinline__ bool clip_box(const KParams &P, const T d[3], T &t0, T &t1) {
  T tn = T(0), tf = T(INFINITY);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T o = T(P.eye[k]);
    if (d[k] == T(0)) {
      if (o < T(P.bmin[k]) || o > T(P.bmax[k])) return false;
      continue;
    }
    T ta = (T(P.bmin[k]) - o) / d[k];
    T tb = (T(P.bmax[k]) - o) / d[k];
    if (ta > tb) {
      const T s = ta;
      ta = tb;
      tb = s;
    }
    tn = ta > tn ? ta : tn;
    tf = tb < tf ? tb : tf;
  }
  if (tn > tf) return false;
  if (!clip_sphere(P, d, tn, tf)) return false;
  t0 = tn;
  t1 = tf;
  return true;
}

// The escape potential ln(max(||z_m||^2, 1e-30)) * 2^-m (m = N when inside) is held as
// its two parts: pot_log(||z_m||^2) and m.
template <typename T>
__device__ __forceinline__ T pot_log(T n2) {
  return log(n2 > T(1e-30) ? n2 : T(1e-30));
}

// The potential itself, lv 2^-m, for stencils whose max_iter keeps it and the squares of
// its differences in range (the lane-refill kernels at small max_iter).
template <typename T>
__device__ __forceinline__ T potential(T n2, int m) {
  const T v = n2 > T(1e-30) ? n2 : T(1e-30);
  return log(v) * ldexp(T(1), -m);
}

// Potential lv1 2^-m1 < lv2 2^-m2, compared with both scaled by 2^min(m1, m2).
template <typename T>
__device__ __forceinline__ bool pot_less(T lv1, int m1, T lv2, int m2) {
  const int mm = m1 < m2 ? m1 : m2;
  return lv1 * ldexp(T(1), mm - m1) < lv2 * ldexp(T(1), mm - m2);
}

// One point of the central-difference stencil of the normal: point k (0..5, in the
// order +x, -x, +y, -y, +z, -z) with potential lv 2^-m. The components carry the
// potential times 2^m0, m0 being the least escape index of the stencil so far (a
// smaller one rescales them by a power of two, exactly). The normalised gradient does
// not see that common factor, and the scaled terms stay representable at any max_iter:
// unscaled, 2^-m flushes to zero in FP32 beyond m = 126, and the squares of the
// differences of a smooth stencil beyond about m = 53.
template <typename T>
__device__ __forceinline__ void stencil_add(T &gx, T &gy, T &gz, int &m0, int k, T lv, int m) {
  if (k == 0) {
    m0 = m;
  } else if (m < m0) {
    const T s = ldexp(T(1), m - m0);
    gx *= s;
    gy *= s;
    gz *= s;
    m0 = m;
  }
  const T G = lv * ldexp(T(1), m0 - m);
  const T sg = (k & 1) ? -G : G;
  const int axis = k >> 1;
  if (axis == 0)
    gx += sg;
  else if (axis == 1)
    gy += sg;
  else
    gz += sg;
}

// Outputs of one pixel.
struct PixelOut {
  float depth, shade, nx, ny, nz;
  int32_t first_hit;
  uint8_t mask, flags;
};

__device__ __forceinline__ void write_pixel(const KOut &o, int64_t idx, const PixelOut &r) {
  o.mask[idx] = r.mask;
  o.depth[idx] = r.depth;
  o.shade[idx] = r.shade;
  if (o.image8) o.image8[idx] = (uint8_t)floorf(fmaf(255.0f, r.shade, 0.5f));
  if (o.normal) {
    o.normal[3 * idx + 0] = r.nx;
    o.normal[3 * idx + 1] = r.ny;
    o.normal[3 * idx + 2] = r.nz;
  }
  if (o.first_hit) o.first_hit[idx] = r.first_hit;
  if (o.flags) o.flags[idx] = r.flags;
}

__device__ __forceinline__ PixelOut miss_pixel(uint8_t flags) {
  PixelOut r;
  r.depth = INFINITY;
  r.shade = 0.0f;
  r.nx = r.ny = r.nz = 0.0f;
  r.first_hit = -1;
  r.mask = 0;
  r.flags = flags;
  return r;
}

// Unit normal from the central-difference gradient g; -d when g is zero or not
// finite. Shade: phong_shade.
template <typename T>
__device__ __forceinline__ void finish_hit(const KParams &P, const T g[3], const T d[3], T thit,
                                           int kstar, uint8_t flags, PixelOut &r) {
  const T gl = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  T n[3];
  if (gl > T(0) && isfinite(gl)) {
    n[0] = g[0] / gl;
    n[1] = g[1] / gl;
    n[2] = g[2] / gl;
  } else {
    n[0] = -d[0];
    n[1] = -d[1];
    n[2] = -d[2];
    flags |= DQJ_FLAG_FALLBACK;
  }
  const T s = phong_shade(P, n, d);
  r.depth = (float)thit;
  r.shade = (float)s;
  r.nx = (float)n[0];
  r.ny = (float)n[1];
  r.nz = (float)n[2];
  r.first_hit = kstar;
  r.mask = 1;
  r.flags = flags;
}

// Wave-wide sum, then one 64-bit atomic per wave.
__device__ __forceinline__ void wave_add_u64(unsigned long long *dst, unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(dst, v);
}

}  // namespace dqj

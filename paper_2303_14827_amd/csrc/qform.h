// qform.h -- the FP32 update in "q form" with the FMA's x2 output modifier
// (library-internal; used by the lane-refill marcher and the voxel grid).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "dq_device.h"

namespace dqj {

// The loop carries q = c0 - |a_v|^2 beside zeta, so the new real part is one FMA,
// a0' = a0^2 + q, and tests ||zeta'||^2 - c0 = a0'^2 - q' + |b'|^2 (NORM 0; NORM 1
// drops the |b'|^2) against R^2 - c0. Every other term of the square (Eq. quatsq and
// the dual part, whose cross products cancel) carries a factor 2. With the Julia
// constant halved (h_i = c_i / 2, i >= 1) that factor is the FMA's x2 output modifier:
// round(x) * 2 = round(2 x) exactly, so the result is the same as forming 2 a0 and
// 2 b0 first, without those two operations. 22 VALU operations per update.
//
// The output modifier takes effect only with the IEEE mode bit clear and FP32
// output denormals flushed; enter_update_mode() sets both for the calling wave. The
// march never depends on denormal values (they are far below every escape radius
// and step), and no signalling NaN enters the kernel.
__device__ __forceinline__ void enter_update_mode() {
  asm volatile(
      "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 9, 1), 0\n\t"   // IEEE mode off
      "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 4, 2), 0\n\t"   // FP32 denormals flushed
      "s_nop 3" ::: "memory");
}

__device__ __forceinline__ float dq_update_q_asm(DQ<float> &z, float &q, const float *h) {
  float d, n;
  asm("s_nop 1\n\t"
      "v_fma_f32 %[d], -%[a3], %[b3], %[h4]\n\t"
      "v_fma_f32 %[d], -%[a2], %[b2], %[d]\n\t"
      "v_fma_f32 %[d], -%[a1], %[b1], %[d]\n\t"
      "v_fma_f32 %[b1], %[a0], %[b1], %[h5]\n\t"
      "v_fma_f32 %[b1], %[b0], %[a1], %[b1] mul:2\n\t"
      "v_fma_f32 %[b2], %[a0], %[b2], %[h6]\n\t"
      "v_fma_f32 %[b2], %[b0], %[a2], %[b2] mul:2\n\t"
      "v_fma_f32 %[b3], %[a0], %[b3], %[h7]\n\t"
      "v_fma_f32 %[b3], %[b0], %[a3], %[b3] mul:2\n\t"
      "v_fma_f32 %[b0], %[a0], %[b0], %[d] mul:2\n\t"
      "v_fma_f32 %[a1], %[a0], %[a1], %[h1] mul:2\n\t"
      "v_fma_f32 %[a2], %[a0], %[a2], %[h2] mul:2\n\t"
      "v_fma_f32 %[a3], %[a0], %[a3], %[h3] mul:2\n\t"
      "v_fma_f32 %[a0], %[a0], %[a0], %[q]\n\t"
      "v_fma_f32 %[q], -%[a1], %[a1], %[h0]\n\t"
      "v_fma_f32 %[q], -%[a2], %[a2], %[q]\n\t"
      "v_fma_f32 %[q], -%[a3], %[a3], %[q]\n\t"
      "v_fma_f32 %[n], %[a0], %[a0], -%[q]\n\t"
      "v_fmac_f32_e32 %[n], %[b0], %[b0]\n\t"
      "v_fmac_f32_e32 %[n], %[b1], %[b1]\n\t"
      "v_fmac_f32_e32 %[n], %[b2], %[b2]\n\t"
      "v_fmac_f32_e32 %[n], %[b3], %[b3]"
      : [a0] "+v"(z.a0), [a1] "+v"(z.a1), [a2] "+v"(z.a2), [a3] "+v"(z.a3), [b0] "+v"(z.b0),
        [b1] "+v"(z.b1), [b2] "+v"(z.b2), [b3] "+v"(z.b3), [q] "+v"(q), [d] "=&v"(d),
        [n] "=&v"(n)
      : [h0] "v"(h[0]), [h1] "v"(h[1]), [h2] "v"(h[2]), [h3] "v"(h[3]), [h4] "v"(h[4]),
        [h5] "v"(h[5]), [h6] "v"(h[6]), [h7] "v"(h[7]));
  return n;
}

// The same arithmetic in C++ (the x2 written out: exact, so the values are those of
// the asm form) for the real-part norm.
template <int NORM>
__device__ __forceinline__ float dq_update_q(DQ<float> &z, float &q, const float *h) {
  if constexpr (NORM == 0) {
    return dq_update_q_asm(z, q, h);
  } else {
    const float d = fmaf(-z.a1, z.b1, fmaf(-z.a2, z.b2, fmaf(-z.a3, z.b3, h[4])));
    DQ<float> r;
    r.b1 = 2.0f * fmaf(z.b0, z.a1, fmaf(z.a0, z.b1, h[5]));
    r.b2 = 2.0f * fmaf(z.b0, z.a2, fmaf(z.a0, z.b2, h[6]));
    r.b3 = 2.0f * fmaf(z.b0, z.a3, fmaf(z.a0, z.b3, h[7]));
    r.b0 = 2.0f * fmaf(z.a0, z.b0, d);
    r.a1 = 2.0f * fmaf(z.a0, z.a1, h[1]);
    r.a2 = 2.0f * fmaf(z.a0, z.a2, h[2]);
    r.a3 = 2.0f * fmaf(z.a0, z.a3, h[3]);
    r.a0 = fmaf(z.a0, z.a0, q);
    q = fmaf(-r.a3, r.a3, fmaf(-r.a2, r.a2, fmaf(-r.a1, r.a1, h[0])));
    z = r;
    return fmaf(r.a0, r.a0, -q);
  }
}

// zeta_1 of a march sample on the identity slice, in closed form: zeta_0 =
// (x, y, w, 0 | 0) gives zeta_1 = (x^2 - y^2 - w^2 + c0, 2xy + c1, 2xw + c2, c3 | c_d),
// with q = (c0 - c3^2) - a1^2 - a2^2. The x2 is the output modifier again, and
// c3..c7 are the halves doubled (exact), so no register holds the full constants.
__device__ __forceinline__ void start_axis_q(float x, float y, float w, const float *h,
                                             float c0c3, float &a0, DQ<float> &z, float &q) {
  asm("v_fma_f32 %[a0], %[x], %[x], %[h0]\n\t"
      "v_fma_f32 %[a1], %[x], %[y], %[h1] mul:2\n\t"
      "v_fma_f32 %[a2], %[x], %[w], %[h2] mul:2\n\t"
      "v_fma_f32 %[a0], -%[y], %[y], %[a0]\n\t"
      "v_fma_f32 %[q], -%[a1], %[a1], %[c0c3]\n\t"
      "v_fma_f32 %[a0], -%[w], %[w], %[a0]\n\t"
      "v_fma_f32 %[q], -%[a2], %[a2], %[q]\n\t"
      "v_add_f32_e32 %[a3], %[h3], %[h3]\n\t"
      "v_add_f32_e32 %[b0], %[h4], %[h4]\n\t"
      "v_add_f32_e32 %[b1], %[h5], %[h5]\n\t"
      "v_add_f32_e32 %[b2], %[h6], %[h6]\n\t"
      "v_add_f32_e32 %[b3], %[h7], %[h7]"
      : [a0] "=&v"(a0), [a1] "=&v"(z.a1), [a2] "=&v"(z.a2), [a3] "=v"(z.a3), [b0] "=v"(z.b0),
        [b1] "=v"(z.b1), [b2] "=v"(z.b2), [b3] "=v"(z.b3), [q] "=&v"(q)
      : [x] "v"(x), [y] "v"(y), [w] "v"(w), [h0] "v"(h[0]), [h1] "v"(h[1]), [h2] "v"(h[2]),
        [c0c3] "v"(c0c3), [h3] "v"(h[3]), [h4] "v"(h[4]), [h5] "v"(h[5]), [h6] "v"(h[6]),
        [h7] "v"(h[7]));
}

// The same start with c3..c7 copied from vector registers holding the full constants
// (for kernels with registers to spare: a move issues faster than the doubling).
__device__ __forceinline__ void start_axis_q_mov(float x, float y, float w, const float *h,
                                                 const float *c, float c0c3, float &a0,
                                                 DQ<float> &z, float &q) {
  asm("v_fma_f32 %[a0], %[x], %[x], %[h0]\n\t"
      "v_fma_f32 %[a1], %[x], %[y], %[h1] mul:2\n\t"
      "v_fma_f32 %[a2], %[x], %[w], %[h2] mul:2\n\t"
      "v_fma_f32 %[a0], -%[y], %[y], %[a0]\n\t"
      "v_fma_f32 %[q], -%[a1], %[a1], %[c0c3]\n\t"
      "v_fma_f32 %[a0], -%[w], %[w], %[a0]\n\t"
      "v_fma_f32 %[q], -%[a2], %[a2], %[q]\n\t"
      "v_mov_b32 %[a3], %[c3]\n\t"
      "v_mov_b32 %[b0], %[c4]\n\t"
      "v_mov_b32 %[b1], %[c5]\n\t"
      "v_mov_b32 %[b2], %[c6]\n\t"
      "v_mov_b32 %[b3], %[c7]"
      : [a0] "=&v"(a0), [a1] "=&v"(z.a1), [a2] "=&v"(z.a2), [a3] "=v"(z.a3), [b0] "=v"(z.b0),
        [b1] "=v"(z.b1), [b2] "=v"(z.b2), [b3] "=v"(z.b3), [q] "=&v"(q)
      : [x] "v"(x), [y] "v"(y), [w] "v"(w), [h0] "v"(h[0]), [h1] "v"(h[1]), [h2] "v"(h[2]),
        [c0c3] "v"(c0c3), [c3] "v"(c[3]), [c4] "v"(c[4]), [c5] "v"(c[5]), [c6] "v"(c[6]),
        [c7] "v"(c[7]));
}

// q = c0 - |a_v|^2 of a state.
__device__ __forceinline__ float q_of(const DQ<float> &z, float c0) {
  return fmaf(-z.a3, z.a3, fmaf(-z.a2, z.a2, fmaf(-z.a1, z.a1, c0)));
}

}  // namespace dqj

// render_de.hip -- distance-estimate ray march (section "Ray-Marching", Eq. distfract2).
//
// From the box entry the ray is stepped by the distance estimate
// 0.5 |z_m| ln|z_m| / |z'_m| of the current point, clamped to [de_min_step, de_max_step],
// until the estimate falls below de_hit_eps (hit there), a step lands inside the set
// (the step is bisected B times), the ray leaves the box, or S steps were taken (miss).
// The derivative norm follows |z'_{n+1}| = 2 |z_n| |z'_n| from |z'_0| = 1 (Eq. distfract;
// norms are the escape norm). Normal and shade are those of the fixed-step path.
//
// Two kernels: render_de_refill_kernel, the production form, is the persistent
// lane-refill design of render_refill.hip (one update per trip on every lane; a march
// point that escapes computes its estimate and starts the next point at once; hits,
// misses, bisection and normal points take the slow path; idle lanes take new rays of
// the wave's tile), and render_de_kernel, one thread per pixel, the yardstick.
//
// FP32 range: |z'_n|^2 grows like (4 R^2)^n, beyond FP32 for n >= 22 at R = 4, so the
// kernel carries D_n = |z'_n|^2 / (4 R^2)^n, which obeys D_{n+1} = D_n |z_n|^2 / R^2 and
// stays <= 1 while the orbit has not escaped. The estimate is formed in base-2 logs:
//   log2(|z_m| / |z'_m|) = (log2 |z_m|^2 - log2 D_m - m log2(4 R^2)) / 2.
// D_m may underflow to 0 on orbits that stay very small for a long time; the estimate is
// then +inf and the step is clamped to de_max_step, as a huge estimate would be.
#include "dq_device.h"
#include "launch.h"
#include "persist.h"
#include "qform.h"
#include "refill.h"
#include "tile_order.h"
#include <cstring>

namespace dqj {

namespace {

// The march points iterate the q-form update (q = c0 - |a_v|^2 carried; norms are
// held minus c0 and tested against R^2 - c0). Per-lane copies of its constants: h
// (c0 and c_i / 2), R^2 - c0, 1 / R^2 and c0 / R^2 (for the derivative factor
// |z_n|^2 / R^2 = (n - c0) / R^2 + c0 / R^2 of a held norm n).
struct QConst {
  float h[8];
  float R2c, inv_r2, c0r;
};

__device__ __forceinline__ void load_qconst(const KParams &P, QConst &K) {
  using persist::uniform_f;
  K.h[0] = to_vgpr(uniform_f(P.c[0]));
#pragma unroll
  for (int i = 1; i < 8; ++i) K.h[i] = to_vgpr(uniform_f(0.5f * P.c[i]));
  K.R2c = to_vgpr(uniform_f(P.R2 - P.c[0]));
  K.inv_r2 = to_vgpr(uniform_f(P.de_inv_r2));
  K.c0r = to_vgpr(uniform_f(P.c[0] * P.de_inv_r2));
}

// zeta_0 of a world point and its q (identity slice: (x, y, w, 0 | 0)).
template <bool AXIS>
__device__ __forceinline__ void de_start(const KParams &P, float x, float y, float w, float c0,
                                         DQ<float> &z, float &q) {
  if (AXIS)
    z = DQ<float>{x, y, w, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  else
    z = slice_map<float>(P, x, y, w);
  q = q_of(z, c0);
}

// ||z||^2 - c0 of a state under NORM.
template <int NORM>
__device__ __forceinline__ float norm2_of(const DQ<float> &z, float q) {
  float n2 = fmaf(z.a0, z.a0, -q);
  if (NORM == 0) n2 = fmaf(z.b3, z.b3, fmaf(z.b2, z.b2, fmaf(z.b1, z.b1, fmaf(z.b0, z.b0, n2))));
  return n2;
}

// One update (returns the new norm minus c0).
template <int NORM>
__device__ __forceinline__ float de_update(DQ<float> &z, float &q, const float *h) {
  return dq_update_q<NORM>(z, q, h);
}

// Estimate 0.5 |z_m| ln|z_m| / |z'_m| from n2 = |z_m|^2 and D = D_m:
// 0.5 |z| ln|z| / |z'| = 0.5 * 2^q * (ln 2 / 2) * log2 |z|^2.
__device__ __forceinline__ float de_estimate(float n2, float D, int m, float log2_4r2) {
  const float l2n = __builtin_amdgcn_logf(n2);
  const float q = 0.5f * (l2n - __builtin_amdgcn_logf(D) - (float)m * log2_4r2);
  return 0.25f * 0.69314718f * l2n * __builtin_amdgcn_exp2f(q);
}

// Escape index m of zeta_0 = z (0 when it stays inside for N updates) with |z_m|^2 in
// *n2out (|z_N|^2 when inside) and, when DE, the distance estimate of an escaping point
// in *de. The estimate is formed once, after the loop.
template <int NORM, bool DE>
__device__ __forceinline__ int classify_de(const KParams &P, const QConst &K, DQ<float> z, float q,
                                           float *de, float *n2out) {
  float n2 = norm2_of<NORM>(z, q);
  float D = 1.0f;
  int n = 0;
  bool esc = false;
  while (n < P.N) {
    ++n;
    if (DE) D = D * fmaf(n2, K.inv_r2, K.c0r);
    n2 = de_update<NORM>(z, q, K.h);
    if (n2 > K.R2c) {
      esc = true;
      break;
    }
  }
  n2 += K.h[0];
  *n2out = n2;
  if (!esc) return 0;
  if (DE) *de = de_estimate(n2, D, n, P.de_log2_4r2);
  return n;
}

template <int NORM, bool AXIS, bool COUNT>
__device__ void render_pixel_de(const KParams &P, const QConst &K, int i, int j, PixelOut &r,
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
    DQ<float> z;
    float q;
    de_start<AXIS>(P, fmaf(t, d[0], P.eye[0]), fmaf(t, d[1], P.eye[1]), fmaf(t, d[2], P.eye[2]),
                   K.h[0], z, q);
    float de = 0.0f, n2;
    const int m = classify_de<NORM, true>(P, K, z, q, &de, &n2);
    if constexpr (COUNT) iters += m ? m : P.N;
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
  if (bisect) {
    for (int b = 0; b < P.B; ++b) {
      const float tm = 0.5f * (lo + hi);
      DQ<float> z;
      float q, n2, unused;
      de_start<AXIS>(P, fmaf(tm, d[0], P.eye[0]), fmaf(tm, d[1], P.eye[1]), fmaf(tm, d[2], P.eye[2]),
                     K.h[0], z, q);
      const int m = classify_de<NORM, false>(P, K, z, q, &unused, &n2);
      if constexpr (COUNT) iters += m ? m : P.N;
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
      DQ<float> z;
      float q, n2, unused;
      de_start<AXIS>(P, x[0], x[1], x[2], K.h[0], z, q);
      int m = classify_de<NORM, false>(P, K, z, q, &unused, &n2);
      m = m ? m : P.N;
      if constexpr (COUNT) iters += m;
      stencil_add(g[0], g[1], g[2], m0, 2 * a + sgn, pot_log(n2), m);
    }
  }
  finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
}

// Blocks of 8 x (8 waves_per_block) pixels, one wave per 8 x 8 square: a block keeps its
// slot on the CU until its slowest wave is done, and DE work per wave varies widely, so
// small blocks free slots sooner; a square wave's rays are more alike than a 16 x 4
// stripe's (the three-frame batch of 1024^2 frames: 2.22 ms with stripes, 1.86 ms with
// squares, the same image).
//
// Blocks are dispatched in the order of their index, and a launch ends with its slowest
// waves, whose rays creep along the set near the image centre. So the block index is
// mapped centre-out (tile_order.h): the long rays start first and the short rays at the
// image edge fill the ramp-down (a 1024^2 frame 16% faster, the same image).
template <int NORM, bool AXIS, bool COUNT>
__device__ __forceinline__ void render_de_block(const KParams &P, const KOut &out, int bx, int by) {
  const int i = bx * 8 + (threadIdx.x & 7);
  const int j = by * (blockDim.x >> 3) + (threadIdx.x >> 3);
  enter_update_mode();
  QConst K;
  load_qconst(P, K);
  unsigned long long iters = 0;
  if (i < P.W && j < P.H) {
    PixelOut r;
    render_pixel_de<NORM, AXIS, COUNT>(P, K, i, j, r, iters);
    write_pixel(out, (int64_t)j * P.W + i, r);
  }
  if constexpr (COUNT) {
    if (out.iters) wave_add_u64(out.iters, iters);
  }
}

// COUNT: the launch has an update counter to fill (the other kernels compile the
// counting out).
template <int NORM, bool AXIS, bool COUNT>
__global__ __launch_bounds__(256) void render_de_kernel(KParams P, KOut out) {
  const uint32_t t = centre_out_tile(blockIdx.y * gridDim.x + blockIdx.x, (int)gridDim.x, (int)gridDim.y);
  render_de_block<NORM, AXIS, COUNT>(P, out, (int)(t % gridDim.x), (int)(t / gridDim.x));
}

// Several frames in one launch (records from a device table; the grid is the largest
// frame's blocks times the number of frames). The frames are interleaved in dispatch
// order: block g of the launch renders block g / n of frame g % n, each frame's blocks
// taken centre-out, so every frame's long rays start in the first part of the launch and
// one frame's slow waves overlap the others' work (three 1024^2 frames: 1.73 ms with the
// frames in turn and row order, 1.56 ms, the same images).
template <int NORM, bool AXIS, bool COUNT>
__global__ __launch_bounds__(256) void render_de_batch_kernel(const FrameDesc *__restrict__ table) {
  const uint32_t g = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  const persist::ConstFrame F = (persist::ConstFrame)table + g % gridDim.z;
  const KParams &P = F->P;
  const int X = (P.W + 7) / 8, Y = (P.H + 7) / 8;
  const uint32_t b = g / gridDim.z;
  if (b >= (uint32_t)(X * Y)) return;   // a frame smaller than the largest
  const uint32_t t = centre_out_tile(b, X, Y);
  render_de_block<NORM, AXIS, COUNT>(P, F->out, (int)(t % (uint32_t)X), (int)(t / (uint32_t)X));
}

}  // namespace

hipError_t launch_render_de(const KParams &P, const KOut &out, int waves_per_block, hipStream_t s) {
  const int wpb = waves_per_block < 1 ? 1 : (waves_per_block > 4 ? 4 : waves_per_block);
  const int bh = 8 * wpb;
  dim3 grid((P.W + 7) / 8, (P.H + bh - 1) / bh);
  const bool axis = P.axis_slice != 0;
#define DQJ_DE_DIRECT(NM, AX)                                                               \
  do {                                                                                      \
    if (out.iters)                                                                          \
      hipLaunchKernelGGL((render_de_kernel<NM, AX, true>), grid, dim3(64 * wpb), 0, s, P, out); \
    else                                                                                    \
      hipLaunchKernelGGL((render_de_kernel<NM, AX, false>), grid, dim3(64 * wpb), 0, s, P, out); \
  } while (0)
  if (P.norm == 0) {
    if (axis)
      DQJ_DE_DIRECT(0, true);
    else
      DQJ_DE_DIRECT(0, false);
  } else {
    if (axis)
      DQJ_DE_DIRECT(1, true);
    else
      DQJ_DE_DIRECT(1, false);
  }
#undef DQJ_DE_DIRECT
  return hipGetLastError();
}

hipError_t launch_render_de_batch(const FrameDesc *table_dev, int nframes, int max_w, int max_h,
                                  int norm, bool all_axis, bool count, hipStream_t s) {
  const dim3 grid((max_w + 7) / 8, (max_h + 7) / 8, nframes);
#define DQJ_DE_BATCH(NM, AX)                                                                 \
  do {                                                                                       \
    if (count)                                                                               \
      hipLaunchKernelGGL((render_de_batch_kernel<NM, AX, true>), grid, dim3(64), 0, s, table_dev); \
    else                                                                                     \
      hipLaunchKernelGGL((render_de_batch_kernel<NM, AX, false>), grid, dim3(64), 0, s, table_dev); \
  } while (0)
  if (norm == 0) {
    if (all_axis)
      DQJ_DE_BATCH(0, true);
    else
      DQJ_DE_BATCH(0, false);
  } else {
    if (all_axis)
      DQJ_DE_BATCH(1, true);
    else
      DQJ_DE_BATCH(1, false);
  }
#undef DQJ_DE_BATCH
  return hipGetLastError();
}

}  // namespace dqj

// ---------------------------------------------------------------------------
// Persistent lane-refill form.
// ---------------------------------------------------------------------------
namespace dqj {

using namespace persist;

namespace {

enum { DE_IDLE = 0, DE_MARCH = 1, DE_BISECT = 2, DE_NORMAL = 3 };

}  // namespace

template <int NORM, bool AXIS, bool BATCH, bool COUNT>
__global__ __launch_bounds__(1024) void render_de_refill_kernel(FrameDesc single,
                                                                const FrameDesc *__restrict__ table,
                                                                const LaunchHeader *__restrict__ hdr,
                                                                int nframes, uint32_t total_tiles,
                                                                uint32_t *__restrict__ counter,
                                                                int TW, int TH) {
  const int lane = lane_id();
  const int tile_rays = TW * TH;
  if constexpr (BATCH) {
    if (hdr) {
      nframes = (int)uniform(((ConstHeader)hdr)->nframes);
      total_tiles = uniform(((ConstHeader)hdr)->total_tiles);
    }
  }
  const float kNaN = __builtin_nanf("");
  const ConstFrame ctable = (ConstFrame)table;
  typename FramePtr<BATCH>::type F;
  if constexpr (BATCH)
    F = nullptr;
  else
    F = &single;
  int frame = -1;
  uint32_t tile_local = 0;
  int next_r = 0;
  bool have_tile = false, pending = false, exhausted = false;
  uint32_t pend_tile = 0;
  QConst K;     // per-lane copies of the update's constants (vector-register operands)
#pragma unroll
  for (int i = 0; i < 8; ++i) K.h[i] = 0.0f;
  K.R2c = K.inv_r2 = K.c0r = 0.0f;
  float ex = 0.0f, ey = 0.0f, ez = 0.0f;
  float l4r2 = 0.0f, eps = 0.0f, smin = 0.0f, smax = 0.0f;
  int N = 1, S = 1;
  // trip counter and deadlines as in render_refill_kernel
  uint32_t trip = 0;
  const uint32_t kIdleAhead = 0x7FFFFFFFu;

  int phase = DE_IDLE;
  DQ<float> z{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
  float q = kNaN;
  float D = 1.0f;          // |z'_n|^2 / (4 R^2)^n of the current march point
  float n2prev = 0.0f;     // |z_n|^2 - c0 of the current point (the next derivative step needs it)
  uint32_t dl = kIdleAhead;
  int pix = 0;
  float dx = 0, dy = 0, dz = 0, t0 = 0, t1 = 0, t = 0, tprev = 0;
  int k = 0, b = 0, sidx = 0, kstar = -1;
  float lo = 0, hi = 0, thit = 0, gx = 0, gy = 0, gz = 0;
  uint32_t it_lane = 0;

  enter_update_mode();
  for (;;) {
    ++trip;
    // ---- one update on every lane, the derivative norm carried along
    D = D * fmaf(n2prev, K.inv_r2, K.c0r);
    const float n2 = de_update<NORM>(z, q, K.h);   // norm minus c0
    n2prev = n2;
    const bool esc = n2 > K.R2c;
    const bool expired = (int)(trip - dl) >= 0;

    // ---- an escaped march point: its distance estimate and the next step
    bool fast = false;
    float de = 0.0f;
    if (esc && phase == DE_MARCH) {
      const int m = N - (int)(dl - trip);
      de = de_estimate(n2 + K.h[0], D, m, l4r2);
      const float tn = t + fminf(fmaxf(de, smin), smax);
      fast = de >= eps && tn <= t1 && k + 1 < S;
      if (fast) {
        if (COUNT) it_lane += (uint32_t)m;
        tprev = t;
        t = tn;
        ++k;
        de_start<AXIS>(F->P, fmaf(t, dx, ex), fmaf(t, dy, ey), fmaf(t, dz, ez), K.h[0], z, q);
        n2prev = norm2_of<NORM>(z, q);
        D = 1.0f;
        dl = trip + (uint32_t)N;
      }
    }

    // ---- everything else that retires: march end (hit, miss), bisection, normal
    if ((esc || expired) && !fast) {
      const KParams &P = F->P;
      float n2c = n2;
      asm volatile("" : "+v"(n2c));
      const bool inside = !(n2c > K.R2c);
      const int m = N - (int)(dl - trip);
      if (COUNT) it_lane += (uint32_t)m;
      bool next_normal = false, restart = false;
      float tr = 0.0f;
      if (phase == DE_MARCH) {
        if (inside) {              // the step landed inside: bisect it (or hit at t0)
          kstar = k;
          if (k == 0) {
            thit = t0;
            next_normal = true;
          } else {
            lo = tprev;
            hi = t;
            if (P.B == 0) {
              thit = 0.5f * (lo + hi);
              next_normal = true;
            } else {
              b = 0;
              phase = DE_BISECT;
              tr = 0.5f * (lo + hi);
              restart = true;
            }
          }
        } else if (de < eps) {     // the estimate fell below the threshold: hit here
          kstar = k;
          thit = t;
          next_normal = true;
        } else {                   // left the box or ran out of steps: miss
          write_pixel(F->out, pix, miss_pixel(DQJ_FLAG_BOX));
          phase = DE_IDLE;
        }
      } else if (phase == DE_BISECT) {
        const float tm = 0.5f * (lo + hi);
        if (inside)
          hi = tm;
        else
          lo = tm;
        ++b;
        if (b >= P.B) {
          thit = 0.5f * (lo + hi);
          next_normal = true;
        } else {
          tr = 0.5f * (lo + hi);
          restart = true;
        }
      } else {   // DE_NORMAL: stencil point sidx just retired (b: least escape index)
        stencil_add(gx, gy, gz, b, sidx, pot_log(n2c + K.h[0]), m);
        ++sidx;
      }
      if (next_normal) {
        phase = DE_NORMAL;
        // the four-neighbour normal is formed after the frame: no stencil points
        sidx = P.normal_mode != 0 ? 6 : 0;
        gx = gy = gz = 0.0f;
      }
      if (phase == DE_NORMAL && sidx == 6) {   // the hit is finished (g = 0: no stencil)
        const float g[3] = {gx, gy, gz};
        const float d[3] = {dx, dy, dz};
        PixelOut r;
        finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
        write_pixel(F->out, pix, r);
        phase = DE_IDLE;
      }
      float px = 0, py = 0, pz = 0;
      if (restart) {
        px = fmaf(tr, dx, ex);
        py = fmaf(tr, dy, ey);
        pz = fmaf(tr, dz, ez);
      } else if (phase == DE_NORMAL) {
        const int axis = sidx >> 1;
        const float hs = (sidx & 1) ? -P.h : P.h;
        px = fmaf(thit, dx, ex) + (axis == 0 ? hs : 0.0f);
        py = fmaf(thit, dy, ey) + (axis == 1 ? hs : 0.0f);
        pz = fmaf(thit, dz, ez) + (axis == 2 ? hs : 0.0f);
      }
      if (phase != DE_IDLE) {
        de_start<AXIS>(P, px, py, pz, K.h[0], z, q);
        dl = trip + (uint32_t)N;
      } else {
        z = DQ<float>{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
        q = kNaN;
        dl = trip + kIdleAhead;
      }
    }

    // ---- hand new rays to idle lanes
    uint64_t idle = __builtin_amdgcn_ballot_w64(phase == DE_IDLE);
    while (idle) {
      if (!have_tile) {
        if (exhausted) break;
        if (!pending) {
          uint32_t tt = 0;
          if (lane == 0) tt = atomicAdd(counter, 1u);
          tt = uniform(tt);
          if (tt >= total_tiles) {
            exhausted = true;
            break;
          }
          pend_tile = tt;
          pending = true;
        }
        const int f = BATCH ? find_frame(ctable, nframes, pend_tile) : 0;
        if (f != frame) {
          if (idle != ~0ull) break;  // finish this frame's rays first
          if (COUNT && frame >= 0 && F->out.iters) wave_add_u64(F->out.iters, it_lane);
          it_lane = 0;
          frame = f;
          if constexpr (BATCH) F = ctable + (int)uniform((uint32_t)f);
          load_qconst(F->P, K);
          N = (int)uniform((uint32_t)F->P.N);
          S = (int)uniform((uint32_t)F->P.S);
          ex = uniform_f(F->P.eye[0]);
          ey = uniform_f(F->P.eye[1]);
          ez = uniform_f(F->P.eye[2]);
          l4r2 = uniform_f(F->P.de_log2_4r2);
          eps = uniform_f(F->P.de_eps);
          smin = uniform_f(F->P.de_min_step);
          smax = uniform_f(F->P.de_max_step);
        }
        tile_local = pend_tile - F->tile_begin + F->tile_offset;
        pending = false;
        have_tile = true;
        next_r = 0;
      }
      const int rank = rank_in(idle);
      const int avail = tile_rays - next_r;
      if (phase == DE_IDLE && rank < avail) {
        const KParams &P = F->P;
        const int r = next_r + rank;
        const int i = (int)(tile_local % F->tiles_x) * TW + r % TW;
        const int j = (int)(tile_local / F->tiles_x) * TH + r / TW;
        if (i < P.W && j < P.H) {
          pix = j * P.W + i;
          float d[3];
          pixel_dir(P, i, j, d);
          float ta, tb;
          if (clip_box(P, d, ta, tb)) {
            dx = d[0];
            dy = d[1];
            dz = d[2];
            t0 = ta;
            t1 = tb;
            t = ta;
            tprev = ta;
            k = 0;
            kstar = -1;
            phase = DE_MARCH;
            de_start<AXIS>(P, fmaf(t, dx, ex), fmaf(t, dy, ey), fmaf(t, dz, ez), K.h[0], z, q);
            n2prev = norm2_of<NORM>(z, q);
            D = 1.0f;
            dl = trip + (uint32_t)N;
          } else {
            write_pixel(F->out, pix, miss_pixel(0));
          }
        }
      }
      const int cnt = __popcll(idle);
      next_r += cnt < avail ? cnt : avail;
      if (next_r >= tile_rays) have_tile = false;
      idle = __builtin_amdgcn_ballot_w64(phase == DE_IDLE);
    }

    if (exhausted && !__builtin_amdgcn_ballot_w64(phase != DE_IDLE)) break;
  }
  if (COUNT && frame >= 0 && F->out.iters) wave_add_u64(F->out.iters, it_lane);
}

// Lock-step persistent form: every lane holds one ray and one current point (a march
// point, a bisection point or a normal stencil point). Each pass classifies all lanes'
// points together (the loop runs until the last lane's point escapes or reaches
// max_iter), then every lane advances its own ray once -- step, bisect, accumulate the
// normal, or finish -- and lanes whose ray ended take new rays of the wave's tile. The
// per-point work is paid once per classification, not once per update, and a wave no
// longer waits for its slowest ray: it waits for its slowest point.
template <int NORM, bool AXIS, bool COUNT>
__global__ __launch_bounds__(1024) void render_de_lockstep_kernel(FrameDesc F, uint32_t *__restrict__ counter,
                                                                  int TW, int TH) {
  const KParams &P = F.P;
  const int lane = lane_id();
  const int tile_rays = TW * TH;
  enter_update_mode();
  QConst K;
  load_qconst(P, K);
  const float l4r2 = P.de_log2_4r2;
  const float eps = P.de_eps, smin = P.de_min_step, smax = P.de_max_step;
  const float ex = P.eye[0], ey = P.eye[1], ez = P.eye[2];
  const int N = P.N, S = P.S, B = P.B;

  uint32_t tile = 0;
  int next_r = 0;
  bool have_tile = false, exhausted = false;

  int phase = DE_IDLE;
  int pix = 0;
  float dx = 0, dy = 0, dz = 0, t0 = 0, t1 = 0, t = 0, tprev = 0;
  float px = 0, py = 0, pz = 0;        // the lane's current point
  int k = 0, b = 0, sidx = 0, kstar = -1;
  float lo = 0, hi = 0, thit = 0, gx = 0, gy = 0, gz = 0;
  unsigned long long it_lane = 0;

  for (;;) {
    // ---- hand new rays to idle lanes
    uint64_t idle = __builtin_amdgcn_ballot_w64(phase == DE_IDLE);
    while (idle) {
      if (!have_tile) {
        if (exhausted) break;
        uint32_t tt = 0;
        if (lane == 0) tt = atomicAdd(counter, 1u);
        tt = uniform(tt);
        if (tt >= F.ntiles) {
          exhausted = true;
          break;
        }
        tile = tt;
        next_r = 0;
        have_tile = true;
      }
      const int rank = rank_in(idle);
      const int avail = tile_rays - next_r;
      if (phase == DE_IDLE && rank < avail) {
        const int r = next_r + rank;
        const int i = (int)(tile % F.tiles_x) * TW + r % TW;
        const int j = (int)(tile / F.tiles_x) * TH + r / TW;
        if (i < P.W && j < P.H) {
          pix = j * P.W + i;
          float d[3];
          pixel_dir(P, i, j, d);
          float ta, tb;
          if (clip_box(P, d, ta, tb)) {
            dx = d[0];
            dy = d[1];
            dz = d[2];
            t0 = ta;
            t1 = tb;
            t = ta;
            tprev = ta;
            k = 0;
            kstar = -1;
            phase = DE_MARCH;
            px = fmaf(t, dx, ex);
            py = fmaf(t, dy, ey);
            pz = fmaf(t, dz, ez);
          } else {
            write_pixel(F.out, pix, miss_pixel(0));
          }
        }
      }
      const int cnt = __popcll(idle);
      next_r += cnt < avail ? cnt : avail;
      if (next_r >= tile_rays) have_tile = false;
      idle = __builtin_amdgcn_ballot_w64(phase == DE_IDLE);
    }
    if (exhausted && !__builtin_amdgcn_ballot_w64(phase != DE_IDLE)) break;

    // ---- classify every busy lane's point together
    float n2 = 0.0f, D = 1.0f;
    int m = N;
    bool inside = true;
    if (phase != DE_IDLE) {
      DQ<float> z;
      float qv;
      de_start<AXIS>(P, px, py, pz, K.h[0], z, qv);
      n2 = norm2_of<NORM>(z, qv);
      int n = 0;
      while (n < N) {
        ++n;
        D = D * fmaf(n2, K.inv_r2, K.c0r);
        n2 = de_update<NORM>(z, qv, K.h);
        if (n2 > K.R2c) {
          inside = false;
          break;
        }
      }
      n2 += K.h[0];
      m = inside ? N : n;
      if (COUNT) it_lane += (unsigned long long)m;
    }

    // ---- advance each lane's ray by one point
    bool next_normal = false;
    if (phase == DE_MARCH) {
      if (inside) {               // the step landed inside: bisect it (or hit at t0)
        kstar = k;
        if (k == 0) {
          thit = t0;
          next_normal = true;
        } else if (B == 0) {
          thit = 0.5f * (tprev + t);
          next_normal = true;
        } else {
          lo = tprev;
          hi = t;
          b = 0;
          phase = DE_BISECT;
        }
      } else {
        const float de = de_estimate(n2, D, m, l4r2);
        if (de < eps) {           // the estimate fell below the threshold: hit here
          kstar = k;
          thit = t;
          next_normal = true;
        } else {
          const float tn = t + fminf(fmaxf(de, smin), smax);
          if (tn <= t1 && k + 1 < S) {
            tprev = t;
            t = tn;
            ++k;
            px = fmaf(t, dx, ex);
            py = fmaf(t, dy, ey);
            pz = fmaf(t, dz, ez);
          } else {                // left the box or ran out of steps: miss
            write_pixel(F.out, pix, miss_pixel(DQJ_FLAG_BOX));
            phase = DE_IDLE;
          }
        }
      }
    } else if (phase == DE_BISECT) {
      const float tm = 0.5f * (lo + hi);
      if (inside)
        hi = tm;
      else
        lo = tm;
      ++b;
      if (b >= B) {
        thit = 0.5f * (lo + hi);
        next_normal = true;
      }
    } else if (phase == DE_NORMAL) {   // (b: the stencil's least escape index)
      stencil_add(gx, gy, gz, b, sidx, pot_log(n2), m);
      ++sidx;
    }
    if (next_normal) {
      phase = DE_NORMAL;
      // the four-neighbour normal is formed after the frame: no stencil points
      sidx = P.normal_mode != 0 ? 6 : 0;
      gx = gy = gz = 0.0f;
    }
    if (phase == DE_NORMAL && sidx == 6) {   // the hit is finished (g = 0: no stencil)
      const float g[3] = {gx, gy, gz};
      const float d[3] = {dx, dy, dz};
      PixelOut r;
      finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
      write_pixel(F.out, pix, r);
      phase = DE_IDLE;
    }
    // next point of a bisecting or normal lane
    if (phase == DE_BISECT) {
      const float tm = 0.5f * (lo + hi);
      px = fmaf(tm, dx, ex);
      py = fmaf(tm, dy, ey);
      pz = fmaf(tm, dz, ez);
    } else if (phase == DE_NORMAL) {
      const int axis = sidx >> 1;
      const float hs = (sidx & 1) ? -P.h : P.h;
      px = fmaf(thit, dx, ex) + (axis == 0 ? hs : 0.0f);
      py = fmaf(thit, dy, ey) + (axis == 1 ? hs : 0.0f);
      pz = fmaf(thit, dz, ez) + (axis == 2 ? hs : 0.0f);
    }
  }
  if (COUNT && F.out.iters) wave_add_u64(F.out.iters, it_lane);
}

__global__ void de_reset_counter_kernel(uint32_t *counter) { *counter = 0u; }

template <bool BATCH, bool COUNT>
static void launch_de_variant(const FrameDesc &single, const FrameDesc *table,
                              const LaunchHeader *hdr, int nframes, uint32_t total_tiles,
                              int norm, bool axis, uint32_t *counter, const Sched &s, int blocks,
                              int threads, hipStream_t stream) {
#define DQJ_DE_LAUNCH(NM, AX)                                                                   \
  hipLaunchKernelGGL((render_de_refill_kernel<NM, AX, BATCH, COUNT>), dim3(blocks),              \
                     dim3(threads), 0, stream, single, table, hdr, nframes, total_tiles, counter, \
                     s.tile_w, s.tile_h)
  if (norm == 0) {
    if (axis)
      DQJ_DE_LAUNCH(0, true);
    else
      DQJ_DE_LAUNCH(0, false);
  } else {
    if (axis)
      DQJ_DE_LAUNCH(1, true);
    else
      DQJ_DE_LAUNCH(1, false);
  }
#undef DQJ_DE_LAUNCH
}

template <bool BATCH>
static hipError_t launch_de_impl(const FrameDesc &single, const FrameDesc *table,
                                 const LaunchHeader *hdr, int nframes, uint32_t total_tiles,
                                 int norm, bool axis, bool count, uint32_t *counter,
                                 const Sched &s, int cus, hipStream_t stream) {
  hipLaunchKernelGGL(de_reset_counter_kernel, dim3(1), dim3(1), 0, stream, counter);
  const int threads = 64 * s.waves_per_block;
  const int blocks = cus * s.blocks_per_cu;
  if (count)
    launch_de_variant<BATCH, true>(single, table, hdr, nframes, total_tiles, norm, axis, counter, s,
                                   blocks, threads, stream);
  else
    launch_de_variant<BATCH, false>(single, table, hdr, nframes, total_tiles, norm, axis, counter, s,
                                    blocks, threads, stream);
  return hipGetLastError();
}

hipError_t launch_render_de_lockstep(const FrameDesc &frame, uint32_t *counter, const Sched &s,
                                     int cus, hipStream_t stream) {
  hipLaunchKernelGGL(de_reset_counter_kernel, dim3(1), dim3(1), 0, stream, counter);
  const int threads = 64 * s.waves_per_block;
  const int blocks = cus * s.blocks_per_cu;
  const bool axis = frame.P.axis_slice != 0, count = frame.out.iters != nullptr;
#define DQJ_DE_LS(NM, AX, CT)                                                                  \
  hipLaunchKernelGGL((render_de_lockstep_kernel<NM, AX, CT>), dim3(blocks), dim3(threads), 0, \
                     stream, frame, counter, s.tile_w, s.tile_h)
  if (frame.P.norm == 0) {
    if (axis) {
      if (count) DQJ_DE_LS(0, true, true); else DQJ_DE_LS(0, true, false);
    } else {
      if (count) DQJ_DE_LS(0, false, true); else DQJ_DE_LS(0, false, false);
    }
  } else {
    if (axis) {
      if (count) DQJ_DE_LS(1, true, true); else DQJ_DE_LS(1, true, false);
    } else {
      if (count) DQJ_DE_LS(1, false, true); else DQJ_DE_LS(1, false, false);
    }
  }
#undef DQJ_DE_LS
  return hipGetLastError();
}

hipError_t launch_render_de_refill(const FrameDesc &frame, uint32_t *counter, const Sched &s, int cus,
                                   hipStream_t stream) {
  return launch_de_impl<false>(frame, nullptr, nullptr, 1, frame.ntiles, frame.P.norm,
                               frame.P.axis_slice != 0, frame.out.iters != nullptr, counter, s, cus,
                               stream);
}

hipError_t launch_render_de_refill_batch(const FrameDesc *table_dev, const LaunchHeader *hdr_dev,
                                         int nframes, uint32_t total_tiles, int norm, bool all_axis,
                                         bool any_count, uint32_t *counter, const Sched &s, int cus,
                                         hipStream_t stream) {
  FrameDesc dummy;
  memset(&dummy, 0, sizeof dummy);
  return launch_de_impl<true>(dummy, table_dev, hdr_dev, nframes, total_tiles, norm, all_axis,
                              any_count, counter, s, cus, stream);
}

}  // namespace dqj

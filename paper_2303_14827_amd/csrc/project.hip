// project.hip -- projection ("shadow") rendering, the second dimension reduction of
// paragraph "Dimension Reduction": the set of R^8 seen through its projection onto the
// slice's 3D space. A world point x is inside when some point of R^8 that projects onto
// it is inside; that fibre is sampled by F offsets (o_f, given by the caller), so the
// test is: some o_f has O + x U + y V + z W + o_f inside (N updates without escape). The
// march, bisection and shade are those of the slice render; the potential of the normal
// is the least potential over the F points (the potential of the union of the fibre's
// sets).
//
// A pixel is rendered by a group of L adjacent lanes: each sample's fibre points are
// shared out over the group, L at a time (lane s of the group takes points s, s + L, ...),
// and the group decides together after each round of L points. A 512 x 512 frame is
// 262144 pixels, half of the chip's 524288 lanes at 8 waves per SIMD; with L > 1 the
// frame fills the chip. Every decision (inside, the bisection bracket, the normal) is
// the same as with one lane per pixel, so is the image; the count takes the points
// in fibre order up to the first inside one, as the one-lane loop does. The offsets
// sit in LDS, read per lane.
#include "dq_device.h"
#include "launch.h"
#include "persist.h"
#include "qform.h"
#include "project.h"
#include "tile_order.h"

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

// Fibre offsets of the launch, copied once per block.
struct FiberLds {
  float4 off[kMaxFiber][2];
};

__device__ __forceinline__ DQ<float> offset_point(const DQ<float> &z0, const FiberLds &fl, int f) {
  const float4 lo = fl.off[f][0], hi = fl.off[f][1];
  return DQ<float>{z0.a0 + lo.x, z0.a1 + lo.y, z0.a2 + lo.z, z0.a3 + lo.w,
                   z0.b0 + hi.x, z0.b1 + hi.y, z0.b2 + hi.z, z0.b3 + hi.w};
}

// Bits (one per lane of this lane's group of L) of the lanes whose p holds.
template <int L>
__device__ __forceinline__ unsigned group_bits(bool p) {
  const unsigned long long b = __builtin_amdgcn_ballot_w64(p);
  return (unsigned)(b >> ((threadIdx.x & 63) & ~(L - 1))) & ((1u << L) - 1u);
}

// 1 when some fibre point over world point (x, y, w) is inside; with COUNT, counts the
// updates of the points up to the first inside one in fibre order. Called by the whole
// group.
template <int NORM, int L, bool COUNT>
__device__ __forceinline__ bool inside_union(const KParams &P, const QC &K, const FiberLds &fl, int F,
                                             int sub, float x, float y, float w,
                                             unsigned long long &iters) {
  const DQ<float> z0 = slice_map<float>(P, x, y, w);
  for (int f0 = 0; f0 < F; f0 += L) {
    const int f = f0 + sub;
    int m = -1;   // -1: no point for this lane in the last round
    if (f < F) {
      float n2;
      m = classify_q<NORM>(offset_point(z0, fl, f), K, P.N, &n2);
    }
    const unsigned in = group_bits<L>(m == 0);
    if constexpr (COUNT) {
      const int first = in ? __builtin_ctz(in) : L;
      if (m >= 0 && sub <= first) iters += m ? m : P.N;
    }
    if (in) return true;
  }
  return false;
}

// Least escape potential over the fibre points of world point (x, y, w), on every lane
// of the group, as its two parts (*lv, the return value m; see stencil_add). A lane
// without fibre points starts from (+inf, 0), which every point's potential is below.
template <int NORM, int L, bool COUNT>
__device__ __forceinline__ int potential_union(const KParams &P, const QC &K, const FiberLds &fl,
                                               int F, int sub, float x, float y, float w,
                                               unsigned long long &iters, float *lv) {
  const DQ<float> z0 = slice_map<float>(P, x, y, w);
  float best = __builtin_huge_valf();
  int best_m = 0;
  for (int f = sub; f < F; f += L) {
    float n2;
    int m = classify_q<NORM>(offset_point(z0, fl, f), K, P.N, &n2);
    m = m ? m : P.N;
    if constexpr (COUNT) iters += m;
    const float l = pot_log(n2);
    if (pot_less(l, m, best, best_m)) {
      best = l;
      best_m = m;
    }
  }
#pragma unroll
  for (int s = 1; s < L; s <<= 1) {
    const float o = __shfl_xor(best, s, 64);
    const int om = __shfl_xor(best_m, s, 64);
    if (pot_less(o, om, best, best_m)) {
      best = o;
      best_m = om;
    }
  }
  *lv = best;
  return best_m;
}

template <int NORM, int L, bool COUNT>
__device__ void render_pixel_project(const KParams &P, const QC &K, const FiberLds &fl, int F,
                                     int sub, int i, int j, PixelOut &r,
                                     unsigned long long &iters) {
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
    if (inside_union<NORM, L, COUNT>(P, K, fl, F, sub, fmaf(t, d[0], P.eye[0]), fmaf(t, d[1], P.eye[1]),
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
      if (inside_union<NORM, L, COUNT>(P, K, fl, F, sub, fmaf(tm, d[0], P.eye[0]), fmaf(tm, d[1], P.eye[1]),
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
  int m0 = 0;
  // (the four-neighbour normal is formed after the frame: no stencil here)
  if (P.normal_mode == 0) {
    for (int a = 0; a < 3; ++a) {
      for (int sgn = 0; sgn < 2; ++sgn) {
        float x[3] = {ph[0], ph[1], ph[2]};
        x[a] = sgn == 0 ? ph[a] + P.h : ph[a] - P.h;
        float lv;
        const int m = potential_union<NORM, L, COUNT>(P, K, fl, F, sub, x[0], x[1], x[2], iters, &lv);
        stencil_add(g[0], g[1], g[2], m0, 2 * a + sgn, lv, m);
      }
    }
  }
  finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
}

template <int NORM, int L, bool COUNT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void render_project_kernel(KParams P, FiberTable fb, int F,
                                                             KOut out) {
  __shared__ FiberLds fl;
  if (threadIdx.x == 0) {
    for (int f = 0; f < F; ++f) {
      fl.off[f][0] = make_float4(fb.off[f][0], fb.off[f][1], fb.off[f][2], fb.off[f][3]);
      fl.off[f][1] = make_float4(fb.off[f][4], fb.off[f][5], fb.off[f][6], fb.off[f][7]);
    }
  }
  __syncthreads();
  // Each wave renders a compact tile of 64 / L pixels (8 x 8, 8 x 4 or 4 x 4), whose rays
  // are more alike than a row's; the block's four waves form a 2 x 2 arrangement of them.
  // Blocks go centre-out in dispatch order (tile_order.h): the long rays near the image
  // centre start first, the short ones at the edge fill the launch's ramp-down (three
  // 512^2 frames 7% faster, the same images).
  constexpr int kWaveW = L == 4 ? 4 : 8, kWaveH = 64 / L / kWaveW;
  const int sub = threadIdx.x & (L - 1);
  const int wave = threadIdx.x >> 6;
  const int pix = (threadIdx.x & 63) / L;
  const uint32_t t = centre_out_tile(blockIdx.y * gridDim.x + blockIdx.x, (int)gridDim.x, (int)gridDim.y);
  const int bx = (int)(t % gridDim.x), by = (int)(t / gridDim.x);
  const int i = bx * (2 * kWaveW) + (wave & 1) * kWaveW + pix % kWaveW;
  const int j = by * (2 * kWaveH) + (wave >> 1) * kWaveH + pix / kWaveW;
  unsigned long long iters = 0;
  enter_update_mode();
  QC K;
  K.h[0] = to_vgpr(P.c[0]);
#pragma unroll
  for (int q = 1; q < 8; ++q) K.h[q] = to_vgpr(0.5f * P.c[q]);
  K.R2c = to_vgpr(P.R2 - P.c[0]);
  if (i < P.W && j < P.H) {
    PixelOut r;
    render_pixel_project<NORM, L, COUNT>(P, K, fl, F, sub, i, j, r, iters);
    if (sub == 0) write_pixel(out, (int64_t)j * P.W + i, r);
  }
  if constexpr (COUNT) wave_add_u64(out.iters, iters);
}

// Several projection frames in one launch. Block g of the launch renders block g / n of
// frame g % n (the frames interleaved in dispatch order, so one frame's slow blocks overlap
// the others' work), each frame's blocks taken centre-out; the fibre offsets come from the
// frame's record in device memory. Otherwise the body is render_project_kernel's.
template <int NORM, int L, bool COUNT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void render_project_batch_kernel(
    const FrameDesc *__restrict__ table, const ProjFiber *__restrict__ fibers, uint32_t nf) {
  constexpr int kWaveW = L == 4 ? 4 : 8, kWaveH = 64 / L / kWaveW;
  const uint32_t g = blockIdx.x;
  const uint32_t fi = g % nf;
  const persist::ConstFrame Fd = (persist::ConstFrame)table + fi;
  const KParams &P = Fd->P;
  const int X = (P.W + 2 * kWaveW - 1) / (2 * kWaveW), Y = (P.H + 2 * kWaveH - 1) / (2 * kWaveH);
  const uint32_t b = g / nf;
  if (b >= (uint32_t)(X * Y)) return;   // a frame smaller than the largest (whole block)
  const ProjFiber *pf = fibers + fi;
  const int F = pf->F;
  __shared__ FiberLds fl;
  if ((int)threadIdx.x < F) {
    const float *o = pf->off[threadIdx.x];
    fl.off[threadIdx.x][0] = make_float4(o[0], o[1], o[2], o[3]);
    fl.off[threadIdx.x][1] = make_float4(o[4], o[5], o[6], o[7]);
  }
  __syncthreads();
  const int sub = threadIdx.x & (L - 1);
  const int wave = threadIdx.x >> 6;
  const int pix = (threadIdx.x & 63) / L;
  const uint32_t t = centre_out_tile(b, X, Y);
  const int bx = (int)(t % (uint32_t)X), by = (int)(t / (uint32_t)X);
  const int i = bx * (2 * kWaveW) + (wave & 1) * kWaveW + pix % kWaveW;
  const int j = by * (2 * kWaveH) + (wave >> 1) * kWaveH + pix / kWaveW;
  unsigned long long iters = 0;
  enter_update_mode();
  QC K;
  K.h[0] = to_vgpr(P.c[0]);
#pragma unroll
  for (int q = 1; q < 8; ++q) K.h[q] = to_vgpr(0.5f * P.c[q]);
  K.R2c = to_vgpr(P.R2 - P.c[0]);
  if (i < P.W && j < P.H) {
    PixelOut r;
    render_pixel_project<NORM, L, COUNT>(P, K, fl, F, sub, i, j, r, iters);
    if (sub == 0) write_pixel(Fd->out, (int64_t)j * P.W + i, r);
  }
  if constexpr (COUNT) {
    if (Fd->out.iters) wave_add_u64(Fd->out.iters, iters);
  }
}

template <int L>
void launch_batch_lanes(const FrameDesc *table, const ProjFiber *fibers, int n, int max_w, int max_h,
                        int norm, bool count, hipStream_t s) {
  constexpr int kWaveW = L == 4 ? 4 : 8, kWaveH = 64 / L / kWaveW;
  const uint32_t per_frame = (uint32_t)(((max_w + 2 * kWaveW - 1) / (2 * kWaveW)) *
                                        ((max_h + 2 * kWaveH - 1) / (2 * kWaveH)));
  const dim3 grid(per_frame * (uint32_t)n);
  if (norm == 0) {
    if (count)
      hipLaunchKernelGGL((render_project_batch_kernel<0, L, true>), grid, dim3(256), 0, s, table, fibers, (uint32_t)n);
    else
      hipLaunchKernelGGL((render_project_batch_kernel<0, L, false>), grid, dim3(256), 0, s, table, fibers, (uint32_t)n);
  } else {
    if (count)
      hipLaunchKernelGGL((render_project_batch_kernel<1, L, true>), grid, dim3(256), 0, s, table, fibers, (uint32_t)n);
    else
      hipLaunchKernelGGL((render_project_batch_kernel<1, L, false>), grid, dim3(256), 0, s, table, fibers, (uint32_t)n);
  }
}

// The counting kernels run only where the caller asked for the update count.
template <int L>
void launch_lanes(const KParams &P, const FiberTable &fb, int F, const KOut &out, hipStream_t s) {
  constexpr int kWaveW = L == 4 ? 4 : 8, kWaveH = 64 / L / kWaveW;
  const dim3 grid((P.W + 2 * kWaveW - 1) / (2 * kWaveW), (P.H + 2 * kWaveH - 1) / (2 * kWaveH));
  const bool count = out.iters != nullptr;
  if (P.norm == 0) {
    if (count)
      hipLaunchKernelGGL((render_project_kernel<0, L, true>), grid, dim3(256), 0, s, P, fb, F, out);
    else
      hipLaunchKernelGGL((render_project_kernel<0, L, false>), grid, dim3(256), 0, s, P, fb, F, out);
  } else {
    if (count)
      hipLaunchKernelGGL((render_project_kernel<1, L, true>), grid, dim3(256), 0, s, P, fb, F, out);
    else
      hipLaunchKernelGGL((render_project_kernel<1, L, false>), grid, dim3(256), 0, s, P, fb, F, out);
  }
}

// Lanes per pixel: the least of 1, 2 and 4 that puts about 2^20 lanes (twice the chip's
// 524288 at 8 waves per SIMD) into the launch, and at most F (a larger group would leave
// lanes without a point in every round). On a 512 x 512 frame of 16 points, 4 lanes per
// pixel took a frame from 3.3 to 2.5 ms; with the compact wave tiles, 4 lanes take 1.9 ms
// against 2.1 for 2. On 1024 x 1024, more than one lane per pixel gained nothing or cost
// time.
int project_lanes(const KParams &P, int F) {
  int lanes = 1;
  while (lanes < 4 && 2 * lanes <= F && (int64_t)P.W * P.H * lanes < (int64_t(1) << 20)) lanes *= 2;
  return lanes;
}

}  // namespace

// Lanes per pixel for a batch: the least of 1, 2 and 4 that puts about 2^21 lanes in the
// launch (its blocks overlap across frames, so more are in flight than in one frame's
// launch), and at most the smallest F.
hipError_t launch_render_project_batch(const FrameDesc *table_dev, const ProjFiber *fibers_dev,
                                       int nframes, int max_w, int max_h, int norm, bool count,
                                       uint64_t pixels, int min_fiber, hipStream_t s) {
  if (nframes < 1 || min_fiber < 1 || min_fiber > kMaxFiber) return hipErrorInvalidValue;
  int lanes = 1;
  while (lanes < 4 && 2 * lanes <= min_fiber && pixels * (uint64_t)lanes < (uint64_t(1) << 21)) lanes *= 2;
  switch (lanes) {
    case 1: launch_batch_lanes<1>(table_dev, fibers_dev, nframes, max_w, max_h, norm, count, s); break;
    case 2: launch_batch_lanes<2>(table_dev, fibers_dev, nframes, max_w, max_h, norm, count, s); break;
    default: launch_batch_lanes<4>(table_dev, fibers_dev, nframes, max_w, max_h, norm, count, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_render_project(const KParams &P, const FiberTable &fb, int F, const KOut &out,
                                 hipStream_t s) {
  if (F < 1 || F > kMaxFiber) return hipErrorInvalidValue;
  switch (project_lanes(P, F)) {
    case 1: launch_lanes<1>(P, fb, F, out, s); break;
    case 2: launch_lanes<2>(P, fb, F, out, s); break;
    default: launch_lanes<4>(P, fb, F, out, s); break;
  }
  return hipGetLastError();
}

}  // namespace dqj

// split.hip -- split-precision form of the ray march.
//
//   1. march_fp16: the fixed-step march (section "Ray-Marching") in packed FP16. A lane
//      owns a ray and classifies two consecutive samples k, k+1 per packed register
//      (half2), so every v_pk_fma_f16 advances two samples. Escape is tracked as the
//      running maximum of ||z_n||^2 (v_pk_max_f16 ignores NaN, so an escaped half stays
//      escaped after it overflows). FP16 orbits near the set's boundary part from the
//      exact ones after some updates, so the march trusts an escape only when it came
//      within T16 = N - ceil(N/4) updates: the samples of pairs that escaped later span a
//      range [kcf, kcl] that FP32 re-checks. The first pair still bounded after N updates
//      gives the FP16 inside sample khat. A ray with neither is a miss; every other ray
//      goes to a compacted candidate list.
//   2. verify_fp32: for each listed ray, classify in FP32 from min(kcf, khat) - w to the
//      first inside sample k32 (up to kcl + w when there is no khat: past it, a miss),
//      confirm that samples k32+1 .. k32+w are inside too, bisect [t_{k32-1}, t_{k32}] in
//      FP32, take the central-difference normal and shade. A ray whose FP32 classes flip
//      within the window after k32, or whose scan starts inside, goes to a second list.
//   3. rebisect_fp64: for each ray of the second list, classify from k - w in FP64 (k
//      the listed sample) to the first inside sample, marching on past the window if
//      needed and back to the start of the inside run if the first sample is already
//      inside, then bisect, take the normal and shade in FP64.
// The three kernels run back to back on one stream; list lengths stay on the device.
#include <cstring>

#include "dq_device.h"
#include "launch.h"
#include "persist.h"
#include "qform.h"
#include "refill.h"
#include "split.h"

namespace dqj {

using namespace persist;

namespace {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

struct DQH {
  h2 a0, a1, a2, a3, b0, b1, b2, b3;
};

__device__ __forceinline__ h2 hfma(h2 a, h2 b, h2 c) { return __builtin_elementwise_fma(a, b, c); }
// Smaller of the two halves (one SDWA instruction; the values here are never NaN).
__device__ __forceinline__ _Float16 min_halves(h2 a) {
  _Float16 r;
  asm("v_min_f16_sdwa %0, %1, %1 dst_sel:WORD_0 dst_unused:UNUSED_PAD src0_sel:WORD_0 "
      "src1_sel:WORD_1"
      : "=v"(r)
      : "v"(a));
  return r;
}
// min(a, b) for finite operands (no canonicalising instruction in front).
__device__ __forceinline__ float fmin_raw(float a, float b) {
  float r;
  asm("v_min_f32_e32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
// Packed maximum that ignores a NaN operand. Written out because the generic form
// first canonicalises its loop-carried operand (an extra instruction per update).
__device__ __forceinline__ h2 hmax_raw(h2 a, h2 b) {
  h2 r;
  asm("v_pk_max_f16 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ h2 hsplat(float v) { return h2{(_Float16)v, (_Float16)v}; }
// Two FP32 values rounded to nearest FP16 and packed (written out so the compiler does
// not fuse the rounding into a mixed-precision FMA, which issues several times slower
// than an FP32 FMA followed by this conversion on gfx950).
__device__ __forceinline__ h2 hpack(float lo, float hi) {
  h2 r;
  asm("v_cvt_pk_f16_f32 %0, %1, %2" : "=v"(r) : "v"(lo), "v"(hi));
  return r;
}

// One packed update of two independent points (one per half), as dq_update.
template <int NORM>
__device__ __forceinline__ h2 pk_update(DQH &z, h2 &s, const h2 *c) {
  const h2 ta = z.a0 + z.a0;
  const h2 tb = z.b0 + z.b0;
  const h2 dot = hfma(z.a3, z.b3, hfma(z.a2, z.b2, z.a1 * z.b1));
  z.b1 = hfma(tb, z.a1, hfma(ta, z.b1, c[5]));
  z.b2 = hfma(tb, z.a2, hfma(ta, z.b2, c[6]));
  z.b3 = hfma(tb, z.a3, hfma(ta, z.b3, c[7]));
  z.b0 = hfma(hsplat(-2.0f), dot, hfma(ta, z.b0, c[4]));
  z.a1 = hfma(ta, z.a1, c[1]);
  z.a2 = hfma(ta, z.a2, c[2]);
  z.a3 = hfma(ta, z.a3, c[3]);
  z.a0 = hfma(z.a0, z.a0, c[0]) - s;
  s = hfma(z.a3, z.a3, hfma(z.a2, z.a2, z.a1 * z.a1));
  h2 n2 = hfma(z.a0, z.a0, s);
  if (NORM == 0) n2 = hfma(z.b3, z.b3, hfma(z.b2, z.b2, hfma(z.b1, z.b1, hfma(z.b0, z.b0, n2))));
  return n2;
}

// Pixel direction in FP64 (for the FP64 pass).
__device__ __forceinline__ void pixel_dir64(const KParams64 &P, int i, int j, double d[3]) {
  const double sx = fma((double)(2 * i + 1), P.inv_w, -1.0) * P.sx_scale;
  const double sy = fma(-(double)(2 * j + 1), P.inv_h, 1.0) * P.sy_scale;
  double v[3];
  for (int k = 0; k < 3; ++k) v[k] = fma(sy, P.up[k], fma(sx, P.right[k], P.fwd[k]));
  const double inv = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  d[0] = v[0] * inv;
  d[1] = v[1] * inv;
  d[2] = v[2] * inv;
}

__device__ __forceinline__ bool clip_box64(const KParams64 &P, const double d[3], double &t0,
                                           double &t1) {
  double tn = 0.0, tf = INFINITY;
  for (int k = 0; k < 3; ++k) {
    const double o = P.eye[k];
    if (d[k] == 0.0) {
      if (o < P.bmin[k] || o > P.bmax[k]) return false;
      continue;
    }
    double ta = (P.bmin[k] - o) / d[k];
    double tb = (P.bmax[k] - o) / d[k];
    if (ta > tb) {
      const double s = ta;
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

template <typename P_T, typename T>
__device__ __forceinline__ DQ<T> slice_map_t(const P_T &P, T x, T y, T z) {
  T v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    v[k] = fma(z, T(P.sw[k]), fma(y, T(P.sv[k]), fma(x, T(P.su[k]), T(P.so[k]))));
  return DQ<T>{v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
}

// Classify the world point eye + t d (precision T). Returns the escape index m
// (N when inside) and sets *inside and *n2.
template <int NORM, typename P_T, typename T>
__device__ __forceinline__ int classify_t(const P_T &P, const T *c, int N, T R2, T t, const T d[3],
                                          T hx, T hy, T hz, bool *inside, T *n2) {
  DQ<T> z = slice_map_t<P_T, T>(P, fma(t, d[0], T(P.eye[0])) + hx, fma(t, d[1], T(P.eye[1])) + hy,
                                fma(t, d[2], T(P.eye[2])) + hz);
  const int m = dq_classify<NORM>(z, c, N, R2, n2);
  *inside = m == 0;
  return m ? m : N;
}

// Bisection + central-difference normal + shade for a hit at sample k (precision T).
template <int NORM, typename P_T, typename T>
__device__ __forceinline__ uint32_t finish_ray(const P_T &P, const T *c, int N, int B, T R2, T h,
                                               const T d[3], T t0, T dt, int k, uint8_t flags,
                                               PixelOut &r) {
  uint32_t it = 0;
  T thit;
  if (k == 0) {
    thit = t0;
  } else {
    T lo = fma(T(k - 1), dt, t0), hi = fma(T(k), dt, t0);
    for (int b = 0; b < B; ++b) {
      const T tm = T(0.5) * (lo + hi);
      bool in;
      T n2;
      it += classify_t<NORM>(P, c, N, R2, tm, d, T(0), T(0), T(0), &in, &n2);
      if (in)
        hi = tm;
      else
        lo = tm;
    }
    thit = T(0.5) * (lo + hi);
  }
  T g[3] = {T(0), T(0), T(0)};
  int m0 = 0;
  // (the four-neighbour normal is formed after the frame: no stencil here)
  for (int a = 0; a < 3 && P.normal_mode == 0; ++a) {
    for (int sg = 0; sg < 2; ++sg) {
      const T hs = sg == 0 ? h : -h;
      bool in;
      T n2;
      const int m = classify_t<NORM>(P, c, N, R2, thit, d, a == 0 ? hs : T(0), a == 1 ? hs : T(0),
                                     a == 2 ? hs : T(0), &in, &n2);
      it += m;
      stencil_add(g[0], g[1], g[2], m0, 2 * a + sg, pot_log(n2), m);
    }
  }
  // shade with this precision's light and coefficients
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
  const T sh = phong_shade(P, n, d);
  r.depth = (float)thit;
  r.shade = (float)sh;
  r.nx = (float)n[0];
  r.ny = (float)n[1];
  r.nz = (float)n[2];
  r.first_hit = k;
  r.mask = 1;
  r.flags = flags;
  return it;
}

// Add each lane's count v to the counter of its frame f (f < 0: nothing), with one
// atomic per distinct frame in the wave. Every lane of the wave must call it.
template <typename FPtrT>
__device__ __forceinline__ void wave_add_by_frame(int f, unsigned long long v, FPtrT F) {
  uint64_t pending = __builtin_amdgcn_ballot_w64(f >= 0 && v != 0);
  const int lane = lane_id();
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const int lf = __shfl(f, leader, 64);
    const bool mine = f == lf && f >= 0 && v != 0;
    unsigned long long x = mine ? v : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    x = __shfl(x, 0, 64);
    if (lane == leader && F->out.iters) atomicAdd(F->out.iters, x);
    pending &= ~__builtin_amdgcn_ballot_w64(mine);
  }
}

// Write a wave's staged candidates (all lanes call it): reserve n list entries and one
// chunk descriptor, copy the entries, describe the chunk.
__device__ __forceinline__ void flush_stage(const SplitEntry *stage, int n, int frame,
                                            uint32_t *ctr, SplitEntry *hits, SplitChunk *chunks,
                                            int lane) {
  uint32_t base = 0, cidx = 0;
  if (lane == 0) {
    base = atomicAdd(ctr + 1, (uint32_t)n);
    cidx = atomicAdd(ctr + 3, 1u);
  }
  base = uniform((uint32_t)__shfl((int)base, 0, 64));
  cidx = uniform((uint32_t)__shfl((int)cidx, 0, 64));
  if (lane < n) hits[base + lane] = stage[lane];
  if (lane == 0) chunks[cidx] = SplitChunk{(uint32_t)frame, base, (uint32_t)n, 0u};
}

}  // namespace

// ---------------------------------------------------------------------------
// 1. FP16 march
// ---------------------------------------------------------------------------
template <int NORM, bool AXIS, bool BATCH, bool COUNT>
__global__ __launch_bounds__(1024) void march_fp16_kernel(FrameDesc single,
                                                          const FrameDesc *__restrict__ table,
                                                          const LaunchHeader *__restrict__ hdr,
                                                          int nframes, uint32_t total_tiles,
                                                          uint32_t *__restrict__ ctr,
                                                          SplitEntry *__restrict__ hits,
                                                          SplitChunk *__restrict__ chunks, int TW,
                                                          int TH) {
  const int lane = lane_id();
  const int tile_rays = TW * TH;
  // Candidates are staged per wave in LDS and written in chunks of up to 64 entries of
  // one frame, one counter update per chunk (the FP32 pass takes whole chunks).
  extern __shared__ SplitEntry split_stage[];
  SplitEntry *const stage = split_stage + (threadIdx.x >> 6) * 64;
  int scnt = 0;   // entries staged (wave-uniform)
  if constexpr (BATCH) {
    if (hdr) {   // sizes of this launch from device memory (graph replays with new tables)
      nframes = (int)uniform(((ConstHeader)hdr)->nframes);
      total_tiles = uniform(((ConstHeader)hdr)->total_tiles);
    }
  }
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
  h2 c[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) c[q] = hsplat(0.0f);
  h2 c3sq = hsplat(0.0f), cdsq = hsplat(0.0f);
  _Float16 R2 = 0;
  float Sf = 0.0f, Sf2h = 0.0f, ex = 0.0f, ey = 0.0f, ez = 0.0f;
  int N = 1;
  bool n_is_1 = false;
  int TmN = 0;   // T16 - N: a pair that escaped after at least T16 updates came near the set
  // Trip counter and deadlines as in the FP32 marcher (wrap-safe compare; idle lanes
  // hold a NaN state, which the running maximum ignores, and a deadline 2^31 - 1 ahead).
  uint32_t trip = 0;
  const uint32_t kIdleAhead = 0x7FFFFFFFu;
  const h2 kNaN2 = hsplat(__builtin_nanf(""));

  int busy = 0;   // an int, not a bool: a per-lane flag the compiler keeps in a VGPR
  DQH z;
  z.a0 = z.a1 = z.a2 = z.a3 = z.b0 = z.b1 = z.b2 = z.b3 = kNaN2;
  h2 s = kNaN2, m2 = hsplat(0.0f);
  uint32_t dl = kIdleAhead;
  int pix = 0;
  // Sample k of the ray is eye + (t0 + k dt) d, computed as k D + X0 with D = dt d and
  // X0 = eye + t0 d (FP32, then rounded to FP16).
  float X0 = 0, Y0 = 0, Z0 = 0, DX = 0, DY = 0, DZ = 0, kp = 0.0f;   // kp: low sample of the pair
  // First and last sample of pairs that escaped only after T16 or more updates (-1: none):
  // the FP32 pass re-checks that range.
  float kcf = -1.0f, kcl = -1.0f;
  uint32_t cnt_lo = 0, cnt_hi = 0, it_lane = 0;
  int emit = 0;                 // this lane's ray becomes a candidate this trip
  int32_t e_kc = 0, e_kend = 0;

  for (;;) {
    ++trip;
    if (COUNT) {
      cnt_lo += (m2.x <= R2) ? 1u : 0u;
      cnt_hi += (m2.y <= R2) ? 1u : 0u;
    }
    const h2 n2 = pk_update<NORM>(z, s, c);
    m2 = hmax_raw(m2, n2);
    // A pair whose samples are both outside moves on to the next pair (fast path)
    // unless it holds the last sample; a pair that holds the last sample, or one that
    // reached max_iter with an inside sample, ends the march (slow path, run first:
    // it leaves the lanes it ends idle, with m2 = 0, so they fail the fast test).
    // The three per-lane tests (both samples out, the pair holds the last sample --
    // kp is integer-valued, so kp > S - 2 is kp >= S - 1.5 --, the deadline has come) are
    // combined as lane masks in scalar registers; left to itself the compiler turns the
    // combination into per-lane selects.
    const _Float16 mn = min_halves(m2);
    const bool both = mn > R2;
    const uint64_t both_m = __builtin_amdgcn_ballot_w64(both);
    const uint64_t last_m = __builtin_amdgcn_ballot_w64(kp >= Sf2h);
    const uint64_t due_m = __builtin_amdgcn_ballot_w64((int)(trip - dl) >= 0);
    if (__builtin_amdgcn_inverse_ballot_w64((both_m & last_m) | (due_m & ~both_m))) {
      const bool esc_lo = m2.x > R2;
      // a last pair that escaped late still extends the range to re-check
      if (both && (int)(trip - dl) >= TmN) {
        kcf = kcf < 0.0f ? kp : kcf;
        kcl = kp + 1.0f;
      }
      if (both && kcf < 0.0f) {   // every sample escaped within T16 updates: a miss
        if (COUNT) it_lane += cnt_lo + cnt_hi;
        write_pixel(F->out, pix, miss_pixel(DQJ_FLAG_BOX));
      } else {
        // an FP16 inside sample khat (the pair reached max_iter): the FP32 pass scans from
        // the first late-escaping sample, or from khat, to its own first inside sample;
        // a ray without one: the FP32 pass re-checks [kcf, kcl]
        int32_t kc, kend;
        if (both) {
          if (COUNT) it_lane += cnt_lo + cnt_hi;
          kc = (int32_t)kcf;
          kend = (int32_t)kcl;
        } else {
          if (COUNT) it_lane += cnt_lo + (esc_lo ? cnt_hi : 0u);
          const int32_t khat = (int32_t)kp + (esc_lo ? 1 : 0);
          kc = kcf >= 0.0f && (int32_t)kcf < khat ? (int32_t)kcf : khat;
          kend = -1;
        }
        emit = 1;
        e_kc = kc;
        e_kend = kend;
      }
      busy = 0;
      z.a0 = z.a1 = z.a2 = z.a3 = z.b0 = z.b1 = z.b2 = z.b3 = kNaN2;
      s = kNaN2;
      m2 = hsplat(0.0f);
      dl = trip + kIdleAhead;
    }
    // stage this trip's candidates, writing out the staged chunk first if they do not fit
    const uint64_t emit_m = __builtin_amdgcn_ballot_w64(emit != 0);
    if (emit_m) {
      const int ne = __popcll(emit_m);
      if (scnt + ne > 64) {
        flush_stage(stage, scnt, frame, ctr, hits, chunks, lane);
        scnt = 0;
      }
      if (emit) stage[scnt + rank_in(emit_m)] = SplitEntry{(uint32_t)frame, (uint32_t)pix, e_kc, e_kend};
      scnt += ne;
      emit = 0;
    }
    // (the pair's test from before the slow path: the lanes it ended fail it too)
    if (__builtin_amdgcn_inverse_ballot_w64(both_m & ~last_m)) {
      if (COUNT) it_lane += cnt_lo + cnt_hi;
      if ((int)(trip - dl) >= TmN) {   // the pair took T16 or more updates to escape
        kcf = kcf < 0.0f ? kp : kcf;
        kcl = kp + 1.0f;
      }
      kp += 2.0f;
      // The high half of the last pair lies past sample S when S is even. Without
      // counting it is pointed at sample S again (a duplicate cannot change the pair's
      // first inside sample); counting launches mark it escaped instead, so it adds
      // no updates.
      const float k1 = COUNT ? kp + 1.0f : fmin_raw(kp + 1.0f, Sf);
      if constexpr (AXIS) {
        const h2 xh = hpack(fmaf(kp, DX, X0), fmaf(k1, DX, X0));
        const h2 yh = hpack(fmaf(kp, DY, Y0), fmaf(k1, DY, Y0));
        const h2 wh = hpack(fmaf(kp, DZ, Z0), fmaf(k1, DZ, Z0));
        // zeta_1 of (x, y, w, 0 | 0) in closed form; m2 starts at ||zeta_1||^2
        const h2 tx = xh + xh;
        const h2 a0 = hfma(-wh, wh, hfma(-yh, yh, hfma(xh, xh, c[0])));
        z.a1 = hfma(tx, yh, c[1]);
        z.a2 = hfma(tx, wh, c[2]);
        z.a3 = c[3];
        z.b0 = c[4];
        z.b1 = c[5];
        z.b2 = c[6];
        z.b3 = c[7];
        s = hfma(z.a2, z.a2, hfma(z.a1, z.a1, c3sq));
        m2 = hfma(a0, a0, s + cdsq);
        // with max_iter 1 the pair is done: a NaN state leaves m2 as it is
        z.a0 = n_is_1 ? kNaN2 : a0;
        dl = trip + (uint32_t)(N - 1);
        if (COUNT) cnt_lo = cnt_hi = 1;
      } else {
        const KParams &P = F->P;
        const float xl = fmaf(kp, DX, X0), xhh = fmaf(k1, DX, X0);
        const float yl = fmaf(kp, DY, Y0), yhh = fmaf(k1, DY, Y0);
        const float wl = fmaf(kp, DZ, Z0), whh = fmaf(k1, DZ, Z0);
        const DQ<float> zl = slice_map<float>(P, xl, yl, wl);
        const DQ<float> zh = slice_map<float>(P, xhh, yhh, whh);
#define DQJ_PK(F_) hpack(zl.F_, zh.F_)
        z.a0 = DQJ_PK(a0);
        z.a1 = DQJ_PK(a1);
        z.a2 = DQJ_PK(a2);
        z.a3 = DQJ_PK(a3);
        z.b0 = DQJ_PK(b0);
        z.b1 = DQJ_PK(b1);
        z.b2 = DQJ_PK(b2);
        z.b3 = DQJ_PK(b3);
#undef DQJ_PK
        s = hfma(z.a3, z.a3, hfma(z.a2, z.a2, z.a1 * z.a1));
        m2 = hsplat(0.0f);
        dl = trip + (uint32_t)N;
        if (COUNT) cnt_lo = cnt_hi = 0;
      }
      if (COUNT && k1 > Sf) {
        m2.y = (_Float16)INFINITY;
        cnt_hi = 0;
      }
    }

    // ---- hand new rays to idle lanes (one exit, as in the FP32 marcher)
    uint64_t idle = __builtin_amdgcn_ballot_w64(busy == 0);
    while (idle) {
      if (!have_tile) {
        if (exhausted) break;
        if (!pending) {
          uint32_t t = 0;
          if (lane == 0) t = atomicAdd(ctr, 1u);
          t = uniform(t);
          if (t >= total_tiles) {
            exhausted = true;
            break;
          }
          pend_tile = t;
          pending = true;
        }
        const int f = BATCH ? find_frame(ctable, nframes, pend_tile) : 0;
        if (f != frame) {
          if (idle != ~0ull) break;
          if (COUNT && frame >= 0 && F->out.iters) wave_add_u64(F->out.iters, it_lane);
          if (scnt > 0) {
            flush_stage(stage, scnt, frame, ctr, hits, chunks, lane);
            scnt = 0;
          }
          it_lane = 0;
          frame = f;
          if constexpr (BATCH) F = ctable + (int)uniform((uint32_t)f);
          float cf[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            cf[q] = uniform_f(F->P.c[q]);
            c[q] = hsplat(cf[q]);
          }
          R2 = (_Float16)uniform_f(F->P.R2);
          N = (int)uniform((uint32_t)F->P.N);
          TmN = (int)uniform((uint32_t)(F->P.T16 - F->P.N));
          ex = uniform_f(F->P.eye[0]);
          ey = uniform_f(F->P.eye[1]);
          ez = uniform_f(F->P.eye[2]);
          Sf = uniform_f((float)F->P.S);
          Sf2h = Sf - 1.5f;
          c3sq = hsplat(cf[3] * cf[3]);
          cdsq = hsplat(NORM == 0 ? cf[4] * cf[4] + cf[5] * cf[5] + cf[6] * cf[6] + cf[7] * cf[7] : 0.0f);
          n_is_1 = N == 1;
        }
        tile_local = pend_tile - F->tile_begin + F->tile_offset;
        pending = false;
        have_tile = true;
        next_r = 0;
      }
      const int rank = rank_in(idle);
      const int avail = tile_rays - next_r;
      if (busy == 0 && rank < avail) {
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
            const float dt = (tb - ta) / (float)P.S;
            X0 = fmaf(ta, d[0], ex);
            Y0 = fmaf(ta, d[1], ey);
            Z0 = fmaf(ta, d[2], ez);
            DX = dt * d[0];
            DY = dt * d[1];
            DZ = dt * d[2];
            // enter as if the pair (-2, -1) had just escaped: the next trip starts pair 0
            kp = -2.0f;
            busy = 1;
            m2 = hsplat(INFINITY);
            z.a0 = z.a1 = z.a2 = z.a3 = z.b0 = z.b1 = z.b2 = z.b3 = hsplat(0.0f);
            s = hsplat(0.0f);
            dl = trip + (uint32_t)N;
            kcf = -1.0f;
            kcl = -1.0f;
            if (COUNT) cnt_lo = cnt_hi = 0;
          } else {
            write_pixel(F->out, pix, miss_pixel(0));
          }
        }
      }
      const int cntw = __popcll(idle);
      next_r += cntw < avail ? cntw : avail;
      if (next_r >= tile_rays) have_tile = false;
      idle = __builtin_amdgcn_ballot_w64(busy == 0);
    }
    if (exhausted && !__builtin_amdgcn_ballot_w64(busy != 0)) break;
  }
  if (scnt > 0) flush_stage(stage, scnt, frame, ctr, hits, chunks, lane);
  if (COUNT && frame >= 0 && F->out.iters) wave_add_u64(F->out.iters, it_lane);
}

// ---------------------------------------------------------------------------
// 2. FP32 pass over the candidate list
// ---------------------------------------------------------------------------
// Persistent waves take the FP16 march's chunks (runs of up to 64 entries of one frame)
// and hand their entries to idle lanes, as the FP32 marcher hands out tiles: the frame's
// constants stay wave-uniform, and a wave starts another frame's chunk only once its
// lanes are idle. Each lane walks its ray one update per trip:
//   SCAN   : FP32 samples k = ks, ks + 1, ... with ks = max(khat - w, 0), up to the first
//            inside one, k32 (to the last sample when the FP16 march found an inside
//            sample, else to kend + w: past that range every sample escaped within T16
//            FP16 updates; past it the ray misses). If sample ks > 0 is already inside,
//            the crossing lies before the scan: FP64 list.
//   CHECK  : samples k32 + 1 .. k32 + w (those up to S); an outside one means the FP32
//            in/out test flips within the window: FP64 list.
//   BISECT : B bisection points of [t(k32 - 1), t(k32)] (none when k32 = 0);
//   NORMAL : the 6 central-difference points, then shade and write the pixel.
// The update is the FP32 marcher's (q form; a scan sample's first update in closed form
// on the identity slice).
enum { VP_IDLE = 0, VP_SCAN = 1, VP_CHECK = 2, VP_BISECT = 3, VP_NORMAL = 4 };

template <int NORM, bool AXIS, bool BATCH, bool COUNT>
__global__ __launch_bounds__(256) void verify_fp32_kernel(FrameDesc single,
                                                          const FrameDesc *__restrict__ table,
                                                          uint32_t *__restrict__ ctr,
                                                          const SplitEntry *__restrict__ hits,
                                                          SplitEntry *__restrict__ amb,
                                                          const SplitChunk *__restrict__ chunks) {
  const int lane = lane_id();
  const ConstFrame ctable = (ConstFrame)table;
  const uint32_t nchunks = uniform(ctr[3]);
  const float kNaN = __builtin_nanf("");
  const float kNoMarch = 1e30f;
  const uint32_t kIdleAhead = 0x7FFFFFFFu;

  // ---- wave-uniform state: the frame and the chunk being handed out
  typename FramePtr<BATCH>::type F;
  if constexpr (BATCH)
    F = nullptr;
  else
    F = &single;
  int frame = -1;
  bool pending = false, exhausted = false;
  uint32_t pend_c = 0, ccount = 0;
  int next_r = 0;
  // per-lane copies of the frame's constants (see the FP32 marcher)
  float h[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] = 0.0f;
  float R2c = 0.0f, c0c3 = 0.0f, cdsq = 0.0f, ex = 0.0f, ey = 0.0f, ez = 0.0f;
  int N = 1, S = 0, B = 0, w = 1;
  // the chunk's entries: lane i holds entry i
  int e_pix = 0, e_kc = 0, e_kend = 0;

  // ---- per-lane ray state; idle lanes sit on a NaN state with a far deadline
  int phase = VP_IDLE;
  DQ<float> z{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
  float q = kNaN;
  uint32_t trip = 0, dl = kIdleAhead;
  int pix = 0, ks = 0, k32 = 0, j = 0, b = 0, sidx = 0;
  float dx = 0, dy = 0, dz = 0, t0 = 0, dt = 0, k = kNoMarch, klh = 0.0f;
  float lo = 0, hi = 0, thit = 0, gx = 0, gy = 0, gz = 0;
  uint32_t it = 0;

  enter_update_mode();
  for (;;) {
    ++trip;
    const float n2 = dq_update_q<NORM>(z, q, h);
    const bool esc = n2 > R2c;
    const bool fast = esc && phase == VP_SCAN && k < klh;   // k integer-valued: more scan samples
    const bool slow = (esc || (int)(trip - dl) >= 0) && !fast;
    if (slow) {
      const KParams &P = F->P;
      const bool inside = !esc;
      const int m = N - (int)(dl - trip);   // escape index, or N when inside
      if (COUNT) it += (uint32_t)m;
      bool start_hit = false, to_amb = false;
      int amb_k = 0;
      if (phase == VP_SCAN) {
        if (!inside) {   // the scan's last sample escaped: the ray misses
          write_pixel(F->out, pix, miss_pixel(DQJ_FLAG_BOX));
          phase = VP_IDLE;
        } else if ((int)k == ks && ks > 0) {
          to_amb = true;
          amb_k = ks;
        } else {
          k32 = (int)k;
          j = 1;
          phase = VP_CHECK;
        }
        k = kNoMarch;
      } else if (phase == VP_CHECK) {
        if (!inside) {
          to_amb = true;
          amb_k = k32;
        } else {
          ++j;
        }
      } else if (phase == VP_BISECT) {
        const float tm = 0.5f * (lo + hi);
        if (inside)
          hi = tm;
        else
          lo = tm;
        ++b;
      } else {   // VP_NORMAL: stencil point sidx just retired (b: least escape index)
        stencil_add(gx, gy, gz, b, sidx, pot_log(n2 + h[0]), m);
        ++sidx;
      }
      // the window after k32 is confirmed: bracket the crossing
      if (phase == VP_CHECK && !to_amb && (j > w || k32 + j > S)) start_hit = true;
      if (start_hit) {
        b = 0;
        if (k32 == 0) {
          thit = t0;
          phase = VP_NORMAL;
        } else {
          lo = fmaf((float)(k32 - 1), dt, t0);
          hi = fmaf((float)k32, dt, t0);
          phase = VP_BISECT;
        }
      }
      if (phase == VP_BISECT && b >= B) {
        thit = 0.5f * (lo + hi);
        phase = VP_NORMAL;
      }
      if (to_amb) {
        const uint32_t slot = atomicAdd(ctr + 2, 1u);
        amb[slot] = SplitEntry{(uint32_t)frame, (uint32_t)pix, (int32_t)amb_k, -1};
        phase = VP_IDLE;
      }
      if (phase == VP_NORMAL && sidx == 6) {
        const float g[3] = {gx, gy, gz};
        const float d[3] = {dx, dy, dz};
        PixelOut r;
        finish_hit(P, g, d, thit, k32, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
        write_pixel(F->out, pix, r);
        phase = VP_IDLE;
      }
      float px = 0, py = 0, pz = 0;
      if (phase == VP_CHECK || phase == VP_BISECT) {
        const float tr = phase == VP_CHECK ? fmaf((float)(k32 + j), dt, t0) : 0.5f * (lo + hi);
        px = fmaf(tr, dx, ex);
        py = fmaf(tr, dy, ey);
        pz = fmaf(tr, dz, ez);
      } else if (phase == VP_NORMAL) {
        const int axis = sidx >> 1;
        const float hs = (sidx & 1) ? -P.h : P.h;
        px = fmaf(thit, dx, ex) + (axis == 0 ? hs : 0.0f);
        py = fmaf(thit, dy, ey) + (axis == 1 ? hs : 0.0f);
        pz = fmaf(thit, dz, ez) + (axis == 2 ? hs : 0.0f);
      }
      if (phase != VP_IDLE) {
        if (AXIS)
          z = DQ<float>{px, py, pz, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        else
          z = slice_map<float>(P, px, py, pz);
        q = q_of(z, h[0]);
        dl = trip + (uint32_t)N;
      } else {
        z = DQ<float>{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
        q = kNaN;
        dl = trip + kIdleAhead;
      }
    }
    if (fast) {   // the next scan sample
      if (COUNT) it += (uint32_t)N - (dl - trip);
      k += 1.0f;
      const float t = fmaf(k, dt, t0);
      const float x = fmaf(t, dx, ex);
      const float y = fmaf(t, dy, ey);
      const float wz = fmaf(t, dz, ez);
      if constexpr (AXIS) {
        float a0;
        start_axis_q(x, y, wz, h, c0c3, a0, z, q);
        // zeta_1 is tested: an escaped sample is parked on a state that escapes on the
        // next update; with max_iter 1 an inside one is parked on NaN
        const bool esc1 = fmaf(a0, a0, cdsq - q) > R2c;
        const bool n1 = N == 1;
        z.a0 = esc1 ? 1e18f : (n1 ? kNaN : a0);
        dl = trip + (uint32_t)(N - 1) + ((esc1 || n1) ? 1u : 0u);
      } else {
        z = slice_map<float>(F->P, x, y, wz);
        q = q_of(z, h[0]);
        dl = trip + (uint32_t)N;
      }
    }

    // ---- hand the chunk's entries to idle lanes
    uint64_t idle = __builtin_amdgcn_ballot_w64(phase == VP_IDLE);
    while (idle) {
      if (next_r >= (int)ccount) {   // the chunk is handed out: take the next one
        if (exhausted) break;
        if (!pending) {
          uint32_t c = 0;
          if (lane == 0) c = atomicAdd(ctr + 4, 1u);
          c = uniform((uint32_t)__shfl((int)c, 0, 64));
          if (c >= nchunks) {
            exhausted = true;
            break;
          }
          pend_c = c;
          pending = true;
        }
        const int f = (int)uniform(chunks[pend_c].frame);
        if (f != frame) {
          if (idle != ~0ull) break;   // finish this frame's rays first
          if (COUNT && frame >= 0 && F->out.iters) wave_add_u64(F->out.iters, it);
          it = 0;
          frame = f;
          if constexpr (BATCH) F = ctable + f;
          const KParams &P = F->P;
          float c[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) c[i] = uniform_f(P.c[i]);
          h[0] = to_vgpr(c[0]);
#pragma unroll
          for (int i = 1; i < 8; ++i) h[i] = to_vgpr(uniform_f(0.5f * c[i]));
          R2c = to_vgpr(uniform_f(P.R2 - c[0]));
          c0c3 = to_vgpr(uniform_f(fmaf(-c[3], c[3], c[0])));
          cdsq = NORM == 0 ? uniform_f(fmaf(c[7], c[7], fmaf(c[6], c[6], fmaf(c[5], c[5], c[4] * c[4]))))
                           : 0.0f;
          ex = to_vgpr(uniform_f(P.eye[0]));
          ey = to_vgpr(uniform_f(P.eye[1]));
          ez = to_vgpr(uniform_f(P.eye[2]));
          N = (int)uniform((uint32_t)P.N);
          S = (int)uniform((uint32_t)P.S);
          B = (int)uniform((uint32_t)P.B);
          w = (int)uniform((uint32_t)P.fp64_window);
        }
        const uint32_t cbase = uniform(chunks[pend_c].base);
        ccount = uniform(chunks[pend_c].count);
        pending = false;
        next_r = 0;
        if (lane < (int)ccount) {
          const SplitEntry en = hits[cbase + lane];
          e_pix = (int)en.pix;
          e_kc = en.khat;
          e_kend = en.kend;
        }
      }
      const int rank = rank_in(idle);
      const int src = next_r + rank;
      const int s_pix = __shfl(e_pix, src & 63, 64), s_kc = __shfl(e_kc, src & 63, 64),
                s_kend = __shfl(e_kend, src & 63, 64);
      if (phase == VP_IDLE && src < (int)ccount) {
        const KParams &P = F->P;
        pix = s_pix;
        const int ii = pix % P.W, jj = pix / P.W;
        float d[3], ta, tb;
        pixel_dir(P, ii, jj, d);
        clip_box(P, d, ta, tb);   // the FP16 march found this ray's segment with the same code
        dx = d[0];
        dy = d[1];
        dz = d[2];
        t0 = ta;
        dt = (tb - ta) / (float)S;
        ks = s_kc - w > 0 ? s_kc - w : 0;
        const int klast = s_kend < 0 ? S : (s_kend + w < S ? s_kend + w : S);
        klh = (float)klast - 0.5f;
        // enter as if sample ks - 1 had just escaped: the fast path starts sample ks
        k = (float)(ks - 1);
        phase = VP_SCAN;
        sidx = P.normal_mode != 0 ? 6 : 0;
        gx = gy = gz = 0.0f;
        z = DQ<float>{1e18f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        q = 0.0f;
        dl = trip + (uint32_t)N;
        if (COUNT) it -= 1u;
      }
      const int cnt = __popcll(idle), avail = (int)ccount - next_r;
      next_r += cnt < avail ? cnt : avail;
      idle = __builtin_amdgcn_ballot_w64(phase == VP_IDLE);
    }
    if (exhausted && !__builtin_amdgcn_ballot_w64(phase != VP_IDLE)) break;
  }
  if (COUNT && frame >= 0 && F->out.iters) wave_add_u64(F->out.iters, it);
}

// ---------------------------------------------------------------------------
// 3. FP64 march and re-bisection over the rays the FP32 pass hands on
// ---------------------------------------------------------------------------
template <int NORM, bool BATCH, bool COUNT>
__global__ __launch_bounds__(256) void rebisect_fp64_kernel(FrameDesc single,
                                                            const FrameDesc *__restrict__ table,
                                                            const uint32_t *__restrict__ amb_ctr,
                                                            const SplitEntry *__restrict__ amb) {
  const ConstFrame ctable = (ConstFrame)table;
  const uint32_t n = *amb_ctr;
  const uint32_t wave0 = blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = wave0; base < n; base += stride) {
    const uint32_t e = base + (threadIdx.x & 63u);
    uint32_t it = 0;
    int fr = -1;
    typename FramePtr<BATCH>::type F;
    if constexpr (BATCH)
      F = ctable;
    else
      F = &single;
    if (e < n) {
      const SplitEntry en = amb[e];
      if constexpr (BATCH) F = ctable + en.frame;
      fr = (int)en.frame;
      const KParams64 &Q = F->P64;
      const int W = F->P.W, S = F->P.S, N = F->P.N, B = F->P.B;
      const int i = (int)(en.pix % (uint32_t)W), j = (int)(en.pix / (uint32_t)W);
      double d[3], t0, t1;
      pixel_dir64(Q, i, j, d);
      PixelOut r;
      if (!clip_box64(Q, d, t0, t1)) {
        r = miss_pixel(DQJ_FLAG_FP64);
      } else {
        const double dt = (t1 - t0) / (double)S;
        const int w = F->P.fp64_window;
        int klo = en.khat - w > 0 ? en.khat - w : 0;
        int kstar = -1;
        for (int k = klo; k <= S; ++k) {
          bool in;
          double n2;
          it += classify_t<NORM>(Q, Q.c, N, Q.R2, fma((double)k, dt, t0), d, 0.0, 0.0, 0.0, &in, &n2);
          if (in) {
            kstar = k;
            break;
          }
        }
        // The window starts inside: the FP16 march crossed late. Walk back to the start
        // of this inside run (samples before an outside one are not re-checked).
        while (kstar == klo && kstar > 0) {
          bool in;
          double n2;
          it += classify_t<NORM>(Q, Q.c, N, Q.R2, fma((double)(kstar - 1), dt, t0), d, 0.0, 0.0,
                                 0.0, &in, &n2);
          if (!in) break;
          --kstar;
          --klo;
        }
        if (kstar < 0) {
          r = miss_pixel(DQJ_FLAG_BOX | DQJ_FLAG_FP64);
        } else {
          it += finish_ray<NORM>(Q, Q.c, N, B, Q.R2, Q.h, d, t0, dt, kstar,
                                 (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT | DQJ_FLAG_FP64), r);
        }
      }
      write_pixel(F->out, en.pix, r);
    }
    if (COUNT) wave_add_by_frame(fr, it, F);
  }
}

__global__ void reset_split_counters_kernel(uint32_t *ctr) {
  if (threadIdx.x < 8) ctr[threadIdx.x] = 0u;
}

template <bool BATCH, bool COUNT>
static void launch_split_variant(const FrameDesc &single, const FrameDesc *table,
                                 const LaunchHeader *hdr, int nframes,
                                 uint32_t total_tiles, int norm, bool axis, const SplitScratch &sc,
                                 const Sched &s, int cus, hipStream_t stream) {
  const int threads = 64 * s.waves_per_block;
  const int blocks = cus * s.blocks_per_cu;
  const size_t stage_lds = sizeof(SplitEntry) * 64 * (size_t)s.waves_per_block;
#define DQJ_MARCH(NM, AX)                                                                     \
  hipLaunchKernelGGL((march_fp16_kernel<NM, AX, BATCH, COUNT>), dim3(blocks), dim3(threads),  \
                     stage_lds, stream, single, table, hdr, nframes, total_tiles, sc.ctr, sc.hits, \
                     sc.chunks, s.tile_w, s.tile_h)
  if (norm == 0) {
    if (axis)
      DQJ_MARCH(0, true);
    else
      DQJ_MARCH(0, false);
  } else {
    if (axis)
      DQJ_MARCH(1, true);
    else
      DQJ_MARCH(1, false);
  }
#undef DQJ_MARCH
  const int vblocks = cus * 8;
#define DQJ_VERIFY(NM, AX)                                                                      \
  hipLaunchKernelGGL((verify_fp32_kernel<NM, AX, BATCH, COUNT>), dim3(vblocks), dim3(256), 0,    \
                     stream, single, table, sc.ctr, sc.hits, sc.amb, sc.chunks);                  \
  hipLaunchKernelGGL((rebisect_fp64_kernel<NM, BATCH, COUNT>), dim3(cus * 2), dim3(256), 0, stream, \
                     single, table, sc.ctr + 2, sc.amb)
  if (norm == 0) {
    if (axis) {
      DQJ_VERIFY(0, true);
    } else {
      DQJ_VERIFY(0, false);
    }
  } else {
    if (axis) {
      DQJ_VERIFY(1, true);
    } else {
      DQJ_VERIFY(1, false);
    }
  }
#undef DQJ_VERIFY
}

template <bool BATCH>
static hipError_t launch_split_impl(const FrameDesc &single, const FrameDesc *table,
                                    const LaunchHeader *hdr, int nframes,
                                    uint32_t total_tiles, int norm, bool axis, bool count,
                                    const SplitScratch &sc, const Sched &s, int cus,
                                    hipStream_t stream) {
  hipLaunchKernelGGL(reset_split_counters_kernel, dim3(1), dim3(64), 0, stream, sc.ctr);
  if (count)
    launch_split_variant<BATCH, true>(single, table, hdr, nframes, total_tiles, norm, axis, sc, s,
                                      cus, stream);
  else
    launch_split_variant<BATCH, false>(single, table, hdr, nframes, total_tiles, norm, axis, sc, s,
                                       cus, stream);
  return hipGetLastError();
}

hipError_t launch_render_split(const FrameDesc &frame, const SplitScratch &sc, const Sched &s,
                               int cus, hipStream_t stream) {
  return launch_split_impl<false>(frame, nullptr, nullptr, 1, frame.ntiles, frame.P.norm,
                                  frame.P.axis_slice != 0, frame.out.iters != nullptr, sc, s, cus,
                                  stream);
}

hipError_t launch_render_split_batch(const FrameDesc *table_dev, const LaunchHeader *hdr_dev,
                                     int nframes, uint32_t total_tiles, int norm, bool all_axis,
                                     bool any_count, const SplitScratch &sc, const Sched &s, int cus,
                                     hipStream_t stream) {
  FrameDesc dummy;
  memset(&dummy, 0, sizeof dummy);
  return launch_split_impl<true>(dummy, table_dev, hdr_dev, nframes, total_tiles, norm, all_axis,
                                 any_count, sc, s, cus, stream);
}

}  // namespace dqj

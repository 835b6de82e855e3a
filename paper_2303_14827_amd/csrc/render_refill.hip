// render_refill.hip -- persistent FP32 ray marcher with per-lane work refill.
//
// Each lane owns one ray and walks the method as a small state machine:
//   MARCH  : classify sample k of the fixed-step march (section "Ray-Marching");
//            outside -> sample k+1, inside -> BISECT (or NORMAL when k = 0 or B = 0);
//   BISECT : classify the bracket midpoint B times;
//   NORMAL : classify the 6 central-difference points and accumulate the gradient
//            of the escape potential (section "Lighting/Illumination"), then shade
//            (Eq. phong, ambient + diffuse) and write the pixel.
// Every trip of the main loop applies ONE update z <- z^2 + c (Eq. dqjulia2) to
// every busy lane; a lane whose point retires (escaped, or max_iter reached) takes
// its next point at once, and a lane whose ray is finished takes the next ray of
// its wave's tile. So no lane waits for the slowest ray of its wave: the cost of
// divergence is the transition code, not idle lanes.
//
// Waves are persistent and take tiles (tile_w x tile_h pixels) from one global
// atomic counter over all frames of the launch. A wave finishes every ray of a
// frame before it starts a tile of another frame, so the Julia constant and the
// camera stay wave-uniform (scalar registers). Results do not depend on which
// lane or wave computes a pixel: images are bit-identical under any schedule.
// Once the queue has ended, launches without the update counter finish their rays in
// a second loop that runs the same trip without the hand-out. The launch's last frame
// is handed out centre-out (tile_order.h), so its long rays start early.
#include "dq_device.h"
#include "launch.h"
#include "persist.h"
#include "qform.h"
#include "refill.h"
#include "tile_order.h"

#include <cstring>

namespace dqj {

using namespace persist;

namespace {

enum { PH_IDLE = 0, PH_MARCH = 1, PH_BISECT = 2, PH_NORMAL = 3 };


// zeta_0 for a world point and its q.
template <bool AXIS>
__device__ __forceinline__ void start_point(const KParams &P, float x, float y, float zc,
                                            float c0, DQ<float> &z, float &q) {
  if (AXIS)
    z = DQ<float>{x, y, zc, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  else
    z = slice_map<float>(P, x, y, zc);
  q = q_of(z, c0);
}

}  // namespace

// Template switches: NORM (escape norm), AXIS (every frame uses the identity slice,
// so march samples take their first update in closed form), BATCH (frames come from a
// device table), COUNT (accumulate executed updates per frame), STICKY (every frame
// guarantees that a march sample escaping on its first update escapes on the second,
// so that update is not tested; only used with AXIS and without COUNT), HAND (how tiles
// are handed out: one per atomic, guided chunks, or a first tile per wave without the
// counter; see the hand-out).
enum { kHandOne = 0, kHandGuided = 1, kHandFirst = 2 };
template <int NORM, bool AXIS, bool BATCH, bool COUNT, bool STICKY, int HAND, bool WIDE>
__device__ __forceinline__ void refill_body(const FrameDesc &single,
                                            const FrameDesc *__restrict__ table,
                                            const LaunchHeader *__restrict__ hdr, int nframes,
                                            uint32_t total_tiles, uint32_t *__restrict__ counter,
                                            int TW, int TH) {
  static_assert(!STICKY || (AXIS && !COUNT), "STICKY needs AXIS and no counting");
  const int lane = lane_id();
  const int tile_rays = TW * TH;
  if constexpr (BATCH) {
    if (hdr) {   // sizes of this launch from device memory (graph replays with new tables)
      nframes = (int)uniform(((ConstHeader)hdr)->nframes);
      total_tiles = uniform(((ConstHeader)hdr)->total_tiles);
    }
  }
  const float kNaN = __builtin_nanf("");
  const float kNoMarch = 1e30f;   // k outside the march: the fast-path test k < S fails

  // ---- wave-uniform state
  const ConstFrame ctable = (ConstFrame)table;
  // F is null in batch launches until the wave takes its first tile: no read through F
  // (the frame's constants, its outputs) may happen before a tile is assigned. Every
  // such read sits in the slow path or the hand-out below, which only lanes with a ray
  // reach; a read hoisted to the top of the trip dereferences a null pointer.
  typename FramePtr<BATCH>::type F;
  if constexpr (BATCH)
    F = nullptr;
  else
    F = &single;
  int frame = -1;
  uint32_t tile_local = 0;      // tile index within the frame
  int next_r = 0;               // next ray of the tile to hand out
  bool have_tile = false, pending = false, exhausted = false;
  uint32_t spare = 0, spare_n = 0, last_t = 0;   // kHandGuided: the rest of the wave's chunk
  // kHandFirst: the wave's first tile (wave w takes tile w), taken without the counter
  const uint32_t kNoTile = 0xFFFFFFFFu;
  uint32_t first_tile = uniform(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  uint32_t pend_tile = 0;
  float R2c = 0.0f, c0c3 = 0.0f, cdsq = 0.0f, Sfh = 0.0f;
  float ex = 0.0f, ey = 0.0f, ez = 0.0f;   // eye (cached: the table is not provably read-only)
  // Per-lane copies of c0 and of c_i / 2 (i >= 1): the update and the closed-form
  // start compute with vector registers only (scalar-register operands cost more issue
  // time on gfx950). R^2 - c0, the eye, S - 1/2 and c0 - c3^2 below are per-lane
  // copies for the same reason.
  float h[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] = 0.0f;
  int N = 1;
  bool n_is_1 = false;
  // Trip counter: one update per trip. A point started in trip t has had trip - t
  // updates after trip `trip`, so "max_iter reached" is trip - deadline >= 0 (mod 2^32),
  // with the deadline set when the point starts; no per-lane counter is incremented.
  // A ray takes at most (S + B + 8) N <= 2^30 trips, so live deadlines lie less than
  // 2^30 ahead and an idle lane's deadline (2^31 - 1 ahead) is never reached before
  // the lane gets a new ray or the wave ends.
  uint32_t trip = 0;
  const uint32_t kIdleAhead = 0x7FFFFFFFu;

  // ---- per-lane state. Idle lanes sit on a NaN state (never escapes) with a far
  // deadline, so they never retire and need no separate test.
  int phase = PH_IDLE;
  DQ<float> z{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
  float q = kNaN;
  uint32_t dl = kIdleAhead;
  int pix = 0;
  float dx = 0, dy = 0, dz = 0, t0 = 0, dt = 0;
  float k = kNoMarch;     // march sample index (exact in FP32 up to 2^24)
  int b = 0, sidx = 0, kstar = -1;
  float lo = 0, hi = 0, thit = 0, gx = 0, gy = 0, gz = 0;
  uint32_t it_lane = 0;

  enter_update_mode();
  for (;;) {
    ++trip;
    // ---- one update on every lane (n2 is ||zeta||^2 - c0)
    const float n2 = dq_update_q<NORM>(z, q, h);
    // Three per-lane tests, combined as lane masks: the sample escaped, it is past the
    // last march sample (k >= S; k is integer-valued, so k > S - 1/2), its deadline
    // has come. Fast path: an outside march sample with more samples to go starts the
    // next one. Everything else that retires (a march hit or miss, a bisection or
    // normal point) takes the slow path, which runs first; the fast set is fixed
    // before it, and the two sets are disjoint.
    // (The masks are formed explicitly: left to itself the compiler turns the
    // combination into per-lane selects.)
    const uint64_t esc = __builtin_amdgcn_ballot_w64(n2 > R2c);
    const uint64_t last = __builtin_amdgcn_ballot_w64(k > Sfh);
    const uint64_t due = __builtin_amdgcn_ballot_w64((int)(trip - dl) >= 0);
    const uint64_t fast = esc & ~last;

    uint64_t slow = (esc & last) | (due & ~esc);
    if constexpr (HAND == kHandGuided) {
      // Launches of many frames (the guided hand-out): when every retiring lane is a
      // march whose last sample escaped, the misses are written here and the slow
      // path's phase tests are skipped. 4096 frames of 256^2: 135.4-135.5 ms against
      // 136.5-136.8, the same images. In the one-tile kernel the same test made 256
      // frames 5% faster but three 1024^2 frames 0.6-1.2% slower (their tails
      // mix misses with bisection and normal points), so that kernel goes without.
      if (slow != 0 && slow == (esc & last & __builtin_amdgcn_ballot_w64(phase == PH_MARCH))) {
        if (__builtin_amdgcn_inverse_ballot_w64(slow)) {
          if (COUNT) it_lane += (uint32_t)N - (dl - trip);
          write_pixel(F->out, pix, miss_pixel(DQJ_FLAG_BOX));
          phase = PH_IDLE;
          z = DQ<float>{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
          q = kNaN;
          dl = trip + kIdleAhead;
        }
        slow = 0;
      }
    }
    if (__builtin_amdgcn_inverse_ballot_w64(slow)) {
      const KParams &P = F->P;
      // (recomputed from an opaque copy: a shared compare would run on every trip)
      float n2c = n2;
      asm volatile("" : "+v"(n2c));
      const bool inside = !(n2c > R2c);
      const int m = N - (int)(dl - trip);   // escape index, or N when inside
      if (COUNT) it_lane += (uint32_t)m;
      bool next_normal = false;
      bool restart = false;   // start the point at parameter tr on the ray
      float tr = 0.0f;
      if (phase == PH_MARCH) {
        if (inside) {
          kstar = (int)k;
          k = kNoMarch;
          if (kstar == 0) {
            thit = t0;
            next_normal = true;
          } else {
            lo = fmaf((float)(kstar - 1), dt, t0);
            hi = fmaf((float)kstar, dt, t0);
            if (P.B == 0) {
              thit = 0.5f * (lo + hi);
              next_normal = true;
            } else {
              b = 0;
              phase = PH_BISECT;
              tr = 0.5f * (lo + hi);
              restart = true;
            }
          }
        } else {  // the last sample was outside: the ray misses
          write_pixel(F->out, pix, miss_pixel(DQJ_FLAG_BOX));
          phase = PH_IDLE;
        }
      } else if (phase == PH_BISECT) {
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
      } else {  // PH_NORMAL: stencil point sidx just retired
        if constexpr (WIDE) {
          // (b, the bisection counter, holds the stencil's least escape index here)
          stencil_add(gx, gy, gz, b, sidx, pot_log(n2c + h[0]), m);
        } else {   // max_iter <= kUnscaledMaxIter: the potentials as they are
          const float G = potential(n2c + h[0], m);
          const float sg = (sidx & 1) ? -G : G;
          const int axis = sidx >> 1;
          if (axis == 0)
            gx += sg;
          else if (axis == 1)
            gy += sg;
          else
            gz += sg;
        }
        ++sidx;
      }
      if (next_normal) {
        phase = PH_NORMAL;
        // the four-neighbour normal is formed after the frame: no stencil points
        sidx = P.normal_mode != 0 ? 6 : 0;
        gx = gy = gz = 0.0f;
      }
      if (phase == PH_NORMAL && sidx == 6) {   // the hit is finished (g = 0: no stencil)
        const float g[3] = {gx, gy, gz};
        const float d[3] = {dx, dy, dz};
        PixelOut r;
        finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
        write_pixel(F->out, pix, r);
        phase = PH_IDLE;
      }
      float px = 0, py = 0, pz = 0;
      if (restart) {
        px = fmaf(tr, dx, ex);
        py = fmaf(tr, dy, ey);
        pz = fmaf(tr, dz, ez);
      } else if (phase == PH_NORMAL) {
        const int axis = sidx >> 1;
        const float hs = (sidx & 1) ? -P.h : P.h;
        px = fmaf(thit, dx, ex) + (axis == 0 ? hs : 0.0f);
        py = fmaf(thit, dy, ey) + (axis == 1 ? hs : 0.0f);
        pz = fmaf(thit, dz, ez) + (axis == 2 ? hs : 0.0f);
      }
      if (phase != PH_IDLE) {
        start_point<AXIS>(P, px, py, pz, h[0], z, q);
        dl = trip + (uint32_t)N;
      } else {
        z = DQ<float>{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
        q = kNaN;
        dl = trip + kIdleAhead;
      }
    }

    if (__builtin_amdgcn_inverse_ballot_w64(fast)) {
      if (COUNT) it_lane += (uint32_t)N - (dl - trip);
      k += 1.0f;
      const float t = fmaf(k, dt, t0);
      const float x = fmaf(t, dx, ex);
      const float y = fmaf(t, dy, ey);
      const float w = fmaf(t, dz, ez);
      if constexpr (AXIS) {
        // First update in closed form.
        float a0;
        start_axis_q(x, y, w, h, c0c3, a0, z, q);
        if constexpr (STICKY) {
          // zeta_2 escapes whenever zeta_1 does: leave zeta_1 untested (a sample that
          // escaped on it retires after the next update, as a parked one would).
          dl = trip + (uint32_t)(N - 1);
        } else {
          // Test zeta_1. An escaped sample is parked on a state that escapes on the
          // next update (escape index 1); with max_iter 1 an inside one is parked on
          // NaN (never escapes) and retires on its deadline at the next trip.
          const bool esc1 = fmaf(a0, a0, cdsq - q) > R2c;
          a0 = esc1 ? 1e18f : (n_is_1 ? kNaN : a0);
          dl = trip + (uint32_t)(N - 1) + ((esc1 || n_is_1) ? 1u : 0u);
        }
        z.a0 = a0;
      } else {
        start_point<AXIS>(F->P, x, y, w, h[0], z, q);
        dl = trip + (uint32_t)N;
      }
    }

    // ---- hand new rays to idle lanes (one exit: every stop leaves through the
    // loop condition, so the common case costs one ballot and one branch)
    uint64_t idle = __builtin_amdgcn_ballot_w64(phase == PH_IDLE);
    while (idle) {
      if (!have_tile) {
        if (exhausted) break;
        if (!pending) {
          uint32_t t = 0;
          if constexpr (HAND == kHandGuided) {
            // Guided self-scheduling: a chunk of g consecutive tiles per atomic, g = the
            // tiles left (as this wave last saw the counter) / (64 x waves), between 1 and
            // 8. Large launches take whole runs of a frame's tiles early, so a wave changes
            // frames (and waits for its lanes) less often; near the end g falls to 1 and
            // the ramp-down keeps single tiles.
            if (spare_n > 0) {
              t = spare;
              ++spare;
              --spare_n;
            } else {
              const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
              const uint32_t left = total_tiles > last_t ? total_tiles - last_t : 0u;
              uint32_t g = left / (nwaves * 64u);
              g = g < 1u ? 1u : (g > 8u ? 8u : g);
              if (lane == 0) t = atomicAdd(counter, g);
              t = uniform(t);
              last_t = t;
              spare = t + 1u;
              spare_n = g - 1u;
            }
          } else if constexpr (HAND == kHandFirst) {
            // A single frame's launch gives each wave two or three tiles, and at the start
            // all waves would queue on one atomic: the first tiles go one per wave, and the
            // counter hands out tiles from nwaves on (a 1024^2 frame with many hits 7%
            // faster). Batches keep one tile per atomic: there the same change cost 3%.
            t = first_tile;
            if (t == kNoTile) {
              if (lane == 0) t = atomicAdd(counter, 1u);
              t = uniform(t) + gridDim.x * (blockDim.x >> 6);
            }
            first_tile = kNoTile;
          } else {
            if (lane == 0) t = atomicAdd(counter, 1u);
            t = uniform(t);
          }
          if (t >= total_tiles) {
            exhausted = true;
            break;
          }
          pend_tile = t;
          pending = true;
        }
        const int f = BATCH ? find_frame(ctable, nframes, pend_tile) : 0;
        if (f != frame) {
          if (idle != ~0ull) break;  // finish this frame's rays first
          if (COUNT && frame >= 0 && F->out.iters) wave_add_u64(F->out.iters, it_lane);
          it_lane = 0;
          frame = f;
          if constexpr (BATCH) F = ctable + (int)uniform((uint32_t)f);
          float c[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) c[i] = uniform_f(F->P.c[i]);
          h[0] = to_vgpr(c[0]);
#pragma unroll
          for (int i = 1; i < 8; ++i) h[i] = to_vgpr(uniform_f(0.5f * c[i]));
          R2c = to_vgpr(uniform_f(F->P.R2 - c[0]));
          N = (int)uniform((uint32_t)F->P.N);
          n_is_1 = N == 1;
          ex = to_vgpr(uniform_f(F->P.eye[0]));
          ey = to_vgpr(uniform_f(F->P.eye[1]));
          ez = to_vgpr(uniform_f(F->P.eye[2]));
          Sfh = to_vgpr(uniform_f((float)F->P.S - 0.5f));
          c0c3 = to_vgpr(uniform_f(fmaf(-c[3], c[3], c[0])));
          cdsq = NORM == 0 ? uniform_f(fmaf(c[7], c[7], fmaf(c[6], c[6], fmaf(c[5], c[5], c[4] * c[4]))))
                           : 0.0f;
        }
        tile_local = pend_tile - F->tile_begin + F->tile_offset;
        // The launch's last entry goes centre-out when it holds a whole frame (the
        // chunks of a split frame keep the plain order, so together they still cover it).
        if (frame == nframes - 1 && F->tile_offset == 0) {
          const int ty_n = (F->P.H + TH - 1) / TH;
          if (F->ntiles == F->tiles_x * (uint32_t)ty_n)
            tile_local = centre_out_tile(tile_local, (int)F->tiles_x, ty_n);
        }
        pending = false;
        have_tile = true;
        next_r = 0;
      }
      const int rank = rank_in(idle);
      const int avail = tile_rays - next_r;
      if (phase == PH_IDLE && rank < avail) {
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
            dt = (tb - ta) / (float)P.S;
            // Enter the march as if sample -1 had just escaped: the fast path then
            // starts sample 0. Its fictitious update is not counted.
            k = -1.0f;
            kstar = -1;
            phase = PH_MARCH;
            z = DQ<float>{1e18f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
            q = 0.0f;
            dl = trip + (uint32_t)N;
            if (COUNT) it_lane -= 1u;
          } else {
            write_pixel(F->out, pix, miss_pixel(0));
          }
        }
      }
      const int cnt = __popcll(idle);
      next_r += cnt < avail ? cnt : avail;
      if (next_r >= tile_rays) have_tile = false;
      idle = __builtin_amdgcn_ballot_w64(phase == PH_IDLE);
    }

    if (exhausted && !__builtin_amdgcn_ballot_w64(phase != PH_IDLE)) break;
    if (!COUNT && exhausted) break;   // the rest runs in the tail loop below
  }
  if constexpr (!COUNT) {
    // ---- after the tile queue has ended (launches without the update counter): the
    // same trip without the tile hand-out, until every lane is idle. Leaving the
    // hand-out behind shortens each trip of the launch's tail, where few lanes are
    // still busy: plain_1024 6% and a single 1024^2 frame with many hits 12% faster.
    // The trip is written out again rather than shared through a lambda, whose code
    // was many times slower on gfx950.
    for (;;) {
    ++trip;
    // ---- one update on every lane (n2 is ||zeta||^2 - c0)
    const float n2 = dq_update_q<NORM>(z, q, h);
    // Three per-lane tests, combined as lane masks: the sample escaped, it is past the
    // last march sample (k >= S; k is integer-valued, so k > S - 1/2), its deadline
    // has come. Fast path: an outside march sample with more samples to go starts the
    // next one. Everything else that retires (a march hit or miss, a bisection or
    // normal point) takes the slow path, which runs first; the fast set is fixed
    // before it, and the two sets are disjoint.
    // (The masks are formed explicitly: left to itself the compiler turns the
    // combination into per-lane selects.)
    const uint64_t esc = __builtin_amdgcn_ballot_w64(n2 > R2c);
    const uint64_t last = __builtin_amdgcn_ballot_w64(k > Sfh);
    const uint64_t due = __builtin_amdgcn_ballot_w64((int)(trip - dl) >= 0);
    const uint64_t fast = esc & ~last;

    uint64_t slow = (esc & last) | (due & ~esc);
    if constexpr (HAND == kHandGuided) {   // misses only: as in the loop above
      if (slow != 0 && slow == (esc & last & __builtin_amdgcn_ballot_w64(phase == PH_MARCH))) {
        if (__builtin_amdgcn_inverse_ballot_w64(slow)) {
          write_pixel(F->out, pix, miss_pixel(DQJ_FLAG_BOX));
          phase = PH_IDLE;
          z = DQ<float>{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
          q = kNaN;
          dl = trip + kIdleAhead;
        }
        slow = 0;
      }
    }
    if (__builtin_amdgcn_inverse_ballot_w64(slow)) {
      const KParams &P = F->P;
      // (recomputed from an opaque copy: a shared compare would run on every trip)
      float n2c = n2;
      asm volatile("" : "+v"(n2c));
      const bool inside = !(n2c > R2c);
      const int m = N - (int)(dl - trip);   // escape index, or N when inside
      bool next_normal = false;
      bool restart = false;   // start the point at parameter tr on the ray
      float tr = 0.0f;
      if (phase == PH_MARCH) {
        const int kh = inside ? (int)k : -1;
        k = kNoMarch;
        if (kh >= 0) {
          kstar = kh;
          if (kstar == 0) {
            thit = t0;
            next_normal = true;
          } else {
            lo = fmaf((float)(kstar - 1), dt, t0);
            hi = fmaf((float)kstar, dt, t0);
            if (P.B == 0) {
              thit = 0.5f * (lo + hi);
              next_normal = true;
            } else {
              b = 0;
              phase = PH_BISECT;
              tr = 0.5f * (lo + hi);
              restart = true;
            }
          }
        } else {  // no part found an inside sample: the ray misses
          write_pixel(F->out, pix, miss_pixel(DQJ_FLAG_BOX));
          phase = PH_IDLE;
        }
      } else if (phase == PH_BISECT) {
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
      } else {  // PH_NORMAL: stencil point sidx just retired (as in the loop above)
        if constexpr (WIDE) {
          stencil_add(gx, gy, gz, b, sidx, pot_log(n2c + h[0]), m);
        } else {
          const float G = potential(n2c + h[0], m);
          const float sg = (sidx & 1) ? -G : G;
          const int axis = sidx >> 1;
          if (axis == 0)
            gx += sg;
          else if (axis == 1)
            gy += sg;
          else
            gz += sg;
        }
        ++sidx;
      }
      if (next_normal) {
        phase = PH_NORMAL;
        // the four-neighbour normal is formed after the frame: no stencil points
        sidx = P.normal_mode != 0 ? 6 : 0;
        gx = gy = gz = 0.0f;
      }
      if (phase == PH_NORMAL && sidx == 6) {   // the hit is finished (g = 0: no stencil)
        const float g[3] = {gx, gy, gz};
        const float d[3] = {dx, dy, dz};
        PixelOut r;
        finish_hit(P, g, d, thit, kstar, (uint8_t)(DQJ_FLAG_BOX | DQJ_FLAG_HIT), r);
        write_pixel(F->out, pix, r);
        phase = PH_IDLE;
      }
      float px = 0, py = 0, pz = 0;
      if (restart) {
        px = fmaf(tr, dx, ex);
        py = fmaf(tr, dy, ey);
        pz = fmaf(tr, dz, ez);
      } else if (phase == PH_NORMAL) {
        const int axis = sidx >> 1;
        const float hs = (sidx & 1) ? -P.h : P.h;
        px = fmaf(thit, dx, ex) + (axis == 0 ? hs : 0.0f);
        py = fmaf(thit, dy, ey) + (axis == 1 ? hs : 0.0f);
        pz = fmaf(thit, dz, ez) + (axis == 2 ? hs : 0.0f);
      }
      if (phase != PH_IDLE) {
        start_point<AXIS>(P, px, py, pz, h[0], z, q);
        dl = trip + (uint32_t)N;
      } else {
        z = DQ<float>{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
        q = kNaN;
        dl = trip + kIdleAhead;
      }
    }

    if (__builtin_amdgcn_inverse_ballot_w64(fast)) {
      k += 1.0f;
      const float t = fmaf(k, dt, t0);
      const float x = fmaf(t, dx, ex);
      const float y = fmaf(t, dy, ey);
      const float w = fmaf(t, dz, ez);
      if constexpr (AXIS) {
        // First update in closed form.
        float a0;
        start_axis_q(x, y, w, h, c0c3, a0, z, q);
        if constexpr (STICKY) {
          // zeta_2 escapes whenever zeta_1 does: leave zeta_1 untested (a sample that
          // escaped on it retires after the next update, as a parked one would).
          dl = trip + (uint32_t)(N - 1);
        } else {
          // Test zeta_1. An escaped sample is parked on a state that escapes on the
          // next update (escape index 1); with max_iter 1 an inside one is parked on
          // NaN (never escapes) and retires on its deadline at the next trip.
          const bool esc1 = fmaf(a0, a0, cdsq - q) > R2c;
          a0 = esc1 ? 1e18f : (n_is_1 ? kNaN : a0);
          dl = trip + (uint32_t)(N - 1) + ((esc1 || n_is_1) ? 1u : 0u);
        }
        z.a0 = a0;
      } else {
        start_point<AXIS>(F->P, x, y, w, h[0], z, q);
        dl = trip + (uint32_t)N;
      }
    }

    if (!__builtin_amdgcn_ballot_w64(phase != PH_IDLE)) break;
    }
  }
  if (COUNT && frame >= 0 && F->out.iters) wave_add_u64(F->out.iters, it_lane);
}

// Single-frame launches: the frame record is a kernel argument.
template <int NORM, bool AXIS, bool COUNT, bool STICKY, bool WIDE>
__global__ __launch_bounds__(1024) void render_refill_kernel(FrameDesc single,
                                                             const FrameDesc *__restrict__ table,
                                                             const LaunchHeader *__restrict__ hdr,
                                                             int nframes, uint32_t total_tiles,
                                                             uint32_t *__restrict__ counter,
                                                             int TW, int TH) {
  refill_body<NORM, AXIS, false, COUNT, STICKY, kHandFirst, WIDE>(single, table, hdr, nframes,
                                                                  total_tiles, counter, TW, TH);
}

// Batched launches (frames from a device table: the throughput path) are held to 8 waves
// per SIMD. Their allocation then fits 64 VGPRs without spilling; left free, rare code
// of the slow path and the ray set-up pushes it to 65-69 and the occupancy to 7.
template <int NORM, bool AXIS, bool COUNT, bool STICKY, bool GUIDED, bool WIDE>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void
render_refill_batch_kernel(FrameDesc single, const FrameDesc *__restrict__ table,
                           const LaunchHeader *__restrict__ hdr, int nframes,
                           uint32_t total_tiles, uint32_t *__restrict__ counter, int TW, int TH) {
  refill_body<NORM, AXIS, true, COUNT, STICKY, GUIDED ? kHandGuided : kHandOne, WIDE>(
      single, table, hdr, nframes, total_tiles, counter, TW, TH);
}

__global__ void reset_counter_kernel(uint32_t *counter) { *counter = 0u; }

template <bool BATCH, bool COUNT, bool WIDE>
static void launch_refill_variant(const FrameDesc &single, const FrameDesc *table,
                                  const LaunchHeader *hdr, int nframes,
                                  uint32_t total_tiles, int norm, int mode, uint32_t *counter,
                                  const Sched &s, int blocks, int threads, hipStream_t stream) {
  // Guided chunks pay off only where a launch gives each wave many tiles (a sweep of
  // thousands of frames: 4096 frames of 256^2 4% faster); a separate instantiation keeps the
  // one-tile hand-out's code untouched elsewhere. Launches that read their size from a
  // device header (the server's epochs) keep one tile per atomic.
  const uint32_t nwaves = (uint32_t)blocks * (uint32_t)(threads >> 6);
  const bool guided = !COUNT && hdr == nullptr && total_tiles / nwaves >= 64u;
  (void)guided;
#define DQJ_LAUNCH(NM, AX, ST)                                                                 \
  do {                                                                                         \
    if constexpr (BATCH) {                                                                     \
      if (guided)                                                                              \
        hipLaunchKernelGGL((render_refill_batch_kernel<NM, AX, COUNT, ST, !COUNT, WIDE>), dim3(blocks), \
                           dim3(threads), 0, stream, single, table, hdr, nframes, total_tiles, \
                           counter, s.tile_w, s.tile_h);                                       \
      else                                                                                     \
        hipLaunchKernelGGL((render_refill_batch_kernel<NM, AX, COUNT, ST, false, WIDE>), dim3(blocks), \
                           dim3(threads), 0, stream, single, table, hdr, nframes, total_tiles, \
                           counter, s.tile_w, s.tile_h);                                       \
    } else                                                                                     \
      hipLaunchKernelGGL((render_refill_kernel<NM, AX, COUNT, ST, WIDE>), dim3(blocks), dim3(threads), \
                         0, stream, single, table, hdr, nframes, total_tiles, counter,         \
                         s.tile_w, s.tile_h);                                                  \
  } while (0)
  // counting launches test every first update, so they never take the STICKY variant
  mode &= kSliceMask;
  if (COUNT && mode == kSliceIdentitySticky) mode = kSliceIdentity;
  if (norm == 0) {
    if (mode == kSliceGeneral)
      DQJ_LAUNCH(0, false, false);
    else if (COUNT || mode == kSliceIdentity)
      DQJ_LAUNCH(0, true, false);
    else
      DQJ_LAUNCH(0, true, !COUNT);
  } else {
    if (mode == kSliceGeneral)
      DQJ_LAUNCH(1, false, false);
    else if (COUNT || mode == kSliceIdentity)
      DQJ_LAUNCH(1, true, false);
    else
      DQJ_LAUNCH(1, true, !COUNT);
  }
#undef DQJ_LAUNCH
}

template <bool BATCH>
static hipError_t launch_refill_impl(const FrameDesc &single, const FrameDesc *table,
                                     const LaunchHeader *hdr, int nframes,
                                     uint32_t total_tiles, int norm, int mode, bool count,
                                     uint32_t *counter, const Sched &s, int cus,
                                     hipStream_t stream) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, stream, counter);
  const int threads = 64 * s.waves_per_block;
  const int blocks = cus * s.blocks_per_cu;
#define DQJ_VARIANT(CT, WD)                                                                 \
  launch_refill_variant<BATCH, CT, WD>(single, table, hdr, nframes, total_tiles, norm, mode, counter, \
                                       s, blocks, threads, stream)
  const bool wide = (mode & kModeWide) != 0;
  if (count) {
    if (wide)
      DQJ_VARIANT(true, true);
    else
      DQJ_VARIANT(true, false);
  } else {
    if (wide)
      DQJ_VARIANT(false, true);
    else
      DQJ_VARIANT(false, false);
  }
#undef DQJ_VARIANT
  return hipGetLastError();
}

int slice_mode_of(const KParams &P) {
  const int wide = P.N > kUnscaledMaxIter ? kModeWide : 0;
  if (!P.axis_slice) return kSliceGeneral | wide;
  return (P.sticky1 ? kSliceIdentitySticky : kSliceIdentity) | wide;
}

int combine_slice_mode(int a, int b) {
  const int sa = a & kSliceMask, sb = b & kSliceMask;
  return (sa < sb ? sa : sb) | ((a | b) & kModeWide);
}

hipError_t launch_render_refill(const FrameDesc &frame, uint32_t *counter, const Sched &s, int cus,
                                hipStream_t stream) {
  return launch_refill_impl<false>(frame, nullptr, nullptr, 1, frame.ntiles, frame.P.norm,
                                   slice_mode_of(frame.P), frame.out.iters != nullptr, counter, s,
                                   cus, stream);
}

hipError_t launch_render_refill_batch(const FrameDesc *table_dev, const LaunchHeader *hdr_dev,
                                      int nframes, uint32_t total_tiles, int norm, int slice_mode,
                                      bool any_count, uint32_t *counter, const Sched &s, int cus,
                                      hipStream_t stream) {
  FrameDesc dummy;
  memset(&dummy, 0, sizeof dummy);
  return launch_refill_impl<true>(dummy, table_dev, hdr_dev, nframes, total_tiles, norm, slice_mode,
                                  any_count, counter, s, cus, stream);
}

}  // namespace dqj

// voxel.hip -- dense voxel-grid classification: the paper's first prototype (section
// "Ray-Marching" and its voxel-versus-ray-traced figure) as a throughput kernel. Every
// voxel centre x_i = box_min + (i + 1/2)(box_max - box_min)/n of the box is mapped
// through the slice and classified: N updates with the escape test after each
// (section "Practical Considerations"), under either algebra of the square.
//
// Design: persistent waves, one voxel per lane at a time, one update per trip on every
// lane (the lane-refill design of the ray marcher without rays). A lane walks a run of
// voxels along x. When its voxel escapes or reaches max_iter it writes the
// voxel's byte and starts the next voxel of its run in the same trip -- on the identity
// slice with the first update in closed form. Lanes whose run has ended take the next
// runs of the wave's chunk; waves take chunks of runs from one atomic counter, so the
// uneven cost of voxels (1 update far from the set, N inside it) never idles a lane.
// Runs interleave the lanes of a wave along the grid's memory order (see kPer).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>

#include "dq_device.h"
#include "kparams.h"
#include "persist.h"
#include "qform.h"
#include "runtime_internal.h"

namespace dqj {

using namespace persist;

namespace {

// The grid's voxels, in memory order ((k ny + j) nx + i), are cut into segments of
// stride * kPer voxels; a segment holds `stride` runs, and run o takes voxels o,
// o + stride, o + 2 stride, ... of the segment, across row ends. stride is 64 (the
// largest power of two <= nx on narrower grids, so a step crosses at most one row end).
// The 64 lanes of a wave thus walk a segment side by side and their one-byte stores land
// in a few cache lines at a time (on 1024^3 this took the kernel from 6.0 to 3.8 ms
// against lanes on contiguous runs, whose partly written lines overflow the L2). A chunk
// -- one atomic on the global counter, which sustains some 8e7 atomics/s, so chunks must
// not be small -- is the kChunk runs of kChunk / stride segments; larger chunks leave a
// longer tail (16k voxels per atomic measured best). Lanes drift apart within a segment,
// and the lines a wave has open grow with the segment: with 64-voxel runs (4 KB segments)
// the L2 wrote each mask line back 2.7 times over on 1024^3, with 32-voxel runs 1.2 times,
// at the same speed once the hand-out below divides in 32 bits (16-voxel runs: 1.03 times,
// but the hand-out then costs 12% of the time).
constexpr int kPer = 32;                  // voxels per run
constexpr uint32_t kChunk = 512;          // runs per chunk

struct GridDesc {
  KParams P;
  uint8_t *mask;                 // nx*ny*nz, x fastest: 1 inside, 0 outside
  int32_t *escape;               // optional: escape index, 0 when inside
  unsigned long long *iters;     // optional: updates run, accumulated
  float x0, dx, y0, dy, z0, dz;  // voxel centre of index i along an axis: fma(i, d, o)
  int32_t nx, ny, nz;
  int32_t stride;                // lanes' step through the voxels (see kPer)
  uint64_t nvox;                 // nx * ny * nz
  uint32_t nchunks;              // ceil(nvox / (kChunk * kPer))
};

// The square printed with Eq. dqjulia2: a' = a^2 + c_r, b' = b^2 + c_d, each quaternion
// squared as (s, v)^2 = (s^2 - |v|^2, 2 s v) (Eq. quatsq), in the q form of the dual
// update (q = c0 - |a_v|^2 carried, h the constant with h_i = c_i / 2 for i >= 1;
// returns the norm minus c0).
template <int NORM>
__device__ __forceinline__ float dq_update_cw(DQ<float> &z, float &q, const float *h) {
  const float qb = fmaf(-z.b3, z.b3, fmaf(-z.b2, z.b2, fmaf(-z.b1, z.b1, 2.0f * h[4])));
  DQ<float> r;
  r.a0 = fmaf(z.a0, z.a0, q);
  r.a1 = 2.0f * fmaf(z.a0, z.a1, h[1]);
  r.a2 = 2.0f * fmaf(z.a0, z.a2, h[2]);
  r.a3 = 2.0f * fmaf(z.a0, z.a3, h[3]);
  r.b0 = fmaf(z.b0, z.b0, qb);
  r.b1 = 2.0f * fmaf(z.b0, z.b1, h[5]);
  r.b2 = 2.0f * fmaf(z.b0, z.b2, h[6]);
  r.b3 = 2.0f * fmaf(z.b0, z.b3, h[7]);
  q = q_of(r, h[0]);
  float n2 = fmaf(r.a0, r.a0, -q);
  if (NORM == 0) n2 = fmaf(r.b3, r.b3, fmaf(r.b2, r.b2, fmaf(r.b1, r.b1, fmaf(r.b0, r.b0, n2))));
  z = r;
  return n2;
}

template <int NORM, bool CW>
__device__ __forceinline__ float grid_update(DQ<float> &z, float &q, const float *h) {
  if constexpr (CW)
    return dq_update_cw<NORM>(z, q, h);
  else
    return dq_update_q<NORM>(z, q, h);
}

// zeta_0 of voxel x on the run (y, z): on the identity slice zeta_1 in closed form,
// (x^2 - y^2 - z^2 + c0, 2xy + c1, 2xz + c2, c3 | c_d) under either algebra. Unless
// STICKY, a voxel that escapes on zeta_1 is parked on a state that escapes on the next
// update (escape index 1), and with max_iter 1 an inside one is parked on NaN and
// retires on its deadline. STICKY (the frame guarantees that escaping on zeta_1 implies
// escaping on zeta_2) leaves zeta_1 untested: classes are unchanged, escape indices are
// not kept.
template <bool AXIS, bool STICKY>
__device__ __forceinline__ void start_voxel(const KParams &P, float x, float yw, float zw,
                                            const float *h, const float *cf, float c0c3,
                                            float cdsq, float R2c,
                                            int N, bool n_is_1, uint32_t trip, DQ<float> &z,
                                            float &q, uint32_t &dl) {
  if constexpr (AXIS) {
    float a0;
    start_axis_q_mov(x, yw, zw, h, cf, c0c3, a0, z, q);
    if constexpr (STICKY) {
      dl = trip + (uint32_t)(N - 1);
    } else {
      const bool esc1 = fmaf(a0, a0, cdsq - q) > R2c;
      a0 = esc1 ? 1e18f : (n_is_1 ? __builtin_nanf("") : a0);
      dl = trip + (uint32_t)(N - 1) + ((esc1 || n_is_1) ? 1u : 0u);
    }
    z.a0 = a0;
  } else {
    z = slice_map<float>(P, x, yw, zw);
    q = q_of(z, h[0]);
    dl = trip + (uint32_t)N;
  }
}

// Template switches: NORM (escape norm), AXIS (identity slice: first update in closed
// form), CW (component-wise square), EXTRA (write escape indices and count updates),
// STICKY (see start_voxel; AXIS and not EXTRA only).
template <int NORM, bool AXIS, bool CW, bool EXTRA, bool STICKY>
__global__ __launch_bounds__(1024) void classify_grid_kernel(GridDesc G, uint32_t *__restrict__ counter) {
  const int lane = lane_id();
  const float kNaN = __builtin_nanf("");
  const uint32_t kIdleAhead = 0x7FFFFFFFu;
  // per-lane copies of c0 and c_i / 2 (the q form), of R^2 - c0 and of c0 - c3^2
  float h[8];
  h[0] = to_vgpr(G.P.c[0]);
#pragma unroll
  for (int q = 1; q < 8; ++q) h[q] = to_vgpr(0.5f * G.P.c[q]);
  const float R2c = to_vgpr(G.P.R2 - G.P.c[0]);
  float cf[8];   // c3..c7 in full, for the closed-form start
#pragma unroll
  for (int q = 0; q < 8; ++q) cf[q] = q >= 3 ? to_vgpr(G.P.c[q]) : 0.0f;
  const int N = G.P.N;
  const bool n_is_1 = N == 1;
  // |c_d|^2: the dual part of zeta_1 on the identity slice is c_d under both algebras
  const float cdsq = NORM == 0 ? fmaf(G.P.c[7], G.P.c[7], fmaf(G.P.c[6], G.P.c[6],
                                      fmaf(G.P.c[5], G.P.c[5], G.P.c[4] * G.P.c[4])))
                               : 0.0f;
  const float c0c3 = to_vgpr(fmaf(-G.P.c[3], G.P.c[3], G.P.c[0]));
  // the grid's axes and sizes, also as per-lane copies (the retire step reads them on
  // nearly every trip; scalar-register operands would cost a move or a slower issue)
  const float x0 = to_vgpr(G.x0), dx = to_vgpr(G.dx);
  const float y0 = to_vgpr(G.y0), dy = to_vgpr(G.dy);
  const float z0 = to_vgpr(G.z0), dz = to_vgpr(G.dz);

  // wave-uniform hand-out state
  uint32_t chunk = 0, next_r = 0;
  const uint32_t kNoChunk = 0xFFFFFFFFu;
  const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
  uint32_t first_chunk = uniform(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  bool have_chunk = false, exhausted = false;

  // per-lane state: an idle lane sits on NaN (never escapes) with a far deadline
  uint32_t trip = 0;
  DQ<float> z{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
  float q = kNaN;
  uint32_t dl = kIdleAhead;
  // the current voxel's mask byte and the end of its run's segment (memory order)
  uint8_t *pv = G.mask, *pend = G.mask;
  int i = 0, j = 0, k = 0;         // grid coordinates of the current voxel
  float yw = 0.0f, zw = 0.0f;      // world y, z of row (j, k)
  const int stride = G.stride;
  const int nx = (int)__float_as_uint(to_vgpr(__uint_as_float((uint32_t)G.nx)));
  const int ny = (int)__float_as_uint(to_vgpr(__uint_as_float((uint32_t)G.ny)));
  unsigned long long it_lane = 0;
  const bool small = G.nvox <= 0xFFFFFFFFull;   // voxel indices fit 32 bits

  enter_update_mode();
  for (;;) {
    ++trip;
    const float n2 = grid_update<NORM, CW>(z, q, h);   // norm minus c0
    const bool esc = n2 > R2c;
    if (esc || (int)(trip - dl) >= 0) {
      // the voxel retires: escape index m, or N when it stayed inside
      *pv = esc ? 0 : 1;
      if (EXTRA) {
        const int m = N - (int)(dl - trip);
        if (G.escape) G.escape[pv - G.mask] = esc ? m : 0;
        it_lane += (unsigned long long)m;
      }
      // Start the next voxel of the run. A lane that has just passed the end of its run
      // starts a voxel it never retires: the hand-out below, in this same trip, gives it
      // a new run or parks it.
      // step to the run's next voxel; at most one row end lies in between
      pv += stride;
      i += stride;
      const bool wrap = i >= nx;
      i = wrap ? i - nx : i;
      j += wrap ? 1 : 0;
      const bool wrapj = j >= ny;
      j = wrapj ? 0 : j;
      k += wrapj ? 1 : 0;
      yw = fmaf((float)j, dy, y0);
      zw = fmaf((float)k, dz, z0);
      start_voxel<AXIS, STICKY>(G.P, fmaf((float)i, dx, x0), yw, zw, h, cf, c0c3, cdsq, R2c, N,
                                n_is_1, trip, z, q, dl);
    }

    // ---- hand runs to idle lanes (rare: a run lasts dozens of trips)
    uint64_t idle = __builtin_amdgcn_ballot_w64(pv >= pend);
    if (idle) {
      while (idle) {
        if (!have_chunk) {
          if (exhausted) break;
          // The first chunk of every wave comes without the counter (wave w takes chunk
          // w), which then hands out chunks from nwaves on: at the start all waves would
          // queue on one atomic (about 60-80 us of the launch on 1024^3).
          uint32_t t = first_chunk;
          if (t == kNoChunk) {
            if (lane == 0) t = atomicAdd(counter, 1u);
            t = uniform(t) + nwaves;
          }
          first_chunk = kNoChunk;
          if (t >= G.nchunks) {
            exhausted = true;
            break;
          }
          chunk = t;
          next_r = 0;
          have_chunk = true;
        }
        const uint32_t avail = kChunk - next_r;
        const uint32_t rank = (uint32_t)rank_in(idle);
        if (pv >= pend && rank < avail) {
          const uint32_t run = next_r + rank;             // run within the chunk
          const uint64_t seg = (uint64_t)chunk * (kChunk / stride) + run / stride;
          const uint64_t s0 = seg * (uint64_t)stride * kPer;
          const uint64_t v = s0 + run % stride;
          pv = G.mask + v;
          pend = G.mask + min(s0 + (uint64_t)stride * kPer, G.nvox);   // pv >= pend: an empty run
          if (small) {   // 32-bit division: several times cheaper than 64-bit on the GPU
            const uint32_t v32 = (uint32_t)v, row = v32 / (uint32_t)nx, kk = row / (uint32_t)ny;
            i = (int)(v32 - row * (uint32_t)nx);
            j = (int)(row - kk * (uint32_t)ny);
            k = (int)kk;
          } else {
            const uint64_t row = v / (uint64_t)nx;
            i = (int)(v - row * (uint64_t)nx);
            j = (int)(row % (uint64_t)ny);
            k = (int)(row / (uint64_t)ny);
          }
          yw = fmaf((float)j, dy, y0);
          zw = fmaf((float)k, dz, z0);
          start_voxel<AXIS, STICKY>(G.P, fmaf((float)i, dx, x0), yw, zw, h, cf, c0c3, cdsq, R2c, N,
                                    n_is_1, trip, z, q, dl);
        }
        const uint32_t cnt = (uint32_t)__popcll(idle);
        next_r += cnt < avail ? cnt : avail;
        if (next_r >= kChunk) have_chunk = false;
        idle = __builtin_amdgcn_ballot_w64(pv >= pend);
      }
      // lanes left without a run sit on NaN (never escapes) with a far deadline
      if (pv >= pend) {
        z = DQ<float>{kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN, kNaN};
        q = kNaN;
        dl = trip + kIdleAhead;
      }
      if (exhausted && !__builtin_amdgcn_ballot_w64(pv < pend)) break;
    }
  }
  if (EXTRA && G.iters) wave_add_u64(G.iters, it_lane);
}

__global__ void grid_reset_counter_kernel(uint32_t *counter) { *counter = 0u; }

template <bool EXTRA, bool STICKY>
void launch_grid_variant(const GridDesc &g, uint32_t *counter, int blocks, int threads,
                         hipStream_t stream) {
#define DQJ_GRID(NM, AX, CWA)                                                               \
  hipLaunchKernelGGL((classify_grid_kernel<NM, AX, CWA, EXTRA, STICKY && AX>), dim3(blocks), \
                     dim3(threads), 0, stream, g, counter)
  const bool axis = g.P.axis_slice != 0, cw = g.P.algebra != 0;
  if (g.P.norm == 0) {
    if (axis) {
      if (cw) DQJ_GRID(0, true, true); else DQJ_GRID(0, true, false);
    } else {
      if (cw) DQJ_GRID(0, false, true); else DQJ_GRID(0, false, false);
    }
  } else {
    if (axis) {
      if (cw) DQJ_GRID(1, true, true); else DQJ_GRID(1, true, false);
    } else {
      if (cw) DQJ_GRID(1, false, true); else DQJ_GRID(1, false, false);
    }
  }
#undef DQJ_GRID
}

}  // namespace

}  // namespace dqj

using namespace dqj;

extern "C" dqj_status dqj_classify_grid(const dqj_params *params, int32_t nx, int32_t ny,
                                        int32_t nz, uint8_t *mask_dev, int32_t *escape_dev,
                                        unsigned long long *iters_dev, void *hip_stream) {
  try {
    dqj_status s = validate_params(params);
    if (s != DQJ_OK) return s;
    if (params->precision != DQJ_PREC_FP32)
      return fail(DQJ_E_UNSUPPORTED, "grid classification runs in FP32");
    if (nx < 1 || ny < 1 || nz < 1 || nx > 4096 || ny > 4096 || nz > 4096)
      return fail(DQJ_E_INVALID, "grid sizes must be in 1..4096 (got %d x %d x %d)", nx, ny, nz);
    if (!mask_dev) return fail(DQJ_E_INVALID, "mask is required");
    int cus = 0;
    s = current_device(nullptr, &cus);
    if (s != DQJ_OK) return s;
    GridDesc g;
    memset(&g, 0, sizeof g);
    pack_params(*params, g.P);
    g.mask = mask_dev;
    g.escape = escape_dev;
    g.iters = iters_dev;
    const int32_t n[3] = {nx, ny, nz};
    float o[3], d[3];
    for (int a = 0; a < 3; ++a) {
      const double step = (params->box_max[a] - params->box_min[a]) / n[a];
      d[a] = (float)step;
      o[a] = (float)(params->box_min[a] + 0.5 * step);
    }
    g.x0 = o[0];
    g.dx = d[0];
    g.y0 = o[1];
    g.dy = d[1];
    g.z0 = o[2];
    g.dz = d[2];
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.stride = 64;
    while (g.stride > nx) g.stride >>= 1;
    g.nvox = (uint64_t)nx * (uint64_t)ny * (uint64_t)nz;
    const uint64_t per_chunk = (uint64_t)kChunk * kPer;
    g.nchunks = (uint32_t)((g.nvox + per_chunk - 1) / per_chunk);
    hipStream_t stream = (hipStream_t)hip_stream;
    uint32_t *counter = nullptr;
    hipError_t e = stream_counter(stream, &counter);
    if (e != hipSuccess) return hip_fail(e, "grid counter");
    hipLaunchKernelGGL(grid_reset_counter_kernel, dim3(1), dim3(1), 0, stream, counter);
    const int threads = 256, blocks = cus * 8;
    // the first-update guarantee is derived for the product-rule square
    const bool sticky = g.P.sticky1 != 0 && g.P.algebra == 0;
    if (escape_dev || iters_dev)
      launch_grid_variant<true, false>(g, counter, blocks, threads, stream);
    else if (sticky)
      launch_grid_variant<false, true>(g, counter, blocks, threads, stream);
    else
      launch_grid_variant<false, false>(g, counter, blocks, threads, stream);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "grid launch");
    return DQJ_OK;
  } catch (const std::bad_alloc &) {
    return fail(DQJ_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(DQJ_E_DEVICE, "unexpected internal error");
  }
}

// runtime.hip -- host runtime and C ABI exports: validation, FP64 -> FP32 parameter
// packing, device checks, error reporting, and launches of the render kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dqj.h"
#include "kparams.h"
#include "launch.h"
#include "refill.h"
#include "split.h"
#include "runtime_internal.h"

namespace dqj {

static thread_local std::string t_last_error;

dqj_status fail(dqj_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return s;
}

dqj_status hip_fail(hipError_t e, const char *what) {
  return fail(DQJ_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---- device checks --------------------------------------------------------

struct DevInfo {
  bool probed = false;
  bool gfx950 = false;
  int cus = 0;
  int clock_khz = 0;
  int mem_clock_khz = 0;
  size_t total_mem = 0;
  char arch[64] = {0};
};

static std::mutex g_dev_mu;
static std::vector<DevInfo> g_dev;

static const DevInfo *probe_device(int dev) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  DevInfo &d = g_dev[dev];
  if (!d.probed) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      snprintf(d.arch, sizeof d.arch, "%s", prop.gcnArchName);
      d.gfx950 = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
      d.cus = prop.multiProcessorCount;
      d.clock_khz = prop.clockRate;
      d.mem_clock_khz = prop.memoryClockRate;
      d.total_mem = prop.totalGlobalMem;
    }
    d.probed = true;
  }
  return &d;
}

dqj_status current_device(int *dev, int *cus) {
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  const DevInfo *info = probe_device(d);
  if (!info->gfx950)
    return fail(DQJ_E_UNSUPPORTED, "device %d is '%s'; this library runs on gfx950 only", d,
                info->arch);
  if (dev) *dev = d;
  if (cus) *cus = info->cus;
  return DQJ_OK;
}

// ---- validation -----------------------------------------------------------

static bool fin(double x) { return std::isfinite(x); }

dqj_status validate_params(const dqj_params *p) {
  if (!p) return fail(DQJ_E_INVALID, "params is NULL");
  if (p->struct_size != sizeof(dqj_params))
    return fail(DQJ_E_INVALID, "params.struct_size %u != %zu", p->struct_size, sizeof(dqj_params));
  for (int k = 0; k < 8; ++k)
    if (!fin(p->c[k]) || !fin(p->slice_origin[k]) || !fin(p->slice_axes[0][k]) ||
        !fin(p->slice_axes[1][k]) || !fin(p->slice_axes[2][k]))
      return fail(DQJ_E_INVALID, "c or slice has a non-finite component");
  for (int k = 0; k < 3; ++k) {
    if (!fin(p->box_min[k]) || !fin(p->box_max[k]) || !(p->box_min[k] < p->box_max[k]))
      return fail(DQJ_E_INVALID, "box_min must be < box_max and finite (axis %d)", k);
    if (!fin(p->eye[k]) || !fin(p->target[k]) || !fin(p->up[k]) || !fin(p->light_dir[k]))
      return fail(DQJ_E_INVALID, "camera or light has a non-finite component");
  }
  if (p->width < 1 || p->width > 16384 || p->height < 1 || p->height > 16384)
    return fail(DQJ_E_INVALID, "width/height must be in 1..16384 (got %d x %d)", p->width,
                p->height);
  if (p->max_iter < 1 || p->max_iter > 4096)
    return fail(DQJ_E_INVALID, "max_iter must be in 1..4096 (got %d)", p->max_iter);
  if (p->march_steps < 1 || p->march_steps > (1 << 20))
    return fail(DQJ_E_INVALID, "march_steps must be in 1..2^20 (got %d)", p->march_steps);
  if (p->bisect_steps < 0 || p->bisect_steps > 64)
    return fail(DQJ_E_INVALID, "bisect_steps must be in 0..64 (got %d)", p->bisect_steps);
  if (!fin(p->escape_radius) || !(p->escape_radius > 0))
    return fail(DQJ_E_INVALID, "escape_radius must be finite and > 0");
  if (!fin(p->fov_y_deg) || !(p->fov_y_deg > 0) || !(p->fov_y_deg < 180))
    return fail(DQJ_E_INVALID, "fov_y_deg must be in (0, 180)");
  if (!fin(p->normal_h) || !(p->normal_h > 0))
    return fail(DQJ_E_INVALID, "normal_h must be finite and > 0");
  if ((int64_t)(p->march_steps + p->bisect_steps + 8) * p->max_iter > (int64_t)1 << 30)
    return fail(DQJ_E_INVALID, "(march_steps + bisect_steps + 8) * max_iter must not exceed 2^30");
  if (!fin(p->k_ambient) || !fin(p->k_diffuse))
    return fail(DQJ_E_INVALID, "k_ambient/k_diffuse must be finite");
  if (p->norm != DQJ_NORM_EUCLID8 && p->norm != DQJ_NORM_REALPART)
    return fail(DQJ_E_INVALID, "norm must be DQJ_NORM_EUCLID8 or DQJ_NORM_REALPART");
  if (p->precision != DQJ_PREC_FP32 && p->precision != DQJ_PREC_SPLIT &&
      p->precision != DQJ_PREC_FP64)
    return fail(DQJ_E_INVALID, "precision must be one of DQJ_PREC_*");
  if (p->march != DQJ_MARCH_FIXED && p->march != DQJ_MARCH_DE)
    return fail(DQJ_E_INVALID, "march must be one of DQJ_MARCH_*");
  if (p->march == DQJ_MARCH_DE) {
    if (!(p->de_hit_eps > 0.0 && std::isfinite(p->de_hit_eps)) ||
        !(p->de_min_step > 0.0 && std::isfinite(p->de_min_step)) ||
        !(p->de_max_step >= p->de_min_step && std::isfinite(p->de_max_step)))
      return fail(DQJ_E_INVALID,
                  "DE march needs de_hit_eps > 0 and 0 < de_min_step <= de_max_step, finite");
  }
  if (p->algebra != DQJ_ALGEBRA_DUAL && p->algebra != DQJ_ALGEBRA_COMPONENTWISE)
    return fail(DQJ_E_INVALID, "algebra must be one of DQJ_ALGEBRA_*");
  if (p->normal_mode != DQJ_NORMAL_POTENTIAL && p->normal_mode != DQJ_NORMAL_NEIGHBOUR4)
    return fail(DQJ_E_INVALID, "normal_mode must be one of DQJ_NORMAL_*");
  if (!fin(p->k_specular) || !(p->k_specular >= 0.0))
    return fail(DQJ_E_INVALID, "k_specular must be finite and >= 0");
  if (!fin(p->shininess) || !(p->shininess >= 1.0) || !(p->shininess <= 1e4))
    return fail(DQJ_E_INVALID, "shininess must be in [1, 1e4]");
  if (!fin(p->cull_radius) || !(p->cull_radius >= 0.0))
    return fail(DQJ_E_INVALID, "cull_radius must be finite and >= 0");
  if (p->fiber_count < 0 || p->fiber_count > kMaxFiber)
    return fail(DQJ_E_INVALID, "fiber_count must be in 0..%d (got %d)", kMaxFiber, p->fiber_count);
  if (p->fiber_reserved != 0) return fail(DQJ_E_INVALID, "fiber_reserved must be 0");
  if (p->fiber_count > 0) {
    if (!p->fiber) return fail(DQJ_E_INVALID, "fiber is NULL with fiber_count %d", p->fiber_count);
    for (int i = 0; i < 8 * p->fiber_count; ++i)
      if (!fin(p->fiber[i])) return fail(DQJ_E_INVALID, "fiber[%d] is not finite", i);
  }
  if (p->precision == DQJ_PREC_SPLIT && (p->fp64_window < 1 || p->fp64_window > 8))
    return fail(DQJ_E_INVALID, "fp64_window must be in 1..8 for split precision");
  if (p->precision == DQJ_PREC_SPLIT && !(p->escape_radius * p->escape_radius < 65504.0))
    return fail(DQJ_E_INVALID, "split precision needs escape_radius^2 < 65504 (FP16 range)");
  const double f[3] = {p->target[0] - p->eye[0], p->target[1] - p->eye[1], p->target[2] - p->eye[2]};
  const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(fl > 0)) return fail(DQJ_E_INVALID, "eye and target coincide");
  const double ul = std::sqrt(p->up[0] * p->up[0] + p->up[1] * p->up[1] + p->up[2] * p->up[2]);
  const double cx = f[1] * p->up[2] - f[2] * p->up[1];
  const double cy = f[2] * p->up[0] - f[0] * p->up[2];
  const double cz = f[0] * p->up[1] - f[1] * p->up[0];
  if (!(std::sqrt(cx * cx + cy * cy + cz * cz) > 1e-9 * fl * ul))
    return fail(DQJ_E_INVALID, "up is parallel to the view direction");
  const double ll = std::sqrt(p->light_dir[0] * p->light_dir[0] + p->light_dir[1] * p->light_dir[1] +
                              p->light_dir[2] * p->light_dir[2]);
  if (!(ll > 0)) return fail(DQJ_E_INVALID, "light_dir is zero");
  return DQJ_OK;
}

dqj_status check_render_modes(const dqj_params &p, bool single) {
  if (p.algebra != DQJ_ALGEBRA_DUAL)
    return fail(DQJ_E_UNSUPPORTED, "the component-wise algebra is offered by dqj_classify_grid only");
  if (p.fiber_count > 0) {
    if (!single) return fail(DQJ_E_UNSUPPORTED, "projection rendering is offered by dqj_render and batches only");
    if (p.precision != DQJ_PREC_FP32 || p.march != DQJ_MARCH_FIXED)
      return fail(DQJ_E_UNSUPPORTED, "projection rendering runs the FP32 fixed-step march");
  }
  if (p.normal_mode == DQJ_NORMAL_NEIGHBOUR4 && !single)
    return fail(DQJ_E_UNSUPPORTED, "the four-neighbour normal is offered by dqj_render only");
  return DQJ_OK;
}

dqj_status validate_out(const dqj_frame_out *o) {
  if (!o) return fail(DQJ_E_INVALID, "out is NULL");
  if (o->struct_size != sizeof(dqj_frame_out))
    return fail(DQJ_E_INVALID, "out.struct_size %u != %zu", o->struct_size, sizeof(dqj_frame_out));
  if (!o->mask || !o->depth || !o->shade)
    return fail(DQJ_E_INVALID, "out.mask, out.depth and out.shade are required");
  return DQJ_OK;
}

// ---- packing --------------------------------------------------------------

void pack_params(const dqj_params &p, KParams &k) {
  memset(&k, 0, sizeof k);
  for (int i = 0; i < 8; ++i) {
    k.c[i] = (float)p.c[i];
    k.so[i] = (float)p.slice_origin[i];
    k.su[i] = (float)p.slice_axes[0][i];
    k.sv[i] = (float)p.slice_axes[1][i];
    k.sw[i] = (float)p.slice_axes[2][i];
  }
  bool axis = true;
  for (int i = 0; i < 8; ++i) {
    axis = axis && p.slice_origin[i] == 0.0;
    axis = axis && p.slice_axes[0][i] == (i == 0 ? 1.0 : 0.0);
    axis = axis && p.slice_axes[1][i] == (i == 1 ? 1.0 : 0.0);
    axis = axis && p.slice_axes[2][i] == (i == 2 ? 1.0 : 0.0);
  }
  k.axis_slice = axis ? 1 : 0;
  // camera basis in FP64, rounded once
  double f[3] = {p.target[0] - p.eye[0], p.target[1] - p.eye[1], p.target[2] - p.eye[2]};
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (double &x : f) x /= fl;
  double r[3] = {f[1] * p.up[2] - f[2] * p.up[1], f[2] * p.up[0] - f[0] * p.up[2],
                 f[0] * p.up[1] - f[1] * p.up[0]};
  double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (double &x : r) x /= rl;
  const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2],
                       r[0] * f[1] - r[1] * f[0]};
  const double tan_half = std::tan(0.5 * p.fov_y_deg * M_PI / 180.0);
  double l[3] = {p.light_dir[0], p.light_dir[1], p.light_dir[2]};
  const double ll = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
  for (int i = 0; i < 3; ++i) {
    k.eye[i] = (float)p.eye[i];
    k.fwd[i] = (float)f[i];
    k.right[i] = (float)r[i];
    k.up[i] = (float)u[i];
    k.bmin[i] = (float)p.box_min[i];
    k.bmax[i] = (float)p.box_max[i];
    k.light[i] = (float)(l[i] / ll);
  }
  k.sx_scale = (float)(tan_half * (double)p.width / (double)p.height);
  k.sy_scale = (float)tan_half;
  k.inv_w = (float)(1.0 / p.width);
  k.inv_h = (float)(1.0 / p.height);
  k.R2 = (float)(p.escape_radius * p.escape_radius);
  k.h = (float)p.normal_h;
  k.ka = (float)p.k_ambient;
  k.kd = (float)p.k_diffuse;
  k.W = p.width;
  k.H = p.height;
  k.N = p.max_iter;
  k.S = p.march_steps;
  k.B = p.bisect_steps;
  k.norm = p.norm;
  k.fp64_window = p.fp64_window;
  // FP16 orbits of points near the set's boundary part from the exact orbit after some
  // updates, so the FP16 march trusts an escape only when it comes within T16 updates;
  // samples that escape later are re-checked in FP32. T16 = N - ceil(N/4) with the
  // 8-square norm, ceil(3N/8) with the real-part norm, whose set is rougher (measured on
  // FP16-emulated orbits against FP64: these depths lose no crossing on sampled rays).
  {
    const int N = p.max_iter;
    const int t = p.norm == DQJ_NORM_REALPART ? (3 * N + 7) / 8 : N - (N + 3) / 4;
    k.T16 = t > 1 ? t : 1;
  }
  k.march = p.march;
  k.de_eps = (float)p.de_hit_eps;
  k.de_min_step = (float)p.de_min_step;
  k.de_max_step = (float)p.de_max_step;
  k.de_inv_r2 = (float)(1.0 / (p.escape_radius * p.escape_radius));
  k.de_log2_4r2 = (float)std::log2(4.0 * p.escape_radius * p.escape_radius);
  k.algebra = p.algebra;
  k.normal_mode = p.normal_mode;
  k.ks = (float)p.k_specular;
  k.shininess = (float)p.shininess;
  k.cull_r2 = (float)(p.cull_radius * p.cull_radius);
  // On the identity slice zeta_0 = (x, y, z, 0 | 0), so zeta_1 = (a | c_d) with a real
  // quaternion a. If zeta_1 escapes, |a|^2 > R^2 - |c_d|^2 (8 squares) or > R^2 (real
  // part). The real part of zeta_2 is a^2 + c_r and the quaternion norm is
  // multiplicative, so |a^2 + c_r| >= |a|^2 - |c_r|: once that bound on |a|^2 is at
  // least R + |c_r|, zeta_2 escapes too. A 1% margin covers FP32 rounding of the
  // state. Kernels then may let such a point run one more update instead of testing
  // zeta_1 (the classification is the same; only the escape index differs).
  {
    double cr = 0, cd = 0;
    for (int i = 0; i < 4; ++i) {
      cr += (double)k.c[i] * (double)k.c[i];
      cd += (double)k.c[4 + i] * (double)k.c[4 + i];
    }
    const double R = std::sqrt((double)k.R2);
    const double q = (double)k.R2 - (p.norm == DQJ_NORM_REALPART ? 0.0 : cd);
    k.sticky1 = (k.axis_slice && k.N > 1 && q >= 1.01 * (R + std::sqrt(cr)) + 1e-6) ? 1 : 0;
  }
}

void pack_params64(const dqj_params &p, KParams64 &k) {
  memset(&k, 0, sizeof k);
  for (int i = 0; i < 8; ++i) {
    k.c[i] = p.c[i];
    k.so[i] = p.slice_origin[i];
    k.su[i] = p.slice_axes[0][i];
    k.sv[i] = p.slice_axes[1][i];
    k.sw[i] = p.slice_axes[2][i];
  }
  double f[3] = {p.target[0] - p.eye[0], p.target[1] - p.eye[1], p.target[2] - p.eye[2]};
  const double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (double &x : f) x /= fl;
  double r[3] = {f[1] * p.up[2] - f[2] * p.up[1], f[2] * p.up[0] - f[0] * p.up[2],
                 f[0] * p.up[1] - f[1] * p.up[0]};
  const double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (double &x : r) x /= rl;
  const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2],
                       r[0] * f[1] - r[1] * f[0]};
  const double tan_half = std::tan(0.5 * p.fov_y_deg * M_PI / 180.0);
  const double ll = std::sqrt(p.light_dir[0] * p.light_dir[0] + p.light_dir[1] * p.light_dir[1] +
                              p.light_dir[2] * p.light_dir[2]);
  for (int i = 0; i < 3; ++i) {
    k.eye[i] = p.eye[i];
    k.fwd[i] = f[i];
    k.right[i] = r[i];
    k.up[i] = u[i];
    k.bmin[i] = p.box_min[i];
    k.bmax[i] = p.box_max[i];
    k.light[i] = p.light_dir[i] / ll;
  }
  k.sx_scale = tan_half * (double)p.width / (double)p.height;
  k.sy_scale = tan_half;
  k.inv_w = 1.0 / p.width;
  k.inv_h = 1.0 / p.height;
  k.R2 = p.escape_radius * p.escape_radius;
  k.h = p.normal_h;
  k.ka = p.k_ambient;
  k.kd = p.k_diffuse;
  k.ks = p.k_specular;
  k.shininess = p.shininess;
  k.cull_r2 = p.cull_radius * p.cull_radius;
  k.normal_mode = p.normal_mode;
}

KOut to_kout(const dqj_frame_out &o) {
  KOut k;
  k.mask = o.mask;
  k.depth = o.depth;
  k.shade = o.shade;
  k.image8 = o.image8;
  k.normal = o.normal;
  k.first_hit = o.first_hit;
  k.flags = o.flags;
  k.iters = o.iters;
  return k;
}

Sched resolve_schedule(const dqj_schedule *s, int cus) {
  (void)cus;
  Sched r;
  r.kernel = DQJ_KERNEL_REFILL;
  r.tile_w = 8;
  r.tile_h = 8;
  r.waves_per_block = 4;
  r.blocks_per_cu = 8;
  if (s) {
    if (s->kernel) r.kernel = s->kernel;
    if (s->tile_w) r.tile_w = s->tile_w;
    if (s->tile_h) r.tile_h = s->tile_h;
    if (s->waves_per_block) r.waves_per_block = s->waves_per_block;
    if (s->blocks_per_cu) r.blocks_per_cu = s->blocks_per_cu;
  }
  return r;
}

static dqj_status check_schedule(const dqj_schedule *s) {
  if (!s) return DQJ_OK;
  if (s->struct_size != sizeof(dqj_schedule))
    return fail(DQJ_E_INVALID, "schedule.struct_size %u != %zu", s->struct_size, sizeof(dqj_schedule));
  if (s->kernel < 0 || s->kernel > DQJ_KERNEL_LOCKSTEP)
    return fail(DQJ_E_INVALID, "schedule.kernel must be one of DQJ_KERNEL_*");
  if (s->tile_w < 0 || s->tile_h < 0 || s->tile_w * s->tile_h > 4096)
    return fail(DQJ_E_INVALID, "schedule tile must satisfy tile_w * tile_h <= 4096");
  if (s->waves_per_block < 0 || s->waves_per_block > 16)
    return fail(DQJ_E_INVALID, "schedule.waves_per_block must be in 0..16");
  if (s->blocks_per_cu < 0 || s->blocks_per_cu > 32)
    return fail(DQJ_E_INVALID, "schedule.blocks_per_cu must be in 0..32");
  return DQJ_OK;
}

// ---- per-stream device scratch ---------------------------------------------
// Each (device, stream) pair gets one 256-byte device block for its persistent
// kernels' tile counter. Work on one stream is ordered, so the block is never used
// by two launches at once.

struct StreamSlot {
  int dev;
  hipStream_t stream;
  uint32_t *counter;
  void *scratch;
  size_t scratch_bytes;
};
static std::mutex g_slot_mu;
static std::vector<StreamSlot> g_slots;

static StreamSlot *find_slot(int dev, hipStream_t stream, hipError_t *err) {
  for (StreamSlot &s : g_slots)
    if (s.dev == dev && s.stream == stream) return &s;
  void *p = nullptr;
  *err = hipMalloc(&p, 256);
  if (*err != hipSuccess) return nullptr;
  g_slots.push_back(StreamSlot{dev, stream, (uint32_t *)p, nullptr, 0});
  return &g_slots.back();
}

hipError_t stream_counter(hipStream_t stream, uint32_t **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_slot_mu);
  StreamSlot *s = find_slot(dev, stream, &e);
  if (!s) return e;
  *out = s->counter;
  return hipSuccess;
}

// Device scratch private to (current device, stream), grown on demand. Work on one
// stream is ordered, so reuse by the next call on the stream is safe; growing first
// waits for the stream so the old block is no longer in use.
hipError_t stream_scratch(hipStream_t stream, size_t bytes, void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_slot_mu);
  StreamSlot *s = find_slot(dev, stream, &e);
  if (!s) return e;
  if (s->scratch_bytes < bytes) {
    if (s->scratch) {
      e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return e;
      (void)hipFree(s->scratch);
      s->scratch = nullptr;
      s->scratch_bytes = 0;
    }
    e = hipMalloc(&s->scratch, bytes);
    if (e != hipSuccess) return e;
    s->scratch_bytes = bytes;
  }
  *out = s->scratch;
  return hipSuccess;
}

// ---- fixed scratch of dqj_render_noalloc -------------------------------------
// A file-scope device array, one copy per GPU, holds what dqj_render keeps in its
// per-stream blocks: the tile counter and, for split renders, the candidate and FP64
// lists. On the host the array's name is only a stand-in: host code uses the address
// hipGetSymbolAddress returns with the device current, looked up once per device.

static_assert(split_scratch_bytes(DQJ_NOALLOC_MAX_SPLIT_PIXELS) == DQJ_NOALLOC_SCRATCH_BYTES,
              "the fixed scratch holds the lists of the largest split frame it accepts");
static __device__ __align__(256) unsigned char scratch[DQJ_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_fixed_mu;
static void *g_fixed[kMaxDevices];

static hipError_t fixed_scratch(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_fixed_mu);
  if (!g_fixed[dev]) {
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_fixed[dev] = ptr;
  }
  *out = g_fixed[dev];
  return hipSuccess;
}

// Tile counter of a persistent launch: the start of the fixed scratch when one is
// given, else the stream's own block.
static hipError_t launch_counter(void *fixed, hipStream_t stream, uint32_t **out) {
  if (fixed) {
    *out = (uint32_t *)fixed;
    return hipSuccess;
  }
  return stream_counter(stream, out);
}

static hipError_t launch_render_fp32_at(const KParams &P, const KOut &out, const Sched &s, int cus,
                                        void *fixed, hipStream_t stream) {
  if (s.kernel == DQJ_KERNEL_DIRECT) return launch_render_direct(P, out, stream);
  FrameDesc f;
  memset(&f, 0, sizeof f);
  f.P = P;  // P64 is unused by the FP32 kernels
  f.out = out;
  f.tile_begin = 0;
  set_tiles(f, s.tile_w, s.tile_h);
  uint32_t *counter = nullptr;
  hipError_t e = launch_counter(fixed, stream, &counter);
  if (e != hipSuccess) return e;
  return launch_render_refill(f, counter, s, cus, stream);
}

hipError_t launch_render_fp32(const KParams &P, const KOut &out, const Sched &s, int cus,
                              hipStream_t stream) {
  return launch_render_fp32_at(P, out, s, cus, nullptr, stream);
}

// One frame. fixed: base of the fixed scratch (dqj_render_noalloc), or null to use
// the stream's own blocks.
static dqj_status render_impl(const dqj_params *params, const dqj_frame_out *out,
                              const dqj_schedule *sched, hipStream_t stream, void *fixed = nullptr) {
  dqj_status s = validate_params(params);
  if (s != DQJ_OK) return s;
  s = check_render_modes(*params, true);
  if (s != DQJ_OK) return s;
  s = validate_out(out);
  if (s != DQJ_OK) return s;
  s = check_schedule(sched);
  if (s != DQJ_OK) return s;
  int cus = 0;
  s = current_device(nullptr, &cus);
  if (s != DQJ_OK) return s;
  KParams kp;
  pack_params(*params, kp);
  const KOut ko = to_kout(*out);
  hipError_t e;
  if (params->march == DQJ_MARCH_DE) {
    if (params->precision != DQJ_PREC_FP32)
      return fail(DQJ_E_UNSUPPORTED, "the distance-estimate march runs in FP32 only");
    // The one-thread-per-pixel kernel is the default here: DE march points escape after
    // a few updates, so the refill kernel's per-point estimate and restart run on nearly
    // every trip; the persistent form is taken only when asked for.
    const Sched sc = resolve_schedule(sched, cus);
    if (sched && sched->kernel == DQJ_KERNEL_LOCKSTEP) {
      FrameDesc f;
      memset(&f, 0, sizeof f);
      f.P = kp;
      f.out = ko;
      f.tile_begin = 0;
      set_tiles(f, sc.tile_w, sc.tile_h);
      uint32_t *counter = nullptr;
      e = launch_counter(fixed, stream, &counter);
      if (e == hipSuccess) e = launch_render_de_lockstep(f, counter, sc, cus, stream);
    } else if (!sched || sched->kernel != DQJ_KERNEL_REFILL) {
      e = launch_render_de(kp, ko, (sched && sched->waves_per_block) ? sched->waves_per_block : 1,
                           stream);
    } else {
      FrameDesc f;
      memset(&f, 0, sizeof f);
      f.P = kp;
      f.out = ko;
      f.tile_begin = 0;
      set_tiles(f, sc.tile_w, sc.tile_h);
      uint32_t *counter = nullptr;
      e = launch_counter(fixed, stream, &counter);
      if (e == hipSuccess) e = launch_render_de_refill(f, counter, sc, cus, stream);
    }
    if (e == hipSuccess && kp.normal_mode != 0) e = launch_neighbour_normal(kp, ko, stream);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return DQJ_OK;
  }
  if (sched && sched->kernel == DQJ_KERNEL_LOCKSTEP)
    return fail(DQJ_E_UNSUPPORTED, "the lock-step kernel runs the distance-estimate march only");
  if (params->fiber_count > 0) {
    FiberTable fb;
    memset(&fb, 0, sizeof fb);
    for (int f = 0; f < params->fiber_count; ++f)
      for (int q = 0; q < 8; ++q) fb.off[f][q] = (float)params->fiber[8 * f + q];
    e = launch_render_project(kp, fb, params->fiber_count, ko, stream);
    if (e == hipSuccess && kp.normal_mode != 0) e = launch_neighbour_normal(kp, ko, stream);
    if (e != hipSuccess) return hip_fail(e, "render launch");
    return DQJ_OK;
  }
  switch (params->precision) {
    case DQJ_PREC_FP32:
      e = launch_render_fp32_at(kp, ko, pick_schedule(sched, *params, cus), cus, fixed, stream);
      break;
    case DQJ_PREC_SPLIT: {
      const Sched s = pick_schedule(sched, *params, cus);
      FrameDesc f;
      memset(&f, 0, sizeof f);
      f.P = kp;
      pack_params64(*params, f.P64);
      f.out = ko;
      f.tile_begin = 0;
      set_tiles(f, s.tile_w, s.tile_h);
      const uint64_t pixels = (uint64_t)params->width * (uint64_t)params->height;
      void *lists = fixed;
      if (fixed) {
        if (pixels > DQJ_NOALLOC_MAX_SPLIT_PIXELS)
          return fail(DQJ_E_INVALID,
                      "dqj_render_noalloc: a split frame of %llu pixels needs %zu bytes of scratch; "
                      "the fixed scratch holds %u (at most %u pixels)",
                      (unsigned long long)pixels, split_scratch_bytes(pixels),
                      (unsigned)DQJ_NOALLOC_SCRATCH_BYTES, (unsigned)DQJ_NOALLOC_MAX_SPLIT_PIXELS);
      } else {
        e = stream_scratch(stream, split_scratch_bytes(pixels), &lists);
        if (e != hipSuccess) return fail(DQJ_E_NOMEM, "split scratch: %s", hipGetErrorString(e));
      }
      e = launch_render_split(f, split_scratch_at(lists, pixels), s, cus, stream);
      break;
    }
    default:
      return fail(DQJ_E_UNSUPPORTED, "precision %d is not offered by dqj_render",
                  params->precision);
  }
  if (e == hipSuccess && kp.normal_mode != 0) e = launch_neighbour_normal(kp, ko, stream);
  if (e != hipSuccess) return hip_fail(e, "render launch");
  return DQJ_OK;
}

}  // namespace dqj

using namespace dqj;

#define DQJ_GUARD(body)                                              \
  try {                                                              \
    body                                                             \
  } catch (const std::bad_alloc &) {                                 \
    return fail(DQJ_E_NOMEM, "host allocation failed");              \
  } catch (...) {                                                    \
    return fail(DQJ_E_DEVICE, "unexpected internal error");          \
  }

extern "C" {

dqj_status dqj_render(const dqj_params *params, const dqj_frame_out *out, void *hip_stream) {
  DQJ_GUARD(return render_impl(params, out, nullptr, (hipStream_t)hip_stream);)
}

dqj_status dqj_render_noalloc(const dqj_params *params, const dqj_frame_out *out, void *hip_stream) {
  DQJ_GUARD({
    void *fixed = nullptr;
    const hipError_t e = fixed_scratch(&fixed);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the fixed scratch");
    return render_impl(params, out, nullptr, (hipStream_t)hip_stream, fixed);
  })
}

dqj_status dqj_render_scheduled(const dqj_params *params, const dqj_frame_out *out,
                                const dqj_schedule *sched, void *hip_stream) {
  DQJ_GUARD(return render_impl(params, out, sched, (hipStream_t)hip_stream);)
}

dqj_status dqj_classify_points(const void *pts_dev, int32_t n, int32_t precision,
                               const dqj_params *params, int32_t *escape_iter_dev,
                               float *final_norm2_dev, void *hip_stream) {
  DQJ_GUARD({
    dqj_status s = validate_params(params);
    if (s != DQJ_OK) return s;
    if (params->algebra != DQJ_ALGEBRA_DUAL)
      return fail(DQJ_E_UNSUPPORTED, "the component-wise algebra is offered by dqj_classify_grid only");
    if (n < 0) return fail(DQJ_E_INVALID, "n must be >= 0");
    if (n > 0 && (!pts_dev || !escape_iter_dev))
      return fail(DQJ_E_INVALID, "points and escape_iter are required");
    s = current_device(nullptr, nullptr);
    if (s != DQJ_OK) return s;
    hipError_t e;
    if (precision == DQJ_PREC_FP32) {
      KParams kp;
      pack_params(*params, kp);
      e = launch_classify_f32((const float *)pts_dev, n, kp, escape_iter_dev, final_norm2_dev,
                              (hipStream_t)hip_stream);
    } else if (precision == DQJ_PREC_FP64) {
      KIter64 k;
      for (int i = 0; i < 8; ++i) k.c[i] = params->c[i];
      k.R2 = params->escape_radius * params->escape_radius;
      k.N = params->max_iter;
      k.norm = params->norm;
      e = launch_classify_f64((const double *)pts_dev, n, k, escape_iter_dev, final_norm2_dev,
                              (hipStream_t)hip_stream);
    } else {
      return fail(DQJ_E_INVALID, "classify precision must be DQJ_PREC_FP32 or DQJ_PREC_FP64");
    }
    if (e != hipSuccess) return hip_fail(e, "classify launch");
    return DQJ_OK;
  })
}

dqj_status dqj_device_info_get(int32_t device, dqj_device_info *out) {
  DQJ_GUARD({
    if (!out || out->struct_size != sizeof(dqj_device_info))
      return fail(DQJ_E_INVALID, "out is NULL or has the wrong struct_size");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(DQJ_E_INVALID, "no device %d", device);
    const DevInfo *d = probe_device(device);
    snprintf(out->arch, sizeof out->arch, "%s", d->arch);
    out->compute_units = d->cus;
    out->clock_khz = d->clock_khz;
    out->memory_clock_khz = d->mem_clock_khz;
    out->total_mem_bytes = d->total_mem;
    const double ghz = d->clock_khz * 1e-6;
    out->fp32_vector_peak_tflops = 256.0 * d->cus * ghz * 1e-3;
    out->fp32_unpacked_peak_tflops = 128.0 * d->cus * ghz * 1e-3;
    if (!d->gfx950) return fail(DQJ_E_UNSUPPORTED, "device %d is '%s', not gfx950", device, d->arch);
    return DQJ_OK;
  })
}

const char *dqj_last_error(void) { return t_last_error.c_str(); }

const char *dqj_status_str(dqj_status s) {
  switch (s) {
    case DQJ_OK: return "DQJ_OK";
    case DQJ_PENDING: return "DQJ_PENDING";
    case DQJ_E_INVALID: return "DQJ_E_INVALID";
    case DQJ_E_NOMEM: return "DQJ_E_NOMEM";
    case DQJ_E_BUDGET: return "DQJ_E_BUDGET";
    case DQJ_E_QUEUE_FULL: return "DQJ_E_QUEUE_FULL";
    case DQJ_E_DEVICE: return "DQJ_E_DEVICE";
    case DQJ_E_TIMEOUT: return "DQJ_E_TIMEOUT";
    case DQJ_E_CANCELLED: return "DQJ_E_CANCELLED";
    case DQJ_E_UNSUPPORTED: return "DQJ_E_UNSUPPORTED";
    case DQJ_E_STATE: return "DQJ_E_STATE";
    default: return "DQJ_E_UNKNOWN";
  }
}

}  // extern "C"

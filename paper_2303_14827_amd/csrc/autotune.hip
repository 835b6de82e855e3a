// autotune.hip -- schedule autotuner for the persistent kernels.
//
// A schedule (tile shape, waves per block, blocks per CU) changes speed only: every
// schedule renders bit-identical images. dqj_autotune renders the caller's
// representative frames with each candidate schedule as one batched launch, times
// the launches with HIP events, and keeps the fastest. Results are remembered per
// workload key (image size, max_iter, march and bisection steps, precision, norm,
// slice kind, device) in memory and, if a cache file is given (or DQJ_TUNE_CACHE is
// set), appended to it as JSON lines; batch plans and renders created without an
// explicit schedule use the remembered one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dqj.h"
#include "kparams.h"
#include "runtime_internal.h"

namespace dqj {

namespace {

std::mutex g_tune_mu;
std::map<std::string, Sched> g_tuned;
bool g_file_loaded = false;

std::string key_of(const dqj_params &p, const char *arch) {
  bool axis = true;
  for (int i = 0; i < 8; ++i) {
    axis = axis && p.slice_origin[i] == 0.0 && p.slice_axes[0][i] == (i == 0 ? 1.0 : 0.0) &&
           p.slice_axes[1][i] == (i == 1 ? 1.0 : 0.0) && p.slice_axes[2][i] == (i == 2 ? 1.0 : 0.0);
  }
  char buf[256];
  snprintf(buf, sizeof buf, "W=%d,H=%d,N=%d,S=%d,B=%d,prec=%d,norm=%d,axis=%d,arch=%.6s", p.width,
           p.height, p.max_iter, p.march_steps, p.bisect_steps, p.precision, p.norm, axis ? 1 : 0,
           arch);
  return buf;
}

const char *cache_env() {
  const char *e = getenv("DQJ_TUNE_CACHE");
  return (e && *e) ? e : nullptr;
}

// Reads lines {"key": "...", "tile_w": a, "tile_h": b, "waves_per_block": c, "blocks_per_cu": d, ...}
void load_file(const char *path) {
  FILE *f = fopen(path, "r");
  if (!f) return;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    char key[256];
    Sched s;
    s.kernel = DQJ_KERNEL_REFILL;
    const char *k = strstr(line, "\"key\": \"");
    if (!k) continue;
    k += 8;
    const char *e = strchr(k, '"');
    if (!e || e - k >= (long)sizeof key) continue;
    memcpy(key, k, e - k);
    key[e - k] = 0;
    auto num = [&](const char *name, int *out) {
      const char *q = strstr(line, name);
      if (!q) return false;
      return sscanf(q + strlen(name), "%d", out) == 1;
    };
    if (num("\"tile_w\": ", &s.tile_w) && num("\"tile_h\": ", &s.tile_h) &&
        num("\"waves_per_block\": ", &s.waves_per_block) &&
        num("\"blocks_per_cu\": ", &s.blocks_per_cu))
      g_tuned[key] = s;   // later lines win
  }
  fclose(f);
}

void ensure_loaded() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  if (const char *p = cache_env()) load_file(p);
}

}  // namespace

bool tuned_schedule(const dqj_params &p, Sched *out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  ensure_loaded();
  auto it = g_tuned.find(key_of(p, prop.gcnArchName));
  if (it == g_tuned.end()) return false;
  *out = it->second;
  return true;
}

}  // namespace dqj

using namespace dqj;

extern "C" dqj_status dqj_autotune(const dqj_params *params, const dqj_frame_out *outs, int32_t n,
                                   const char *cache_path, dqj_schedule *best) {
  try {
    if (n < 1 || !params || !outs) return fail(DQJ_E_INVALID, "autotune needs n >= 1 frames");
    if (best && best->struct_size != sizeof(dqj_schedule))
      return fail(DQJ_E_INVALID, "best.struct_size must be sizeof(dqj_schedule)");
    int dev = 0, cus = 0;
    dqj_status st = current_device(&dev, &cus);
    if (st != DQJ_OK) return st;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    for (int32_t i = 0; i < n; ++i) {
      st = validate_params(params + i);
      if (st != DQJ_OK) return st;
      st = check_render_modes(params[i], false);
      if (st != DQJ_OK) return st;
      st = validate_out(outs + i);
      if (st != DQJ_OK) return st;
    }
    struct Cand {
      int tw, th, wpb, bpc;
    };
    const Cand cands[] = {{8, 8, 4, 8},   {8, 8, 4, 4},   {16, 8, 4, 8},  {16, 16, 4, 8},
                          {16, 16, 4, 4}, {32, 16, 4, 8}, {32, 32, 4, 8}, {8, 8, 2, 16},
                          {16, 16, 8, 4}, {64, 16, 4, 8}};
    // timed without update counters: the kernel renders without one use
    std::vector<dqj_frame_out> touts(outs, outs + n);
    for (dqj_frame_out &o : touts) o.iters = nullptr;
    hipStream_t stream = nullptr;
    e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    (void)hipEventCreate(&ev0);
    (void)hipEventCreate(&ev1);
    float best_ms = 1e30f;
    Cand win = cands[0];
    for (const Cand &c : cands) {
      dqj_schedule sc;
      memset(&sc, 0, sizeof sc);
      sc.struct_size = sizeof sc;
      sc.kernel = DQJ_KERNEL_REFILL;
      sc.tile_w = c.tw;
      sc.tile_h = c.th;
      sc.waves_per_block = c.wpb;
      sc.blocks_per_cu = c.bpc;
      dqj_batch_plan *plan = nullptr;
      st = dqj_batch_plan_create(params, touts.data(), n, &sc, stream, &plan);
      if (st != DQJ_OK) break;
      float ms = 1e30f;
      for (int rep = 0; rep < 3 && st == DQJ_OK; ++rep) {   // first replay warms up
        (void)hipEventRecord(ev0, stream);
        st = dqj_batch_plan_launch(plan, stream);
        (void)hipEventRecord(ev1, stream);
        if (hipEventSynchronize(ev1) != hipSuccess) st = fail(DQJ_E_DEVICE, "autotune launch failed");
        float t = 0;
        (void)hipEventElapsedTime(&t, ev0, ev1);
        if (rep > 0) ms = std::min(ms, t);
      }
      dqj_batch_plan_destroy(plan);
      if (st != DQJ_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        win = c;
      }
    }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    (void)hipStreamDestroy(stream);
    if (st != DQJ_OK) return st;
    Sched s;
    s.kernel = DQJ_KERNEL_REFILL;
    s.tile_w = win.tw;
    s.tile_h = win.th;
    s.waves_per_block = win.wpb;
    s.blocks_per_cu = win.bpc;
    const std::string key = key_of(params[0], prop.gcnArchName);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      ensure_loaded();
      g_tuned[key] = s;
    }
    const char *path = cache_path && *cache_path ? cache_path : cache_env();
    if (path) {
      FILE *f = fopen(path, "a");
      if (f) {
        fprintf(f,
                "{\"key\": \"%s\", \"tile_w\": %d, \"tile_h\": %d, \"waves_per_block\": %d, "
                "\"blocks_per_cu\": %d, \"ms\": %.4f, \"frames\": %d}\n",
                key.c_str(), s.tile_w, s.tile_h, s.waves_per_block, s.blocks_per_cu, best_ms, n);
        fclose(f);
      }
    }
    if (best) {
      best->kernel = DQJ_KERNEL_REFILL;
      best->tile_w = s.tile_w;
      best->tile_h = s.tile_h;
      best->waves_per_block = s.waves_per_block;
      best->blocks_per_cu = s.blocks_per_cu;
    }
    return DQJ_OK;
  } catch (...) {
    return fail(DQJ_E_DEVICE, "unexpected internal error");
  }
}

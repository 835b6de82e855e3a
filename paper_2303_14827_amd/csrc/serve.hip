// serve.hip -- the render server: HIP side of continuous batching.
//
// The scheduling decisions live in serve_core (plain C++). This file owns the device
// side: `slots` epoch slots, each with its own stream, device table + launch header,
// device scratch, pinned staging buffer and a HIP graph captured once at creation
// (reset + the persistent kernels, which read the epoch's size from the header). A
// scheduler thread admits requests, builds an epoch from chunks of every active
// request whenever a slot is free, uploads the epoch's table into the slot and
// replays the slot's graph, and retires epochs by polling their completion events.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dqj.h"
#include "kparams.h"
#include "refill.h"
#include "runtime_internal.h"
#include "serve_core.h"
#include "split.h"

namespace dqj {
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void *dev = nullptr;            // [LaunchHeader | FrameDesc x max_chunks]
  void *scratch = nullptr;        // split lists or the tile counter
  void *staging = nullptr;        // pinned copy of [header | table]
  // one graph per slice mode: general, identity, identity with untested first update
  // one per launch mode: slice mode (0-2), plus 3 with kModeWide
  hipGraph_t graph[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool busy = false;
  uint64_t epoch = 0;
};

struct Record {
  FrameDesc frame;   // full-frame descriptor; chunks copy it with their tile range
};

uint64_t resident_bytes_of(const dqj_frame_out &o, uint64_t pixels) {
  uint64_t per = 0;
  per += o.mask ? 1 : 0;
  per += o.depth ? 4 : 0;
  per += o.shade ? 4 : 0;
  per += o.image8 ? 1 : 0;
  per += o.normal ? 12 : 0;
  per += o.first_hit ? 4 : 0;
  per += o.flags ? 1 : 0;
  return per * pixels;
}

}  // namespace
}  // namespace dqj

using namespace dqj;

struct dqj_server {
  serve::Core core;
  std::mutex mu;
  std::condition_variable cv_sched, cv_done;
  std::thread thread;
  bool stop = false;
  bool closing = false;
  int dev = 0, cus = 0;
  int precision = DQJ_PREC_FP32, norm = 0;
  bool count = false;
  Sched sched;
  int max_chunks = 256;
  uint64_t epoch_pixels = 4u << 20;
  std::vector<Slot> slots;
  std::unordered_map<uint64_t, Record> recs;

  explicit dqj_server(const serve::CoreConfig &c) : core(c) {}
};

namespace {

size_t slot_dev_bytes(int max_chunks) {
  return sizeof(LaunchHeader) + sizeof(FrameDesc) * (size_t)max_chunks;
}

void free_slots(dqj_server *s) {
  for (Slot &sl : s->slots) {
    if (sl.busy && sl.done) (void)hipEventSynchronize(sl.done);
    for (int a = 0; a < 6; ++a) {
      if (sl.exec[a]) (void)hipGraphExecDestroy(sl.exec[a]);
      if (sl.graph[a]) (void)hipGraphDestroy(sl.graph[a]);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.scratch) (void)hipFree(sl.scratch);
    if (sl.staging) (void)hipHostFree(sl.staging);
  }
  s->slots.clear();
}

// Capture the slot's graphs (one per launch mode: slice mode a % 3, with kModeWide from
// a = 3 on): a counter/list reset and the persistent kernels, which take the epoch's size
// from the header in device memory. (The split-precision march has no untested-first-
// update form and one stencil sum: its graphs repeat.)
hipError_t capture_slot(dqj_server *s, Slot &sl) {
  const LaunchHeader *hdr = (const LaunchHeader *)sl.dev;
  const FrameDesc *table = (const FrameDesc *)((char *)sl.dev + sizeof(LaunchHeader));
  for (int a = 0; a < 6; ++a) {
    const int mode = (a % 3) | (a >= 3 ? kModeWide : 0);
    hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le;
    if (s->precision == DQJ_PREC_SPLIT)
      le = launch_render_split_batch(table, hdr, 0, 0, s->norm, a % 3 >= 1, s->count,
                                     split_scratch_at(sl.scratch, s->epoch_pixels), s->sched,
                                     s->cus, sl.stream);
    else
      le = launch_render_refill_batch(table, hdr, 0, 0, s->norm, mode, s->count,
                                      (uint32_t *)sl.scratch, s->sched, s->cus, sl.stream);
    e = hipStreamEndCapture(sl.stream, &sl.graph[a]);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&sl.exec[a], sl.graph[a], nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Upload one epoch into a free slot and replay its graph. Caller holds s->mu.
hipError_t launch_epoch(dqj_server *s, Slot &sl, const serve::Epoch &ep) {
  LaunchHeader *h = (LaunchHeader *)sl.staging;
  FrameDesc *tab = (FrameDesc *)((char *)sl.staging + sizeof(LaunchHeader));
  memset(h, 0, sizeof *h);
  uint32_t tile = 0;
  int mode = kSliceIdentitySticky;
  for (size_t i = 0; i < ep.chunks.size(); ++i) {
    const serve::Chunk &c = ep.chunks[i];
    FrameDesc f = s->recs.at(c.ticket).frame;
    f.tile_begin = tile;
    f.tile_offset = c.tile_begin;
    f.ntiles = c.ntiles;
    tab[i] = f;
    tile += c.ntiles;
    mode = combine_slice_mode(mode, slice_mode_of(f.P));
  }
  h->nframes = (uint32_t)ep.chunks.size();
  h->total_tiles = tile;
  const size_t bytes = sizeof(LaunchHeader) + sizeof(FrameDesc) * ep.chunks.size();
  hipError_t e = hipMemcpyAsync(sl.dev, sl.staging, bytes, hipMemcpyHostToDevice, sl.stream);
  const int g = (mode & kSliceMask) + ((mode & kModeWide) ? 3 : 0);
  if (e == hipSuccess) e = hipGraphLaunch(sl.exec[g], sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e == hipSuccess) {
    sl.busy = true;
    sl.epoch = ep.id;
  }
  return e;
}

void scheduler_loop(dqj_server *s) {
  (void)hipSetDevice(s->dev);
  std::unique_lock<std::mutex> lk(s->mu);
  std::vector<uint64_t> finished;
  while (true) {
    bool progressed = false;
    const double t = now_s();
    s->core.admit(t);
    // retire finished epochs
    for (Slot &sl : s->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      sl.busy = false;
      s->core.finish_epoch(sl.epoch, q == hipSuccess, now_s(), &finished);
      progressed = true;
    }
    // launch new epochs into free slots
    for (Slot &sl : s->slots) {
      if (sl.busy || s->stop) continue;
      serve::Epoch ep;
      if (!s->core.build_epoch(now_s(), &ep)) break;
      if (launch_epoch(s, sl, ep) != hipSuccess) {
        s->core.finish_epoch(ep.id, false, now_s(), &finished);
      }
      progressed = true;
    }
    if (!finished.empty()) {
      finished.clear();
      s->cv_done.notify_all();
    }
    bool any_busy = false;
    for (const Slot &sl : s->slots) any_busy = any_busy || sl.busy;
    if (s->stop && !any_busy) break;
    if (progressed) continue;
    if (any_busy)
      s->cv_sched.wait_for(lk, std::chrono::microseconds(50));
    else
      s->cv_sched.wait(lk, [&] { return s->stop || s->core.has_unassigned() ||
                                        s->core.pending_count() > 0; });
  }
  s->cv_done.notify_all();
}

void fill_result(const serve::RequestInfo &r, dqj_request_result *res) {
  if (!res || res->struct_size != sizeof(dqj_request_result)) return;
  res->status = r.status;
  res->t_submit = r.t_submit;
  res->t_admit = r.t_admit;
  res->t_first_launch = r.t_first_launch;
  res->t_done = r.t_done;
  res->chunks = r.chunks;
}

bool final_state(const serve::RequestInfo &r) {
  return r.state == serve::State::Done || r.state == serve::State::Cancelled ||
         r.state == serve::State::Failed;
}

}  // namespace

extern "C" {

dqj_status dqj_serve_create(const dqj_serve_config *cfg, dqj_server **out) {
  if (!out) return fail(DQJ_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg || cfg->struct_size != sizeof(dqj_serve_config))
    return fail(DQJ_E_INVALID, "config is NULL or has the wrong struct_size");
  if (cfg->precision != DQJ_PREC_FP32 && cfg->precision != DQJ_PREC_SPLIT)
    return fail(DQJ_E_UNSUPPORTED, "the server renders in FP32 or split precision");
  if (cfg->norm != DQJ_NORM_EUCLID8 && cfg->norm != DQJ_NORM_REALPART)
    return fail(DQJ_E_INVALID, "norm must be one of DQJ_NORM_*");
  if (cfg->slots < 0 || cfg->slots > 8) return fail(DQJ_E_INVALID, "slots must be in 0..8");
  if (cfg->max_inflight < 0 || cfg->max_pending < 0 || cfg->epoch_pixels < 0 ||
      !(cfg->epoch_work >= 0))
    return fail(DQJ_E_INVALID, "negative limits in the server config");
  if (cfg->policy != DQJ_SERVE_FAIR && cfg->policy != DQJ_SERVE_OLDEST)
    return fail(DQJ_E_INVALID, "policy must be one of DQJ_SERVE_*");
  if (cfg->sched.struct_size != 0 && cfg->sched.struct_size != sizeof(dqj_schedule))
    return fail(DQJ_E_INVALID, "config.sched.struct_size must be 0 or sizeof(dqj_schedule)");
  int dev = 0, cus = 0;
  dqj_status st = current_device(&dev, &cus);
  if (st != DQJ_OK) return st;
  serve::CoreConfig cc;
  if (cfg->hbm_budget_bytes) cc.budget_bytes = cfg->hbm_budget_bytes;
  if (cfg->max_inflight) cc.max_inflight = cfg->max_inflight;
  if (cfg->max_pending) cc.max_pending = cfg->max_pending;
  if (cfg->epoch_pixels) cc.epoch_pixels = (uint64_t)cfg->epoch_pixels;
  if (cfg->epoch_work > 0) cc.epoch_work = cfg->epoch_work;
  cc.oldest_first = cfg->policy == DQJ_SERVE_OLDEST;
  dqj_server *s = nullptr;
  try {
    s = new dqj_server(cc);
  } catch (...) {
    return fail(DQJ_E_NOMEM, "host allocation failed");
  }
  s->dev = dev;
  s->cus = cus;
  s->precision = cfg->precision;
  s->norm = cfg->norm;
  s->count = cfg->count_iters != 0;
  s->sched = resolve_schedule(cfg->sched.struct_size ? &cfg->sched : nullptr, cus);
  s->max_chunks = cc.max_chunks;
  s->epoch_pixels = cc.epoch_pixels;
  const int nslots = cfg->slots ? cfg->slots : 3;
  hipError_t e = hipSuccess;
  s->slots.resize(nslots);
  for (Slot &sl : s->slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&sl.dev, slot_dev_bytes(s->max_chunks));
    if (e == hipSuccess)
      e = hipMalloc(&sl.scratch, s->precision == DQJ_PREC_SPLIT ? split_scratch_bytes(s->epoch_pixels)
                                                                : 256);
    if (e == hipSuccess) e = hipHostMalloc(&sl.staging, slot_dev_bytes(s->max_chunks), hipHostMallocDefault);
    if (e == hipSuccess) e = capture_slot(s, sl);
  }
  if (e != hipSuccess) {
    free_slots(s);
    delete s;
    return hip_fail(e, "server creation");
  }
  s->thread = std::thread(scheduler_loop, s);
  *out = s;
  return DQJ_OK;
}

dqj_status dqj_serve_submit(dqj_server *s, const dqj_params *params, const dqj_frame_out *out,
                            uint64_t *ticket) {
  if (!s || !ticket) return fail(DQJ_E_INVALID, "server and ticket are required");
  dqj_status st = validate_params(params);
  if (st != DQJ_OK) return st;
  st = check_render_modes(*params, false);
  if (st != DQJ_OK) return st;
  st = validate_out(out);
  if (st != DQJ_OK) return st;
  if (params->precision != s->precision)
    return fail(DQJ_E_INVALID, "request precision %d differs from the server's %d",
                params->precision, s->precision);
  if (params->norm != s->norm)
    return fail(DQJ_E_INVALID, "request norm differs from the server's");
  if (params->march != DQJ_MARCH_FIXED)
    return fail(DQJ_E_UNSUPPORTED, "the server runs the fixed-step march");
  Record rec;
  memset(&rec.frame, 0, sizeof rec.frame);
  pack_params(*params, rec.frame.P);
  pack_params64(*params, rec.frame.P64);
  rec.frame.out = to_kout(*out);
  set_tiles(rec.frame, s->sched.tile_w, s->sched.tile_h);
  const uint64_t pixels = (uint64_t)params->width * (uint64_t)params->height;
  serve::RequestSpec spec;
  spec.resident_bytes = resident_bytes_of(*out, pixels);
  spec.tiles = rec.frame.ntiles;
  spec.tile_pixels = (uint32_t)(s->sched.tile_w * s->sched.tile_h);
  // ~3 updates per march sample on average, plus bisection and normal on hits
  spec.work_per_tile = (double)spec.tile_pixels * 3.0 * (double)(params->march_steps + 1);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->closing) return fail(DQJ_E_STATE, "server is shutting down");
  uint64_t t = 0;
  const int32_t r = s->core.submit(spec, now_s(), &t);
  if (r == serve::kBudget)
    return fail(DQJ_E_BUDGET, "request needs %llu resident bytes, above the server budget",
                (unsigned long long)spec.resident_bytes);
  if (r == serve::kQueueFull) return fail(DQJ_E_QUEUE_FULL, "pending queue is full");
  if (r != serve::kOk) return fail(DQJ_E_INVALID, "request rejected by the scheduler");
  s->recs.emplace(t, rec);
  *ticket = t;
  s->cv_sched.notify_one();
  return DQJ_OK;
}

dqj_status dqj_serve_poll(dqj_server *s, uint64_t ticket, dqj_request_result *res) {
  if (!s) return fail(DQJ_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  const serve::RequestInfo *r = s->core.info(ticket);
  if (!r) return fail(DQJ_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  fill_result(*r, res);
  return final_state(*r) ? r->status : DQJ_PENDING;
}

dqj_status dqj_serve_wait(dqj_server *s, uint64_t ticket, int32_t timeout_ms,
                          dqj_request_result *res) {
  if (!s) return fail(DQJ_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  const serve::RequestInfo *r = s->core.info(ticket);
  if (!r) return fail(DQJ_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  auto is_final = [&] { return final_state(*s->core.info(ticket)); };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, is_final);
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), is_final)) {
    fill_result(*s->core.info(ticket), res);
    return fail(DQJ_E_TIMEOUT, "request %llu not finished within %d ms",
                (unsigned long long)ticket, timeout_ms);
  }
  r = s->core.info(ticket);
  fill_result(*r, res);
  return r->status;
}

dqj_status dqj_serve_cancel(dqj_server *s, uint64_t ticket) {
  if (!s) return fail(DQJ_E_INVALID, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<uint64_t> fin;
  const int32_t r = s->core.cancel(ticket, now_s(), &fin);
  if (!fin.empty()) s->cv_done.notify_all();
  if (r == serve::kInvalid) return fail(DQJ_E_INVALID, "unknown ticket");
  if (r == serve::kState) return fail(DQJ_E_STATE, "request is already final");
  return DQJ_OK;
}

dqj_status dqj_serve_stats_get(dqj_server *s, dqj_serve_stats *out) {
  if (!s || !out || out->struct_size != sizeof(dqj_serve_stats))
    return fail(DQJ_E_INVALID, "server or stats record invalid");
  std::lock_guard<std::mutex> lk(s->mu);
  const serve::CoreStats c = s->core.stats();
  out->submitted = c.submitted;
  out->admitted = c.admitted;
  out->completed = c.completed;
  out->cancelled = c.cancelled;
  out->failed = c.failed;
  out->rejected = c.rejected;
  out->epochs = c.epochs;
  out->pending = c.pending;
  out->active = c.active;
  out->resident_bytes = c.resident_bytes;
  out->p50_latency_s = c.p50;
  out->p99_latency_s = c.p99;
  out->max_latency_s = c.max;
  out->mean_latency_s = c.mean;
  return DQJ_OK;
}

dqj_status dqj_serve_destroy(dqj_server *s) {
  if (!s) return DQJ_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->closing = true;
    // pending requests are cancelled; admitted ones stop taking new tiles
    std::vector<uint64_t> fin;
    for (uint64_t t = 1;; ++t) {
      const serve::RequestInfo *r = s->core.info(t);
      if (!r) break;
      if (!final_state(*r)) s->core.cancel(t, now_s(), &fin);
    }
    s->stop = true;
    s->cv_sched.notify_all();
  }
  if (s->thread.joinable()) s->thread.join();
  free_slots(s);
  delete s;
  return DQJ_OK;
}

}  // extern "C"

// batch.hip -- many frames in one persistent launch: dqj_render_batch (eager) and
// dqj_batch_plan_* (captured once into a HIP graph, replayed).
//
// The frames' parameter records and output pointers sit in a device-resident table
// of FrameDesc; the persistent kernel takes (frame, tile) work items from one global
// counter, so small and large frames, and cheap and expensive ones, share the GPU
// without a launch per frame.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "dqj.h"
#include "kparams.h"
#include "launch.h"
#include "refill.h"
#include "split.h"
#include "project.h"
#include "runtime_internal.h"

namespace dqj {

namespace {

// Host-side validation and packing shared by the eager and the captured batch.
dqj_status pack_batch(const dqj_params *params, const dqj_frame_out *outs, int32_t n,
                      const Sched &s, std::vector<FrameDesc> &table, uint32_t &total_tiles,
                      int &norm, bool &all_axis, int &slice_mode, bool &any_count,
                      int &precision, uint64_t &pixels, std::vector<ProjFiber> &fibers) {
  if (n < 1) return fail(DQJ_E_INVALID, "batch size must be >= 1 (got %d)", n);
  if (!params || !outs) return fail(DQJ_E_INVALID, "params and outs are required");
  table.resize(n);
  fibers.clear();
  uint64_t tiles = 0;
  all_axis = true;
  slice_mode = kSliceIdentitySticky;
  any_count = false;
  pixels = 0;
  for (int32_t i = 0; i < n; ++i) {
    dqj_status st = validate_params(params + i);
    if (st != DQJ_OK) return fail(st, "frame %d: %s", i, dqj_last_error());
    // A batch holds projection frames only, or none: they run a kernel of their own.
    const bool proj = params[i].fiber_count > 0;
    if (i > 0 && proj != (params[0].fiber_count > 0))
      return fail(DQJ_E_INVALID, "frame %d: a batch holds projection frames only, or none", i);
    if (proj) {
      st = check_render_modes(params[i], true);   // FP32, fixed-step march
      if (st == DQJ_OK && params[i].normal_mode == DQJ_NORMAL_NEIGHBOUR4)
        st = fail(DQJ_E_UNSUPPORTED, "the four-neighbour normal is offered by dqj_render only");
    } else {
      st = check_render_modes(params[i], false);
    }
    if (st != DQJ_OK) return fail(st, "frame %d: %s", i, dqj_last_error());
    st = validate_out(outs + i);
    if (st != DQJ_OK) return fail(st, "frame %d: %s", i, dqj_last_error());
    if (i > 0 && params[i].march != params[0].march)
      return fail(DQJ_E_INVALID, "frame %d: all frames of a batch must share the march", i);
    if (params[i].march == DQJ_MARCH_DE && params[i].precision != DQJ_PREC_FP32)
      return fail(DQJ_E_UNSUPPORTED, "frame %d: the distance-estimate march runs in FP32 only", i);
    if (params[i].precision != DQJ_PREC_FP32 && params[i].precision != DQJ_PREC_SPLIT)
      return fail(DQJ_E_UNSUPPORTED, "frame %d: batched renders run in FP32 or split precision", i);
    if (i > 0 && params[i].precision != params[0].precision)
      return fail(DQJ_E_INVALID, "frame %d: all frames of a batch must share precision", i);
    if (i > 0 && params[i].norm != params[0].norm)
      return fail(DQJ_E_INVALID, "frame %d: all frames of a batch must share the escape norm", i);
    FrameDesc &f = table[i];
    memset(&f, 0, sizeof f);
    pack_params(params[i], f.P);
    pack_params64(params[i], f.P64);
    f.out = to_kout(outs[i]);
    if (proj) {
      if (fibers.empty()) fibers.resize(n);
      ProjFiber &pf = fibers[i];
      memset(&pf, 0, sizeof pf);
      pf.F = params[i].fiber_count;
      for (int k = 0; k < pf.F; ++k)
        for (int q = 0; q < 8; ++q) pf.off[k][q] = (float)params[i].fiber[8 * k + q];
    }
    pixels += (uint64_t)params[i].width * (uint64_t)params[i].height;
    f.tile_begin = (uint32_t)tiles;
    set_tiles(f, s.tile_w, s.tile_h);
    tiles += f.ntiles;
    all_axis = all_axis && f.P.axis_slice;
    slice_mode = combine_slice_mode(slice_mode, slice_mode_of(f.P));
    any_count = any_count || f.out.iters != nullptr;
  }
  if (tiles >= (1ull << 31)) return fail(DQJ_E_INVALID, "batch has too many tiles (%llu)",
                                         (unsigned long long)tiles);
  total_tiles = (uint32_t)tiles;
  norm = params[0].norm;
  precision = params[0].precision;
  return DQJ_OK;
}

// A batch of distance-estimate frames: one one-thread-per-pixel launch over the table.
hipError_t launch_de_table(const FrameDesc *dev, const std::vector<FrameDesc> &table, int norm,
                           bool all_axis, hipStream_t s) {
  int mw = 0, mh = 0;
  bool count = false;
  for (const FrameDesc &f : table) {
    mw = f.P.W > mw ? f.P.W : mw;
    mh = f.P.H > mh ? f.P.H : mh;
    count = count || f.out.iters != nullptr;
  }
  return launch_render_de_batch(dev, (int)table.size(), mw, mh, norm, all_axis, count, s);
}

// A batch of projection frames: their fibre records follow the FrameDesc table in `dev`.
hipError_t launch_project_table(const FrameDesc *dev, const std::vector<FrameDesc> &table,
                                const std::vector<ProjFiber> &fibers, int norm, uint64_t pixels,
                                hipStream_t s) {
  int mw = 0, mh = 0, min_f = kMaxFiber;
  bool count = false;
  for (size_t i = 0; i < table.size(); ++i) {
    mw = table[i].P.W > mw ? table[i].P.W : mw;
    mh = table[i].P.H > mh ? table[i].P.H : mh;
    min_f = fibers[i].F < min_f ? fibers[i].F : min_f;
    count = count || table[i].out.iters != nullptr;
  }
  const ProjFiber *fdev = (const ProjFiber *)((const char *)dev + sizeof(FrameDesc) * table.size());
  return launch_render_project_batch(dev, fdev, (int)table.size(), mw, mh, norm, count, pixels, min_f, s);
}

// Allocations an eager batch leaves behind until the stream has passed them.
struct Retired {
  hipEvent_t ev;
  void *dev;
  void *host;
};
std::mutex g_ret_mu;
std::vector<Retired> g_retired;

void reap_retired(bool wait) {
  std::lock_guard<std::mutex> lk(g_ret_mu);
  size_t w = 0;
  for (size_t i = 0; i < g_retired.size(); ++i) {
    Retired &r = g_retired[i];
    const hipError_t q = wait ? hipEventSynchronize(r.ev) : hipEventQuery(r.ev);
    if (q == hipSuccess) {
      (void)hipFree(r.dev);
      (void)hipHostFree(r.host);
      (void)hipEventDestroy(r.ev);
    } else {
      g_retired[w++] = r;
    }
  }
  g_retired.resize(w);
}

}  // namespace

}  // namespace dqj

using namespace dqj;

struct dqj_batch_plan {
  int dev = 0;
  FrameDesc *table_dev = nullptr;
  uint32_t *counter_dev = nullptr;
  void *split_scratch = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool launched = false;
};

static void plan_free(dqj_batch_plan *p) {
  if (!p) return;
  if (p->done && p->launched) (void)hipEventSynchronize(p->done);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->done) (void)hipEventDestroy(p->done);
  if (p->table_dev) (void)hipFree(p->table_dev);
  if (p->counter_dev) (void)hipFree(p->counter_dev);
  if (p->split_scratch) (void)hipFree(p->split_scratch);
  delete p;
}

extern "C" {

dqj_status dqj_render_batch(const dqj_params *params, const dqj_frame_out *outs, int32_t n,
                            void *hip_stream) {
  try {
    int cus = 0;
    dqj_status st = current_device(nullptr, &cus);
    if (st != DQJ_OK) return st;
    if (n < 1 || !params) return fail(DQJ_E_INVALID, "batch size must be >= 1 with params");
    const Sched s = pick_schedule(nullptr, params[0], cus);
    std::vector<FrameDesc> table;
    uint32_t total = 0;
    int norm = 0;
    bool all_axis = true, any_count = false;
    int slice_mode = kSliceGeneral;
    int precision = 0;
    uint64_t pixels = 0;
    std::vector<ProjFiber> fibers;
    st = pack_batch(params, outs, n, s, table, total, norm, all_axis, slice_mode, any_count, precision,
                    pixels, fibers);
    if (st != DQJ_OK) return st;
    reap_retired(false);
    hipStream_t stream = (hipStream_t)hip_stream;
    const size_t tbytes = sizeof(FrameDesc) * table.size();
    const size_t bytes = tbytes + sizeof(ProjFiber) * fibers.size();
    Retired r{nullptr, nullptr, nullptr};
    hipError_t e = hipHostMalloc(&r.host, bytes, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
    memcpy(r.host, table.data(), tbytes);
    if (!fibers.empty()) memcpy((char *)r.host + tbytes, fibers.data(), bytes - tbytes);
    e = hipMalloc(&r.dev, bytes);
    if (e != hipSuccess) {
      (void)hipHostFree(r.host);
      return fail(DQJ_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    e = hipMemcpyAsync(r.dev, r.host, bytes, hipMemcpyHostToDevice, stream);
    if (!fibers.empty()) {
      if (e == hipSuccess)
        e = launch_project_table((const FrameDesc *)r.dev, table, fibers, norm, pixels, stream);
    } else if (table[0].P.march == DQJ_MARCH_DE) {
      if (e == hipSuccess) e = launch_de_table((const FrameDesc *)r.dev, table, norm, all_axis, stream);
    } else if (precision == DQJ_PREC_FP32) {
      uint32_t *counter = nullptr;
      if (e == hipSuccess) e = stream_counter(stream, &counter);
      if (e == hipSuccess)
        e = launch_render_refill_batch((const FrameDesc *)r.dev, nullptr, n, total, norm, slice_mode,
                                       any_count, counter, s, cus, stream);
    } else {
      void *scratch = nullptr;
      if (e == hipSuccess) e = stream_scratch(stream, split_scratch_bytes(pixels), &scratch);
      if (e == hipSuccess)
        e = launch_render_split_batch((const FrameDesc *)r.dev, nullptr, n, total, norm, all_axis, any_count,
                                      split_scratch_at(scratch, pixels), s, cus, stream);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r.ev, stream);
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(stream);
      (void)hipFree(r.dev);
      (void)hipHostFree(r.host);
      if (r.ev) (void)hipEventDestroy(r.ev);
      return hip_fail(e, "batch launch");
    }
    std::lock_guard<std::mutex> lk(g_ret_mu);
    g_retired.push_back(r);
    return DQJ_OK;
  } catch (const std::bad_alloc &) {
    return fail(DQJ_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(DQJ_E_DEVICE, "unexpected internal error");
  }
}

dqj_status dqj_batch_plan_create(const dqj_params *params, const dqj_frame_out *outs, int32_t n,
                                 const dqj_schedule *sched, void *hip_stream,
                                 dqj_batch_plan **plan) {
  (void)hip_stream;
  if (!plan) return fail(DQJ_E_INVALID, "plan is NULL");
  *plan = nullptr;
  dqj_batch_plan *p = nullptr;
  try {
    int cus = 0, dev = 0;
    dqj_status st = current_device(&dev, &cus);
    if (st != DQJ_OK) return st;
    if (sched && sched->struct_size != sizeof(dqj_schedule))
      return fail(DQJ_E_INVALID, "schedule.struct_size %u != %zu", sched->struct_size,
                  sizeof(dqj_schedule));
    if (n < 1 || !params) return fail(DQJ_E_INVALID, "batch size must be >= 1 with params");
    const Sched s = pick_schedule(sched, params[0], cus);
    if (s.kernel == DQJ_KERNEL_DIRECT || s.kernel == DQJ_KERNEL_LOCKSTEP)
      return fail(DQJ_E_UNSUPPORTED, "batched renders use the refill kernel");
    std::vector<FrameDesc> table;
    uint32_t total = 0;
    int norm = 0;
    bool all_axis = true, any_count = false;
    int slice_mode = kSliceGeneral;
    int precision = 0;
    uint64_t pixels = 0;
    std::vector<ProjFiber> fibers;
    st = pack_batch(params, outs, n, s, table, total, norm, all_axis, slice_mode, any_count, precision,
                    pixels, fibers);
    if (st != DQJ_OK) return st;
    p = new dqj_batch_plan;
    p->dev = dev;
    const size_t tbytes = sizeof(FrameDesc) * table.size();
    const size_t bytes = tbytes + sizeof(ProjFiber) * fibers.size();
    hipError_t e = hipMalloc(&p->table_dev, bytes);
    if (e != hipSuccess) {
      plan_free(p);
      return fail(DQJ_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    e = hipMalloc(&p->counter_dev, 256);
    if (e == hipSuccess && precision == DQJ_PREC_SPLIT)
      e = hipMalloc(&p->split_scratch, split_scratch_bytes(pixels));
    if (e == hipSuccess) e = hipMemcpy(p->table_dev, table.data(), tbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && !fibers.empty())
      e = hipMemcpy((char *)p->table_dev + tbytes, fibers.data(), bytes - tbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      // The capture holds a counter-reset kernel (not a memset node) and the kernel.
      hipError_t le =
          !fibers.empty()
              ? launch_project_table(p->table_dev, table, fibers, norm, pixels, p->cap_stream)
          : table[0].P.march == DQJ_MARCH_DE
              ? launch_de_table(p->table_dev, table, norm, all_axis, p->cap_stream)
          : precision == DQJ_PREC_FP32
              ? launch_render_refill_batch(p->table_dev, nullptr, n, total, norm, slice_mode, any_count,
                                           p->counter_dev, s, cus, p->cap_stream)
              : launch_render_split_batch(p->table_dev, nullptr, n, total, norm, all_axis, any_count,
                                          split_scratch_at(p->split_scratch, pixels), s, cus,
                                          p->cap_stream);
      e = hipStreamEndCapture(p->cap_stream, &p->graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      plan_free(p);
      return hip_fail(e, "batch plan capture");
    }
    *plan = p;
    return DQJ_OK;
  } catch (const std::bad_alloc &) {
    plan_free(p);
    return fail(DQJ_E_NOMEM, "host allocation failed");
  } catch (...) {
    plan_free(p);
    return fail(DQJ_E_DEVICE, "unexpected internal error");
  }
}

dqj_status dqj_batch_plan_launch(dqj_batch_plan *plan, void *hip_stream) {
  if (!plan) return fail(DQJ_E_INVALID, "plan is NULL");
  hipStream_t stream = (hipStream_t)hip_stream;
  hipError_t e = hipGraphLaunch(plan->exec, stream);
  if (e == hipSuccess) e = hipEventRecord(plan->done, stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  plan->launched = true;
  return DQJ_OK;
}

dqj_status dqj_batch_plan_destroy(dqj_batch_plan *plan) {
  if (!plan) return DQJ_OK;
  plan_free(plan);
  return DQJ_OK;
}

}  // extern "C"

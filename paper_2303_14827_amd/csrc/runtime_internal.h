// runtime_internal.h -- host helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "dqj.h"
#include "kparams.h"

namespace dqj {

dqj_status fail(dqj_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
dqj_status hip_fail(hipError_t e, const char *what);
dqj_status current_device(int *dev, int *cus);
dqj_status validate_params(const dqj_params *p);
dqj_status validate_out(const dqj_frame_out *o);
// Modes a render path offers: the component-wise algebra belongs to grid classification
// only; the four-neighbour normal needs the whole frame's depth, so it is offered by
// single-frame renders (single = true) only.
dqj_status check_render_modes(const dqj_params &p, bool single);
void pack_params(const dqj_params &p, KParams &k);
void pack_params64(const dqj_params &p, KParams64 &k);
KOut to_kout(const dqj_frame_out &o);

// Schedule actually used by a launch (defaults and limits applied).
struct Sched {
  int kernel;           // DQJ_KERNEL_REFILL or DQJ_KERNEL_DIRECT
  int tile_w, tile_h;
  int waves_per_block;
  int blocks_per_cu;
};
Sched resolve_schedule(const dqj_schedule *s, int cus);

// Schedule remembered by the autotuner for this workload (false if none).
bool tuned_schedule(const dqj_params &p, Sched *out);

// Explicit schedule if given, else the autotuned one for p, else the defaults.
inline Sched pick_schedule(const dqj_schedule *s, const dqj_params &p, int cus) {
  Sched t;
  if (!s && tuned_schedule(p, &t)) return t;
  return resolve_schedule(s, cus);
}

// FP32 render of one frame with a schedule (s may be null: defaults).
hipError_t launch_render_fp32(const KParams &P, const KOut &out, const Sched &s, int cus,
                              hipStream_t stream);

// Device word private to (current device, stream) for persistent-kernel tile counters.
hipError_t stream_counter(hipStream_t stream, uint32_t **out);

// Device scratch of at least `bytes` private to (current device, stream).
hipError_t stream_scratch(hipStream_t stream, size_t bytes, void **out);

}  // namespace dqj

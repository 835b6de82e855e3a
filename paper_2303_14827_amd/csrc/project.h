// project.h -- batches of projection ("shadow") frames (library-internal).
#pragma once
#include <hip/hip_runtime.h>

#include "kparams.h"
#include "launch.h"

namespace dqj {

// Fibre offsets of one frame of a projection batch, in the device buffer after the
// batch's FrameDesc table (one record per frame, same order).
struct alignas(16) ProjFiber {
  float off[kMaxFiber][8];
  int32_t F;        // offsets in use, 1..kMaxFiber
  int32_t pad[3];
};

// One launch over n projection frames (table_dev: n FrameDesc; fibers_dev: n ProjFiber).
// The lanes per pixel follow the whole batch's pixel count and its smallest F; blocks of
// all frames are interleaved in dispatch order, each frame's taken centre-out. count: some
// frame has an update counter (out.iters).
hipError_t launch_render_project_batch(const FrameDesc *table_dev, const ProjFiber *fibers_dev,
                                       int nframes, int max_w, int max_h, int norm, bool count,
                                       uint64_t pixels, int min_fiber, hipStream_t s);

}  // namespace dqj

// refill.h -- launchers of the persistent refill kernels (library-internal).
#pragma once
#include <hip/hip_runtime.h>

#include "kparams.h"
#include "runtime_internal.h"

namespace dqj {

// One frame; counter is a device word private to the stream (reset by the launch).
hipError_t launch_render_refill(const FrameDesc &frame, uint32_t *counter, const Sched &s, int cus,
                                hipStream_t stream);

// Modes of a launch. Bits 0-1, the slice mode, ordered so that the mode of several
// frames is the minimum of theirs: general slice; identity slice (first march update in
// closed form); identity slice whose escape guarantees let the first update go untested.
// Bit 2, kModeWide: some frame's max_iter exceeds kUnscaledMaxIter, so the normal's
// stencil is summed relative to its least escape index (stencil_add). At or below it the
// stencil's potentials, and the squares of their differences, stay in FP32 range, and
// the kernel sums them as they are, with the more compact code of the hot loop's slow
// path (three 1024^2 frames at max_iter 24: 2.77-2.78 ms against 2.87-2.91 ms).
enum { kSliceGeneral = 0, kSliceIdentity = 1, kSliceIdentitySticky = 2, kSliceMask = 3,
       kModeWide = 4 };
constexpr int kUnscaledMaxIter = 32;
int slice_mode_of(const KParams &P);
int combine_slice_mode(int a, int b);

// n frames from a device-resident table; all frames share norm; slice_mode is the
// combined mode of all frames (for a launch whose table changes between graph replays,
// the least mode any table may have).
// hdr_dev (may be null) overrides nframes/total_tiles with values read on the device.
hipError_t launch_render_refill_batch(const FrameDesc *table_dev, const LaunchHeader *hdr_dev,
                                      int nframes, uint32_t total_tiles, int norm, int slice_mode,
                                      bool any_count, uint32_t *counter, const Sched &s, int cus,
                                      hipStream_t stream);

// Distance-estimate march on the same persistent design: one frame, or n frames of one
// norm from a device table (all_axis: every frame uses the identity slice).
hipError_t launch_render_de_refill(const FrameDesc &frame, uint32_t *counter, const Sched &s, int cus,
                                   hipStream_t stream);
hipError_t launch_render_de_lockstep(const FrameDesc &frame, uint32_t *counter, const Sched &s,
                                     int cus, hipStream_t stream);
hipError_t launch_render_de_refill_batch(const FrameDesc *table_dev, const LaunchHeader *hdr_dev,
                                         int nframes, uint32_t total_tiles, int norm, bool all_axis,
                                         bool any_count, uint32_t *counter, const Sched &s, int cus,
                                         hipStream_t stream);

// Fill the tile geometry of a frame descriptor (tile_begin must be set by the caller).
inline void set_tiles(FrameDesc &f, int tw, int th) {
  f.tiles_x = (uint32_t)((f.P.W + tw - 1) / tw);
  f.ntiles = f.tiles_x * (uint32_t)((f.P.H + th - 1) / th);
}

}  // namespace dqj

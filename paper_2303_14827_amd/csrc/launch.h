// launch.h -- host-side launchers of the library's kernels (library-internal).
#pragma once
#include <hip/hip_runtime.h>

#include "kparams.h"

namespace dqj {

// FP64 iteration constants for FP64 kernels (the caller's values, not FP32-rounded).
struct KIter64 {
  double c[8];
  double R2;
  int32_t N, norm;
};

// Straightforward FP32 render: one thread per pixel, no lane refill.
hipError_t launch_render_direct(const KParams &P, const KOut &out, hipStream_t s);

// Distance-estimate march in FP32: one thread per pixel, blocks of waves_per_block (1-4)
// waves of 8 x 8 pixels each.
hipError_t launch_render_de(const KParams &P, const KOut &out, int waves_per_block, hipStream_t s);

// The distance-estimate march over n frames of a device table (one-thread-per-pixel kernel,
// frame = blockIdx.z); all frames share norm; all_axis: every frame on the identity slice;
// count: some frame has an update counter (else the kernel without counting runs).
hipError_t launch_render_de_batch(const FrameDesc *table_dev, int nframes, int max_w, int max_h,
                                  int norm, bool all_axis, bool count, hipStream_t s);

// Projection ("shadow") rendering: fibre offsets in R^8 added to every slice point (FP32,
// passed by value as a kernel argument), and the one-thread-per-pixel FP32 render of the
// projection with F of them.
constexpr int kMaxFiber = 32;
struct FiberTable {
  float off[kMaxFiber][8];
};
hipError_t launch_render_project(const KParams &P, const FiberTable &fb, int F, const KOut &out,
                                 hipStream_t s);

// Four-neighbour normal and shade of every hit pixel of a rendered frame, from its depths.
hipError_t launch_neighbour_normal(const KParams &P, const KOut &out, hipStream_t s);

// Classify n points of R^8 (row-major n x 8) in FP32 / FP64.
hipError_t launch_classify_f32(const float *pts, int n, const KParams &P, int32_t *esc,
                               float *n2, hipStream_t s);
hipError_t launch_classify_f64(const double *pts, int n, const KIter64 &P, int32_t *esc,
                               float *n2, hipStream_t s);

}  // namespace dqj

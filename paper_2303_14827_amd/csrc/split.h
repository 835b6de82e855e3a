// split.h -- split-precision launchers and their device scratch (library-internal).
#pragma once
#include <hip/hip_runtime.h>

#include "kparams.h"
#include "runtime_internal.h"

namespace dqj {

// A ray of the candidate list: the FP32 pass scans it from sample khat - w; kend < 0:
// the FP16 march found an inside sample, and the scan runs to the first FP32 inside
// sample; kend >= 0: no FP16 inside sample, and the scan ends after sample kend + w.
// On the FP64 list, khat is the sample the FP64 pass starts from (less w).
struct SplitEntry {
  uint32_t frame;
  uint32_t pix;
  int32_t khat;
  int32_t kend;
};

// A run of consecutive candidate-list entries of one frame (the FP16 march writes its
// candidates in such chunks; the FP32 pass takes a chunk at a time).
struct SplitChunk {
  uint32_t frame;
  uint32_t base;
  uint32_t count;
  uint32_t pad;
};

// Device scratch of one split launch: ctr[0] tile counter, ctr[1] candidate-list length,
// ctr[2] FP64-list length, ctr[3] chunk count, ctr[4] chunks taken by the FP32 pass. The
// lists hold up to one entry per pixel, the chunk array up to one chunk per entry.
struct SplitScratch {
  uint32_t *ctr;
  SplitEntry *hits;
  SplitEntry *amb;
  SplitChunk *chunks;
};

constexpr size_t split_scratch_bytes(uint64_t pixels) {
  return 256 + (2 * sizeof(SplitEntry) + sizeof(SplitChunk)) * (size_t)pixels;
}

inline SplitScratch split_scratch_at(void *base, uint64_t pixels) {
  SplitScratch s;
  s.ctr = (uint32_t *)base;
  s.hits = (SplitEntry *)((char *)base + 256);
  s.amb = s.hits + pixels;
  s.chunks = (SplitChunk *)(s.amb + pixels);
  return s;
}

hipError_t launch_render_split(const FrameDesc &frame, const SplitScratch &sc, const Sched &s,
                               int cus, hipStream_t stream);
// hdr_dev (may be null) overrides nframes/total_tiles with values read on the device.
hipError_t launch_render_split_batch(const FrameDesc *table_dev, const LaunchHeader *hdr_dev,
                                     int nframes, uint32_t total_tiles, int norm, bool all_axis,
                                     bool any_count, const SplitScratch &sc, const Sched &s, int cus,
                                     hipStream_t stream);

}  // namespace dqj

// kparams.h -- the FP32 record one frame's kernels read (library-internal).
//
// The host turns a dqj_params (FP64) into this record: it builds the camera basis
// and all derived constants in FP64 and rounds each once to FP32. Kernels of a
// single frame take it by value (kernel arguments, read through the scalar
// cache); batched and served kernels read it from a device-resident table.
#pragma once
#include <stdint.h>

namespace dqj {

struct alignas(16) KParams {
  float c[8];            // Julia constant [r0..r3 | d0..d3]
  float so[8];           // slice origin O
  float su[8], sv[8], sw[8];   // slice axes U, V, W
  float eye[3];
  float R2;              // escape radius squared
  float fwd[3];
  float h;               // normal step
  float right[3];
  float sx_scale;        // tan(fov_y / 2) * W / H
  float up[3];
  float sy_scale;        // tan(fov_y / 2)
  float bmin[3];
  float inv_w;
  float bmax[3];
  float inv_h;
  float light[3];        // unit vector towards the light
  float ka;
  float kd;
  int32_t W, H, N;       // image size, max_iter
  int32_t S, B;          // march steps, bisection steps
  int32_t norm;          // 0: 8 squares, 1: real part only
  int32_t axis_slice;    // 1 if O = 0 and U, V, W = e0, e1, e2 (zeta_0 = (X, Y, Z, 0 | 0))
  int32_t fp64_window;   // split precision verify window
  int32_t sticky1;       // 1 if, on the identity slice, escaping on the first update
                         // implies escaping on the second (see pack_params)
  int32_t march;         // 0: fixed steps, 1: distance-estimate steps
  float de_eps;          // DE march: hit threshold
  float de_min_step, de_max_step;
  float de_inv_r2;       // 1 / R^2 (the scaled derivative norm, see render_de.hip)
  float de_log2_4r2;     // log2(4 R^2)
  int32_t algebra;       // 0: a^2 + (ab + ba) e, 1: a^2 + b^2 e (grid classification only)
  int32_t normal_mode;   // 0: potential gradient, 1: from the four neighbouring pixels' hits
  float ks;              // specular coefficient (0: none)
  float shininess;       // specular exponent
  float cull_r2;         // bounding sphere radius squared (0: none)
  int32_t T16;           // split precision: updates the FP16 march trusts (a sample
                         // still bounded after T16 updates is a candidate crossing)
  int32_t pad2[2];
};
static_assert(sizeof(KParams) % 16 == 0, "KParams must be 16-byte sized");

// The same frame in FP64 (camera basis and derived constants never rounded to FP32),
// for the FP64 re-bisection of the split-precision path and FP64 classification.
struct alignas(16) KParams64 {
  double c[8];
  double so[8], su[8], sv[8], sw[8];
  double eye[3], fwd[3], right[3], up[3];
  double bmin[3], bmax[3];
  double light[3];
  double sx_scale, sy_scale, inv_w, inv_h;
  double R2, h, ka, kd;
  double ks, shininess, cull_r2;
  int32_t normal_mode, pad;
};

// What one frame writes (device pointers; optional ones may be null).
struct KOut {
  uint8_t *mask;
  float *depth;
  float *shade;
  uint8_t *image8;
  float *normal;
  int32_t *first_hit;
  uint8_t *flags;
  unsigned long long *iters;
};

// One frame of a (possibly single-frame) persistent launch: its parameters, its
// outputs, and where its tiles sit in the launch's global tile sequence.
// An entry may cover a chunk of a frame's tiles: tiles tile_offset .. tile_offset +
// ntiles - 1 of the frame (a served request split across several launches).
struct alignas(16) FrameDesc {
  KParams P;
  KParams64 P64;
  KOut out;
  uint32_t tile_begin;   // first global tile index of this entry in the launch
  uint32_t tiles_x;      // tiles per image row
  uint32_t ntiles;       // tiles of this entry
  uint32_t tile_offset;  // frame tile of this entry's first tile
};

// Device header a launch may read its size from (so one captured graph serves any
// table contents): [0] number of entries, [1] total tiles.
struct LaunchHeader {
  uint32_t nframes;
  uint32_t total_tiles;
  uint32_t pad[62];
};

}  // namespace dqj

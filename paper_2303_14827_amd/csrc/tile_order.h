// tile_order.h -- the order in which a persistent launch hands out the tiles of a frame.
//
// A launch's time ends with its slowest rays: once the tile queue is empty, a wave
// runs on until its last lane has finished. The rays that take longest pass close to
// the set, which a camera aimed at the slice box sees near the image centre, so the
// last frame of a launch is handed out from the centre outward; the long rays then
// start early and the short rays near the image edge fill the ramp-down. Any order
// gives the same images: every pixel is computed the same way wherever it runs.
#pragma once

#include <cstdint>
#include <cmath>

namespace dqj {

// Tiles in the rings at depth >= l of an X x Y tile grid: the rectangle left after l
// tiles are taken off every side.
__host__ __device__ inline uint32_t rings_from(int32_t l, int32_t X, int32_t Y) {
  const int32_t a = X - 2 * l, b = Y - 2 * l;
  return (a > 0 && b > 0) ? (uint32_t)a * (uint32_t)b : 0u;
}

// Tile k (0 <= k < X*Y) of an X x Y tile grid in centre-out order, as ty * X + tx.
// The grid is peeled into rectangular rings (ring l: the tiles l steps in from the
// nearest grid edge); the deepest ring comes first, and each ring is walked clockwise
// from its top-left tile. A bijection on [0, X*Y).
__host__ __device__ inline uint32_t centre_out_tile(uint32_t k, int32_t X, int32_t Y) {
  const int32_t L = ((X < Y ? X : Y) + 1) / 2;   // number of rings
  // k lies in ring l when rings_from(l + 1) <= k < rings_from(l). rings_from(l) = k is
  // a quadratic in l; its smaller root, rounded down, is l up to rounding, then corrected
  // with exact integer tests.
  const double d = (double)X - (double)Y;
  int32_t l = (int32_t)floor(((double)X + (double)Y - sqrt(d * d + 4.0 * (double)k)) * 0.25);
  if (l > L - 1) l = L - 1;
  if (l < 0) l = 0;
  while (l > 0 && rings_from(l, X, Y) <= k) --l;
  while (l + 1 < L && rings_from(l + 1, X, Y) > k) ++l;
  const int32_t j = (int32_t)(k - rings_from(l + 1, X, Y));   // position on the ring
  const int32_t w = X - 2 * l, h = Y - 2 * l;
  int32_t tx, ty;
  if (h == 1) {            // the innermost ring is a row
    tx = l + j;
    ty = l;
  } else if (w == 1) {     // ... or a column
    tx = l;
    ty = l + j;
  } else if (j < w) {      // top row, left to right
    tx = l + j;
    ty = l;
  } else if (j < w + h - 1) {   // right column, downward
    tx = l + w - 1;
    ty = l + 1 + (j - w);
  } else if (j < 2 * w + h - 2) {   // bottom row, right to left
    tx = l + w - 2 - (j - (w + h - 1));
    ty = l + h - 1;
  } else {                 // left column, upward
    tx = l;
    ty = l + h - 2 - (j - (2 * w + h - 2));
  }
  return (uint32_t)ty * (uint32_t)X + (uint32_t)tx;
}

}  // namespace dqj

"""The centre-out tile order of a launch's last frame (csrc/tile_order.h), built for the
host with g++: a bijection on every grid, innermost ring first, rings in depth order.
The GPU tests check the other half, that images do not depend on the order."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_14827_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")

MAIN = r"""
#include "tile_order.h"
#include <cstdio>
#include <vector>
static int depth(int tx, int ty, int X, int Y) {
  int d = tx;
  if (X - 1 - tx < d) d = X - 1 - tx;
  if (ty < d) d = ty;
  if (Y - 1 - ty < d) d = Y - 1 - ty;
  return d;
}
static long check(int X, int Y) {
  long bad = 0;
  std::vector<char> seen((size_t)X * Y, 0);
  int prev = 1 << 30;
  for (uint32_t k = 0; k < (uint32_t)X * (uint32_t)Y; ++k) {
    const uint32_t t = dqj::centre_out_tile(k, X, Y);
    if (t >= (uint32_t)X * (uint32_t)Y || seen[t]) { ++bad; continue; }
    seen[t] = 1;
    const int d = depth((int)(t % X), (int)(t / X), X, Y);
    if (d > prev) ++bad;   // rings come deepest first
    prev = d;
  }
  return bad;
}
int main() {
  long bad = 0;
  for (int X = 1; X <= 64; ++X)
    for (int Y = 1; Y <= 64; ++Y) bad += check(X, Y);
  // up to the grids of the largest frame sides (16384) in 8 x 8 tiles, and of a
  // 16384-pixel row or column in single-pixel tiles
  const int big[][2] = {{240, 135}, {135, 240}, {128, 128}, {1024, 1024}, {4096, 3}, {3, 4096},
                        {2048, 2048}, {16384, 1}, {1, 16384}, {16384, 8}, {8, 16384}};
  for (const auto &g : big) bad += check(g[0], g[1]);
  // a 16384 x 16384 grid (one-pixel tiles of the largest frame), on a stride: every tile in
  // range and the ring depth never rising along the order
  int prev = 1 << 30;
  for (uint32_t k = 0; k < 16384u * 16384u; k += 4099u) {
    const uint32_t t = dqj::centre_out_tile(k, 16384, 16384);
    if (t >= 16384u * 16384u) { ++bad; continue; }
    const int d = depth((int)(t % 16384u), (int)(t / 16384u), 16384, 16384);
    if (d > prev) ++bad;
    prev = d;
  }
  std::printf("%s %ld\n", bad ? "bad" : "ok", bad);
  return bad ? 1 : 0;
}
"""


def test_centre_out_is_a_ring_ordered_bijection(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(MAIN)
    exe = str(tmp_path / "t")
    subprocess.run(["g++", "-std=c++17", "-O2", "-D__host__=", "-D__device__=", "-I", CSRC,
                    str(src), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr

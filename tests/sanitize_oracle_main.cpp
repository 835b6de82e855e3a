// Drives every entry point of the FP64 oracle once on small inputs, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_sanitizers.py). Prints
// "ok" and returns 0 when nothing was reported; the sanitizers abort otherwise.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dqj_oracle.h"

static dqjo_params base_params(int w, int h) {
  dqjo_params p;
  std::memset(&p, 0, sizeof p);
  p.struct_size = sizeof(dqjo_params);
  const double c[8] = {-0.25, 0.35, 0.1, -0.2, 0.3, -0.1, 0.2, 0.05};
  for (int k = 0; k < 8; ++k) p.c[k] = c[k];
  p.slice_axes[0][0] = p.slice_axes[1][1] = p.slice_axes[2][2] = 1.0;
  for (int k = 0; k < 3; ++k) {
    p.box_min[k] = -1.5;
    p.box_max[k] = 1.5;
  }
  p.eye[0] = 1.3;
  p.eye[1] = 1.0;
  p.eye[2] = 2.5;
  p.up[1] = 1.0;
  p.fov_y_deg = 60.0;
  p.width = w;
  p.height = h;
  p.max_iter = 12;
  p.march_steps = 64;
  p.bisect_steps = 8;
  p.escape_radius = 4.0;
  p.fp64_window = 2;
  p.normal_h = 1e-3;
  p.light_dir[0] = p.light_dir[1] = p.light_dir[2] = 1.0 / std::sqrt(3.0);
  p.k_ambient = 0.1;
  p.k_diffuse = 0.9;
  p.de_hit_eps = 1e-4;
  p.de_min_step = 1e-4;
  p.de_max_step = 0.25;
  return p;
}

static uint64_t render_all(const dqjo_params &p, int nthreads) {
  const size_t n = (size_t)p.width * p.height;
  std::vector<uint8_t> mask(n);
  std::vector<double> depth(n), shade(n), normal(3 * n);
  std::vector<int32_t> first(n);
  std::vector<uint64_t> iters(n);
  return dqjo_render(&p, nullptr, 0, mask.data(), depth.data(), shade.data(), normal.data(),
                     first.data(), iters.data(), nthreads);
}

int main() {
  dqjo_params p = base_params(40, 28);
  uint64_t total = 0;
  total += render_all(p, 1);
  total += render_all(p, 2);

  // a pixel list, outputs partly absent
  const int64_t pix[5] = {0, 17, 300, 561, 40 * 28 - 1};
  std::vector<uint8_t> m5(5);
  std::vector<double> d5(5);
  total += dqjo_render(&p, pix, 5, m5.data(), d5.data(), nullptr, nullptr, nullptr, nullptr, 1);

  // c = 0: the ball, every ray through the centre hits
  dqjo_params ball = p;
  for (int k = 0; k < 8; ++k) ball.c[k] = 0.0;
  total += render_all(ball, 1);

  // options: real-part norm, four-neighbour normal, specular term, bounding sphere
  dqjo_params opt = p;
  opt.norm = DQJO_NORM_REALPART;
  opt.normal_mode = 1;
  opt.k_specular = 0.4;
  opt.shininess = 20.0;
  opt.cull_radius = 1.4;
  total += render_all(opt, 1);

  // distance-estimate march
  dqjo_params de = p;
  de.march = 1;
  de.march_steps = 200;
  total += render_all(de, 1);

  // projection over three fibre offsets
  const double fib[24] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0.3, 0.1, 0, 0, 0,
                          0, 0, 0, -0.2, 0, 0.2, 0, 0.1};
  dqjo_params pr = p;
  pr.fiber_count = 3;
  pr.fiber = fib;
  total += render_all(pr, 1);

  // edge sizes
  total += render_all(base_params(1, 1), 1);
  dqjo_params one_step = base_params(7, 3);
  one_step.march_steps = 1;
  one_step.bisect_steps = 0;
  one_step.max_iter = 1;
  total += render_all(one_step, 1);

  // voxel grid, both algebras, full and listed voxels
  std::vector<uint8_t> in(6 * 5 * 4);
  std::vector<int32_t> mv(6 * 5 * 4);
  total += dqjo_classify_grid(&p, 6, 5, 4, nullptr, 0, in.data(), mv.data(), 1);
  dqjo_params alg = p;
  alg.algebra = 1;
  const int64_t vox[3] = {0, 7, 119};
  total += dqjo_classify_grid(&alg, 6, 5, 4, vox, 3, in.data(), mv.data(), 2);

  // points, algebra, rays
  double z0[8] = {0.1, -0.2, 0.3, 0.0, 0.05, 0.0, -0.1, 0.0}, zf[8], out[8], n2 = 0.0, de_v = 0.0;
  int32_t m = 0;
  dqjo_classify(&p, z0, &m, zf, &n2);
  dqjo_distance(&p, z0, &m, &de_v);
  std::vector<double> pts(8 * 9);
  for (size_t k = 0; k < pts.size(); ++k) pts[k] = 0.1 * std::sin((double)k);
  std::vector<uint8_t> ins(9);
  std::vector<int32_t> ms(9);
  std::vector<double> nn(9), zz(8 * 9);
  dqjo_classify_many(&p, pts.data(), 9, ins.data(), ms.data(), nn.data(), zz.data());
  const double a[4] = {0.1, 0.2, -0.3, 0.4}, b[4] = {-0.5, 0.1, 0.2, 0.3};
  double q[4];
  dqjo_quat_mul(a, b, q);
  dqjo_quat_square_eq(a, q);
  dqjo_dq_add(z0, zf, out);
  dqjo_dq_mul(z0, zf, out);
  dqjo_dq_square(z0, out);
  dqjo_orbit(z0, p.c, 5, out);
  const double x[3] = {0.2, -0.1, 0.4};
  dqjo_slice_map(&p, x, out);
  dqjo_potential(&p, x, &m);
  double o3[3], d3[3], t0 = 0.0, t1 = 0.0, nrm[3], sh = 0.0;
  if (dqjo_ray(&p, 20, 14, o3, d3, &t0, &t1)) {
    std::vector<uint8_t> cls(64);
    dqjo_scan_ray(&p, 20, 14, t0, t1, 64, cls.data());
    dqjo_shade_at(&p, 20, 14, 0.5 * (t0 + t1), nrm, &sh);
  }
  if (dqjo_params_size() != sizeof(dqjo_params)) return 2;
  std::printf("ok %llu\n", (unsigned long long)total);
  return 0;
}

// dqj_oracle.cpp -- plain FP64 CPU oracle (test infrastructure only; see dqj_oracle.h).
//
// Built with -O2 -ffp-contract=off -fno-fast-math: every product and sum is rounded
// on its own, IEEE round-to-nearest, so inf/NaN behave as the C standard says.
// Nothing here is blocked, fused or reordered beyond what each cited passage states.
#include "dqj_oracle.h"

#include <math.h>
#include <string.h>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

// ---------------------------------------------------------------------------
// Quaternion operations (Appendix, "Quaternion Operations"). A quaternion is the
// 4-tuple (s, v) = (q0, q1, q2, q3): slot 0 is the scalar s, slots 1..3 the
// vector v on the i, j, k axes.
// ---------------------------------------------------------------------------

// multiplication: [s1, v1][s2, v2] = [s1 s2 - v1.v2, s1 v2 + s2 v1 + v1 x v2]
void dqjo_quat_mul(const double a[4], const double b[4], double out[4]) {
  const double s1 = a[0], s2 = b[0];
  const double v1[3] = {a[1], a[2], a[3]};
  const double v2[3] = {b[1], b[2], b[3]};
  const double dot = v1[0] * v2[0] + v1[1] * v2[1] + v1[2] * v2[2];
  const double cross[3] = {v1[1] * v2[2] - v1[2] * v2[1],
                           v1[2] * v2[0] - v1[0] * v2[2],
                           v1[0] * v2[1] - v1[1] * v2[0]};
  double r[4];
  r[0] = s1 * s2 - dot;
  for (int k = 0; k < 3; ++k) r[k + 1] = s1 * v2[k] + s2 * v1[k] + cross[k];
  memcpy(out, r, sizeof r);
}

// Eq. quatsq: q^2 = (x^2 - y^2 - z^2 - w^2, 2xy, 2xz, 2xw), x the scalar slot.
void dqjo_quat_square_eq(const double q[4], double out[4]) {
  const double x = q[0], y = q[1], z = q[2], w = q[3];
  double r[4];
  r[0] = x * x - y * y - z * z - w * w;
  r[1] = 2.0 * x * y;
  r[2] = 2.0 * x * z;
  r[3] = 2.0 * x * w;
  memcpy(out, r, sizeof r);
}

// ---------------------------------------------------------------------------
// Dual-quaternion operations (Appendix, "Dual-Quaternion Operations").
// zeta = q_r + q_d e, stored as [q_r | q_d] (8 doubles), e^2 = 0 (Introduction,
// "Geometric Properties of Complex & Dual Numbers").
// ---------------------------------------------------------------------------

// addition, the printed "q_r1 + q_r1" read as q_r1 + q_r2.
void dqjo_dq_add(const double x[8], const double y[8], double out[8]) {
  double r[8];
  for (int k = 0; k < 8; ++k) r[k] = x[k] + y[k];
  memcpy(out, r, sizeof r);
}

// multiplication, the printed "q_r1 + q_r2" of the real part read as q_r1 q_r2:
// (q_r1 + q_d1 e)(q_r2 + q_d2 e) = q_r1 q_r2 + (q_r1 q_d2 + q_d1 q_r2) e.
void dqjo_dq_mul(const double x[8], const double y[8], double out[8]) {
  double real[4], t1[4], t2[4], r[8];
  dqjo_quat_mul(x, y, real);          // q_r1 q_r2
  dqjo_quat_mul(x, y + 4, t1);        // q_r1 q_d2
  dqjo_quat_mul(x + 4, y, t2);        // q_d1 q_r2
  for (int k = 0; k < 4; ++k) {
    r[k] = real[k];
    r[k + 4] = t1[k] + t2[k];
  }
  memcpy(out, r, sizeof r);
}

// zeta^2 = zeta zeta = a a + (a b + b a) e. The printed component-wise form
// q_a^2 + q_b^2 e is not what the product rule gives; the product rule is taken.
void dqjo_dq_square(const double z[8], double out[8]) { dqjo_dq_mul(z, z, out); }

static void dq_step(const double z[8], const double c[8], double out[8]) {
  double sq[8];
  dqjo_dq_square(z, sq);
  dqjo_dq_add(sq, c, out);
}

// The square as printed with Eq. dqjulia2, component by component: q_a^2 + q_b^2 e, each
// quaternion squared with the Hamilton product. Offered as an alternative algebra.
static void dq_step_componentwise(const double z[8], const double c[8], double out[8]) {
  double sq[8];
  dqjo_quat_mul(z, z, sq);
  dqjo_quat_mul(z + 4, z + 4, sq + 4);
  dqjo_dq_add(sq, c, out);
}

static void step_for(const dqjo_params *p, const double z[8], double out[8]) {
  if (p->algebra == 1)
    dq_step_componentwise(z, p->c, out);
  else
    dq_step(z, p->c, out);
}

void dqjo_orbit(const double z0[8], const double c[8], int32_t n, double out[8]) {
  double z[8];
  memcpy(z, z0, sizeof z);
  for (int32_t i = 0; i < n; ++i) dq_step(z, c, z);
  memcpy(out, z, sizeof z);
}

// Escape norm. Default: the sum of the squares of all 8 components (the series
// must stay bounded in every component, section "Dual-Quaternion Julia Sets", and
// the estimator uses a quaternion calculation for the real and for the dual part,
// section "Experimental Results"). Alternative: the real quaternion's squares only
// (the dual-number modulus |a + b e| = |a| of the Introduction).
static double escape_norm2(const dqjo_params *p, const double z[8]) {
  double s = 0.0;
  const int ncomp = (p->norm == DQJO_NORM_REALPART) ? 4 : 8;
  for (int k = 0; k < ncomp; ++k) s += z[k] * z[k];
  return s;
}

// Section "Practical Considerations": iterate up to max_iter; a point that has not
// passed the escape limit by then is inside. The test runs after every update
// (z_0 itself is not tested) and is strict: ||z||^2 > R^2 escapes, a tie stays.
int32_t dqjo_classify(const dqjo_params *p, const double z0[8], int32_t *m,
                      double zfinal[8], double *norm2) {
  const double R2 = p->escape_radius * p->escape_radius;
  double z[8];
  memcpy(z, z0, sizeof z);
  double n2 = escape_norm2(p, z);
  int32_t inside = 1;
  int32_t n = 0;
  for (n = 1; n <= p->max_iter; ++n) {
    step_for(p, z, z);
    n2 = escape_norm2(p, z);
    if (n2 > R2) {
      inside = 0;
      break;
    }
  }
  if (inside) n = p->max_iter;
  if (m) *m = n;
  if (zfinal) memcpy(zfinal, z, sizeof z);
  if (norm2) *norm2 = n2;
  return inside;
}

// Distance estimate (section "Ray-Marching", Eq. distfract2 after Hart et al.):
// iterate as dqjo_classify while carrying the derivative norm of Eq. distfract, read
// as |z'_{n+1}| = 2 |z_n| |z'_n| with |z'_0| = 1 (the printed indices are garbled); the
// norms are the escape norm. For a point that escapes at m the estimate is
// 0.5 |z_m| ln|z_m| / |z'_m|. Returns 1 for an inside point (no estimate).
int32_t dqjo_distance(const dqjo_params *p, const double z0[8], int32_t *m, double *de) {
  const double R2 = p->escape_radius * p->escape_radius;
  double z[8];
  memcpy(z, z0, sizeof z);
  double n2 = escape_norm2(p, z);     // |z_0|^2
  double dz = 1.0;                    // |z'_0|
  for (int32_t n = 1; n <= p->max_iter; ++n) {
    dz = 2.0 * sqrt(n2) * dz;         // |z'_n| from |z_{n-1}| and |z'_{n-1}|
    step_for(p, z, z);
    n2 = escape_norm2(p, z);
    if (n2 > R2) {
      const double r = sqrt(n2);
      if (m) *m = n;
      if (de) *de = 0.5 * r * log(r) / dz;
      return 0;
    }
  }
  if (m) *m = p->max_iter;
  if (de) *de = 0.0;
  return 1;
}

void dqjo_classify_many(const dqjo_params *p, const double *pts, int64_t n,
                        uint8_t *inside, int32_t *m, double *norm2, double *zfinal) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    int32_t mi;
    double n2, zf[8];
    const int32_t in = dqjo_classify(p, pts + 8 * i, &mi, zf, &n2);
    if (inside) inside[i] = (uint8_t)in;
    if (m) m[i] = mi;
    if (norm2) norm2[i] = n2;
    if (zfinal) memcpy(zfinal + 8 * i, zf, sizeof zf);
  }
}

// Section "Dimension Reduction": a 3-flat through R^8, zeta_0 = O + X U + Y V + Z W.
void dqjo_slice_map(const dqjo_params *p, const double x[3], double z0[8]) {
  for (int k = 0; k < 8; ++k) {
    z0[k] = p->slice_origin[k] + x[0] * p->slice_axes[0][k] + x[1] * p->slice_axes[1][k] +
            x[2] * p->slice_axes[2][k];
  }
}

static void normalize3(double v[3]) {
  const double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= len;
  v[1] /= len;
  v[2] /= len;
}

static void cross3(const double a[3], const double b[3], double out[3]) {
  double r[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  memcpy(out, r, sizeof r);
}

// Pinhole camera (the paper leaves the camera to the renderer): forward f towards
// the target, right r = f x up, true up u = r x f; vertical field of view; the ray
// through the centre of pixel (i, j), row 0 at the top. Then the ray is clipped to
// the axis-aligned box that bounds the fractal (the paper's bounding-volume cull,
// section "Ray-Marching"), slab by slab.
int32_t dqjo_ray(const dqjo_params *p, int32_t i, int32_t j, double o[3], double d[3],
                 double *t0, double *t1) {
  double f[3] = {p->target[0] - p->eye[0], p->target[1] - p->eye[1], p->target[2] - p->eye[2]};
  normalize3(f);
  double r[3];
  cross3(f, p->up, r);
  normalize3(r);
  double u[3];
  cross3(r, f, u);
  const double pi = 3.14159265358979323846;
  const double tan_half = tan(0.5 * p->fov_y_deg * pi / 180.0);
  const double W = p->width, H = p->height;
  const double sx = (2.0 * (i + 0.5) / W - 1.0) * tan_half * (W / H);
  const double sy = (1.0 - 2.0 * (j + 0.5) / H) * tan_half;
  for (int k = 0; k < 3; ++k) {
    o[k] = p->eye[k];
    d[k] = f[k] + sx * r[k] + sy * u[k];
  }
  normalize3(d);
  double tn = 0.0, tf = INFINITY;
  for (int k = 0; k < 3; ++k) {
    if (d[k] == 0.0) {
      if (o[k] < p->box_min[k] || o[k] > p->box_max[k]) return 0;
      continue;
    }
    double ta = (p->box_min[k] - o[k]) / d[k];
    double tb = (p->box_max[k] - o[k]) / d[k];
    if (ta > tb) {
      const double s = ta;
      ta = tb;
      tb = s;
    }
    if (ta > tn) tn = ta;
    if (tb < tf) tf = tb;
  }
  if (tn > tf) return 0;
  // Bounding sphere about the origin (section "Ray-Marching": rays meet a sphere that
  // encloses the fractal first): |o + t d|^2 <= r^2 for t in [-b - sqrt(q), -b + sqrt(q)],
  // b = o.d, q = b^2 - (|o|^2 - r^2); no real root misses.
  if (p->cull_radius > 0.0) {
    const double b = o[0] * d[0] + o[1] * d[1] + o[2] * d[2];
    const double oo = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    const double q = b * b - (oo - p->cull_radius * p->cull_radius);
    if (q < 0.0) return 0;
    const double sq = sqrt(q);
    const double sa = -b - sq, sb = -b + sq;
    if (sa > tn) tn = sa;
    if (sb < tf) tf = sb;
    if (tn > tf) return 0;
  }
  *t0 = tn;
  *t1 = tf;
  return 1;
}

// Paragraph "Dimension Reduction", approach (2): the projection of the set onto the
// 3D space of the slice. A world point of the projection is inside when some point of
// R^8 that projects onto it is inside; the fibre of points over x is sampled by the F
// offsets p->fiber, tried in order until one is inside. *m is the number of updates
// spent over the points tried (N for the inside one).
static int32_t classify_world(const dqjo_params *p, const double x[3], int32_t *m) {
  double z0[8];
  dqjo_slice_map(p, x, z0);
  if (p->fiber_count <= 0) return dqjo_classify(p, z0, m, nullptr, nullptr);
  int32_t total = 0;
  for (int32_t f = 0; f < p->fiber_count; ++f) {
    double z[8];
    for (int q = 0; q < 8; ++q) z[q] = z0[q] + p->fiber[8 * f + q];
    int32_t mf;
    const int32_t in = dqjo_classify(p, z, &mf, nullptr, nullptr);
    total += mf;
    if (in) {
      *m = total;
      return 1;
    }
  }
  *m = total;
  return 0;
}

// Normals (section "Lighting/Illumination" samples neighbouring points with a small
// delta). The sampled field is the escape potential ln||z_m||^2 / 2^m (2 ln|x| exactly
// for c = 0). Where the norm of a square is the square of the norm (the real-part
// norm, a zero dual part) it is nearly continuous across escape-index changes. Under
// the 8-square norm an orbit whose norm nearly reached R in its dual part can fall
// back, so the potential can jump across the surface, and a stencil across the jump
// tilts the normal.
//
// A potential is held as its two parts: lv = ln(max(||z_m||^2, 1e-30)) and the escape
// index m (N when inside), the value being lv * 2^-m. For a projection the field is the
// least potential over the fibre points (the potential of the union of the fibre's
// inside sets): the parts of the least one, and *total the updates over all F.
static void potential_parts(const dqjo_params *p, const double x[3], double *lv, int32_t *me,
                            int32_t *total) {
  double z0[8];
  dqjo_slice_map(p, x, z0);
  const int32_t F = p->fiber_count > 0 ? p->fiber_count : 1;
  int32_t sum = 0;
  for (int32_t f = 0; f < F; ++f) {
    double z[8], zf[8], n2;
    for (int q = 0; q < 8; ++q) z[q] = z0[q] + (p->fiber_count > 0 ? p->fiber[8 * f + q] : 0.0);
    int32_t mi;
    dqjo_classify(p, z, &mi, zf, &n2);
    sum += mi;
    const double v = n2 > 1e-30 ? n2 : 1e-30;
    const double l = log(v);
    // compare l 2^-mi with the best so far, both scaled by 2^min(mi, me)
    bool less = f == 0;
    if (!less) {
      const int32_t mm = mi < *me ? mi : *me;
      less = l * ldexp(1.0, mm - mi) < *lv * ldexp(1.0, mm - *me);
    }
    if (less) {
      *lv = l;
      *me = mi;
    }
  }
  *total = sum;
}

double dqjo_potential(const dqjo_params *p, const double x[3], int32_t *m) {
  double lv;
  int32_t me, total;
  potential_parts(p, x, &lv, &me, &total);
  if (m) *m = total;
  return lv * ldexp(1.0, -me);
}

struct PixelResult {
  uint8_t mask;
  double depth, shade, normal[3];
  int32_t first_hit;
  uint64_t iters;
};

// Eq. phong with one directional light of unit intensity: ambient, diffuse
// k_d max(0, n.l) and specular k_s max(0, r.v)^s with the reflected light vector
// r = 2 n (n.l) - l and v = -d pointing back to the eye, the specular term only where
// the light reaches the surface (n.l > 0); the sum is clamped to [0, 1].
static double phong(const dqjo_params *p, const double n[3], const double d[3]) {
  double l[3] = {p->light_dir[0], p->light_dir[1], p->light_dir[2]};
  normalize3(l);
  double ndl = n[0] * l[0] + n[1] * l[1] + n[2] * l[2];
  double s = p->k_ambient + p->k_diffuse * (ndl > 0.0 ? ndl : 0.0);
  if (p->k_specular > 0.0 && ndl > 0.0) {
    double rv = 0.0;
    for (int k = 0; k < 3; ++k) rv += (2.0 * n[k] * ndl - l[k]) * (-d[k]);
    if (rv > 0.0) s += p->k_specular * pow(rv, p->shininess);
  }
  if (s < 0.0) s = 0.0;
  if (s > 1.0) s = 1.0;
  return s;
}

// Section "Lighting/Illumination": the normal at a hit point ph is the normalised
// central difference of the potential along the world axes (the ray's reversed
// direction where the difference vanishes or is not finite); the shade is Eq. phong.
// The six potentials are taken relative to their least escape index m0: the difference
// is formed from lv 2^(m0 - m), which is the potential times 2^m0. A common positive
// factor leaves the normalised gradient unchanged (exactly, as a power of two), and
// the scaled terms stay representable at any max_iter: unscaled, 2^-m and its square
// underflow in double precision once m passes about 537. (When all six points stay
// inside, the terms are ln||z_N||^2 at full weight: for c = 0 that is 2^(N+1) ln|x|, a
// radial field; where orbits settle on an attracting cycle, at large max_iter their
// differences are rounding noise, and so is such a normal.) The 6 points' updates are
// added to *iters.
static double hit_normal_shade(const dqjo_params *p, const double d[3], const double ph[3],
                               double n[3], uint64_t *iters) {
  double lv[3][2];
  int32_t me[3][2];
  int32_t m0 = 0;
  for (int a = 0; a < 3; ++a) {
    for (int s = 0; s < 2; ++s) {
      double x[3] = {ph[0], ph[1], ph[2]};
      x[a] = s == 0 ? ph[a] + p->normal_h : ph[a] - p->normal_h;
      int32_t total;
      potential_parts(p, x, &lv[a][s], &me[a][s], &total);
      *iters += (uint64_t)total;
      if ((a == 0 && s == 0) || me[a][s] < m0) m0 = me[a][s];
    }
  }
  // Central differences of the scaled potential along the world axes.
  double g[3];
  for (int a = 0; a < 3; ++a)
    g[a] = lv[a][0] * ldexp(1.0, m0 - me[a][0]) - lv[a][1] * ldexp(1.0, m0 - me[a][1]);
  const double glen = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  if (glen > 0.0 && isfinite(glen)) {
    n[0] = g[0] / glen;
    n[1] = g[1] / glen;
    n[2] = g[2] / glen;
  } else {
    n[0] = -d[0];
    n[1] = -d[1];
    n[2] = -d[2];
  }

  return phong(p, n, d);
}

static PixelResult render_pixel(const dqjo_params *p, int32_t i, int32_t j) {
  PixelResult res;
  res.mask = 0;
  res.depth = INFINITY;
  res.shade = 0.0;
  res.normal[0] = res.normal[1] = res.normal[2] = 0.0;
  res.first_hit = -1;
  res.iters = 0;

  double o[3], d[3], t0, t1;
  if (!dqjo_ray(p, i, j, o, d, &t0, &t1)) return res;

  const int32_t S = p->march_steps;
  int32_t kstar = -1;
  double thit = t0;
  double lo = t0, hi = t0;       // bracket to bisect (when bisect is set)
  int bisect = 0;
  if (p->march == 1) {
    // Distance-estimate march (section "Ray-Marching"): from the box entry, step by the
    // estimate clamped to [min_step, max_step] until it falls below the hit threshold
    // (hit at this point), a step lands inside the set (bisect that step), the ray
    // leaves the box, or S steps were taken (miss).
    double t = t0, tprev = t0;
    for (int32_t k = 0; k < S; ++k) {
      const double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
      double z0[8], de;
      int32_t m;
      dqjo_slice_map(p, x, z0);
      const int32_t in = dqjo_distance(p, z0, &m, &de);
      res.iters += (uint64_t)m;
      if (in) {
        kstar = k;
        if (k == 0) {
          thit = t0;
        } else {
          lo = tprev;
          hi = t;
          bisect = 1;
        }
        break;
      }
      if (de < p->de_hit_eps) {
        kstar = k;
        thit = t;
        break;
      }
      double step = de < p->de_min_step ? p->de_min_step : de;
      if (step > p->de_max_step) step = p->de_max_step;
      tprev = t;
      t = t + step;
      if (t > t1) break;
    }
  } else {
    // Fixed-step march: S steps over [t0, t1], samples t_k = t0 + k dt, k = 0..S.
    const double dt = (t1 - t0) / S;
    for (int32_t k = 0; k <= S; ++k) {
      const double t = t0 + k * dt;
      const double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
      int32_t m;
      const int32_t in = classify_world(p, x, &m);
      res.iters += (uint64_t)m;
      if (in) {
        kstar = k;
        break;
      }
    }
    // Bisection of the bracket [t_{k*-1}, t_{k*}]; a hit on the first sample has no
    // outside end to bracket: the hit is t0.
    if (kstar > 0) {
      lo = t0 + (kstar - 1) * dt;
      hi = t0 + kstar * dt;
      bisect = 1;
    }
  }
  if (kstar < 0) return res;

  // Bisection: the hit is the final midpoint (B = 0: the midpoint of the bracket).
  if (bisect) {
    for (int32_t b = 0; b < p->bisect_steps; ++b) {
      const double tm = 0.5 * (lo + hi);
      const double x[3] = {o[0] + tm * d[0], o[1] + tm * d[1], o[2] + tm * d[2]};
      int32_t m;
      const int32_t in = classify_world(p, x, &m);
      res.iters += (uint64_t)m;
      if (in)
        hi = tm;
      else
        lo = tm;
    }
    thit = 0.5 * (lo + hi);
  }
  const double ph[3] = {o[0] + thit * d[0], o[1] + thit * d[1], o[2] + thit * d[2]};
  res.mask = 1;
  res.depth = thit;
  res.first_hit = kstar;
  // The four-neighbour normal needs the neighbouring pixels' hits: dqjo_render forms it
  // and the shade after every pixel has its depth; no update is spent on it here.
  if (p->normal_mode == 1) return res;

  res.shade = hit_normal_shade(p, d, ph, res.normal, &res.iters);
  return res;
}

// Normal and shade at a caller-given depth t on pixel (i, j)'s ray (the same steps as a
// render's hit, at any point): for checking how a shade depends on where the hit lies.
// Returns 0 when the ray misses the box (nothing written), 1 otherwise.
int32_t dqjo_shade_at(const dqjo_params *p, int32_t i, int32_t j, double t, double normal[3],
                      double *shade) {
  double o[3], d[3], t0, t1;
  if (!dqjo_ray(p, i, j, o, d, &t0, &t1)) return 0;
  const double ph[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
  uint64_t iters = 0;
  *shade = hit_normal_shade(p, d, ph, normal, &iters);
  return 1;
}

// Paragraph "Lighting/Illumination": a normal from the surface through the hit points
// of the four neighbouring pixels (left, right, above, below). dep[0..4] are the depths
// of pixel (i, j) and of (i-1, j), (i+1, j), (i, j-1), (i, j+1) (row 0 at the top; +inf
// for a miss or a pixel outside the image). Along each image axis the tangent is the
// central difference of the neighbours' hit points when both hit, else the one-sided
// difference with the pixel's own hit; the normal is the normalised cross product of the
// horizontal tangent (towards the right) and the vertical tangent (towards the top),
// turned to face the eye. A missing tangent or a vanishing product gives -d.
static void neighbour_normal(const dqjo_params *p, int32_t i, int32_t j, const double dep[5],
                             double n[3], double dc[3]) {
  const int32_t ni[5] = {i, i - 1, i + 1, i, i};
  const int32_t nj[5] = {j, j, j, j - 1, j + 1};
  double P[5][3];
  int hit[5];
  for (int q = 0; q < 5; ++q) {
    hit[q] = isfinite(dep[q]) ? 1 : 0;
    double o[3], d[3], t0, t1;
    const int32_t ii = ni[q] < 0 ? 0 : (ni[q] >= p->width ? p->width - 1 : ni[q]);
    const int32_t jj = nj[q] < 0 ? 0 : (nj[q] >= p->height ? p->height - 1 : nj[q]);
    dqjo_ray(p, ii, jj, o, d, &t0, &t1);
    if (q == 0) memcpy(dc, d, sizeof(double) * 3);
    for (int k = 0; k < 3; ++k) P[q][k] = hit[q] ? o[k] + dep[q] * d[k] : 0.0;
  }
  double tx[3], ty[3];
  int hx = 1, hy = 1;
  for (int k = 0; k < 3; ++k) {
    if (hit[1] && hit[2]) tx[k] = P[2][k] - P[1][k];
    else if (hit[2]) tx[k] = P[2][k] - P[0][k];
    else if (hit[1]) tx[k] = P[0][k] - P[1][k];
    else hx = 0;
    if (hit[3] && hit[4]) ty[k] = P[3][k] - P[4][k];
    else if (hit[3]) ty[k] = P[3][k] - P[0][k];
    else if (hit[4]) ty[k] = P[0][k] - P[4][k];
    else hy = 0;
  }
  double c[3] = {0.0, 0.0, 0.0};
  if (hx && hy) cross3(tx, ty, c);
  const double len = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  if (hx && hy && len > 0.0 && isfinite(len)) {
    for (int k = 0; k < 3; ++k) n[k] = c[k] / len;
    if (n[0] * dc[0] + n[1] * dc[1] + n[2] * dc[2] > 0.0)
      for (int k = 0; k < 3; ++k) n[k] = -n[k];
  } else {
    for (int k = 0; k < 3; ++k) n[k] = -dc[k];
  }
}

static double depth_of(const dqjo_params *p, int32_t i, int32_t j) {
  if (i < 0 || j < 0 || i >= p->width || j >= p->height) return INFINITY;
  return render_pixel(p, i, j).depth;
}

uint64_t dqjo_render(const dqjo_params *p, const int64_t *pix, int64_t npix, uint8_t *mask,
                     double *depth, double *shade, double *normal, int32_t *first_hit,
                     uint64_t *iters, int32_t nthreads) {
  const int64_t W = p->width, H = p->height;
  const int64_t total = pix ? npix : W * H;
  uint64_t sum = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  // Four-neighbour normals of a full frame read the frame's own depth buffer.
  std::vector<double> frame_depth;
  if (p->normal_mode == 1 && !pix) frame_depth.assign((size_t)total, INFINITY);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : sum)
  for (int64_t q = 0; q < total; ++q) {
    const int64_t idx = pix ? pix[q] : q;
    const int32_t i = (int32_t)(idx % W), j = (int32_t)(idx / W);
    PixelResult r = render_pixel(p, i, j);
    if (p->normal_mode == 1) {
      if (!pix) {
        frame_depth[(size_t)q] = r.depth;
      } else if (r.mask) {
        const double dep[5] = {r.depth, depth_of(p, i - 1, j), depth_of(p, i + 1, j),
                               depth_of(p, i, j - 1), depth_of(p, i, j + 1)};
        double dc[3];
        neighbour_normal(p, i, j, dep, r.normal, dc);
        r.shade = phong(p, r.normal, dc);
      }
    }
    if (mask) mask[q] = r.mask;
    if (depth) depth[q] = r.depth;
    if (shade) shade[q] = r.shade;
    if (normal) {
      normal[3 * q + 0] = r.normal[0];
      normal[3 * q + 1] = r.normal[1];
      normal[3 * q + 2] = r.normal[2];
    }
    if (first_hit) first_hit[q] = r.first_hit;
    if (iters) iters[q] = r.iters;
    sum += r.iters;
  }
  if (p->normal_mode == 1 && !pix) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < total; ++q) {
      if (!isfinite(frame_depth[(size_t)q])) continue;
      const int32_t i = (int32_t)(q % W), j = (int32_t)(q / W);
      auto at = [&](int32_t ii, int32_t jj) {
        return (ii < 0 || jj < 0 || ii >= W || jj >= H) ? INFINITY
                                                        : frame_depth[(size_t)(jj * W + ii)];
      };
      const double dep[5] = {frame_depth[(size_t)q], at(i - 1, j), at(i + 1, j), at(i, j - 1),
                             at(i, j + 1)};
      double n[3], dc[3];
      neighbour_normal(p, i, j, dep, n, dc);
      if (shade) shade[q] = phong(p, n, dc);
      if (normal)
        for (int k = 0; k < 3; ++k) normal[3 * q + k] = n[k];
    }
  }
  return sum;
}

// Dense voxel grid (the voxel prototype of section "Ray-Marching"): voxel centres of the
// box, slice-mapped and classified.
uint64_t dqjo_classify_grid(const dqjo_params *p, int32_t nx, int32_t ny, int32_t nz,
                            const int64_t *idx, int64_t nidx, uint8_t *inside, int32_t *m,
                            int32_t nthreads) {
  const int64_t total = idx ? nidx : (int64_t)nx * ny * nz;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  uint64_t sum = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : sum)
  for (int64_t q = 0; q < total; ++q) {
    const int64_t v = idx ? idx[q] : q;
    const int64_t i = v % nx, j = (v / nx) % ny, k = v / ((int64_t)nx * ny);
    const double x[3] = {
        p->box_min[0] + ((double)i + 0.5) * (p->box_max[0] - p->box_min[0]) / nx,
        p->box_min[1] + ((double)j + 0.5) * (p->box_max[1] - p->box_min[1]) / ny,
        p->box_min[2] + ((double)k + 0.5) * (p->box_max[2] - p->box_min[2]) / nz};
    int32_t mi;
    const int32_t in = classify_world(p, x, &mi);
    if (inside) inside[q] = (uint8_t)in;
    if (m) m[q] = in ? 0 : mi;
    sum += (uint64_t)mi;
  }
  return sum;
}

int32_t dqjo_scan_ray(const dqjo_params *p, int32_t i, int32_t j, double ta, double tb,
                      int32_t n, uint8_t *classes) {
  double o[3], d[3], t0, t1;
  dqjo_ray(p, i, j, o, d, &t0, &t1);
  int32_t changes = 0;
  for (int32_t k = 0; k < n; ++k) {
    const double t = ta + (tb - ta) * k / (n - 1);
    const double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    int32_t m;
    classes[k] = (uint8_t)classify_world(p, x, &m);
    if (k > 0 && classes[k] != classes[k - 1]) ++changes;
  }
  return changes;
}

uint32_t dqjo_params_size(void) { return (uint32_t)sizeof(dqjo_params); }

}  // extern "C"

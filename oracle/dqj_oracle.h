/*
 * dqj_oracle.h -- plain, slow FP64 CPU oracle for dual-quaternion Julia ray marching.
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the GPU library's
 * results. Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it. The GPU library never links, loads or calls it, and it shares
 * no source, header or constant with the GPU library.
 *
 * Every function is scalar FP64 code compiled without FMA contraction or fast
 * math. The steps follow the paper in its order and notation:
 *   - algebra: Appendix "Quaternion Operations" (Hamilton product) and
 *     "Dual-Quaternion Operations" (product, with the two printed typos read as
 *     (q_r1 + q_r2) + (q_d1 + q_d2)e for the sum and q_r1 q_r2 + (q_r1 q_d2 + q_d1 q_r2)e
 *     for the product);
 *   - iteration zeta_{n+1} = zeta_n^2 + c (Eq. dqjulia2) with the maximum-iteration
 *     rule of section "Practical Considerations";
 *   - 3D slice of section "Dimension Reduction";
 *   - fixed-step ray march over the bounding box (section "Ray-Marching"),
 *     bisection of the first inside/outside crossing, central-difference normal of
 *     a smooth escape potential (section "Lighting/Illumination"), and the ambient +
 *     diffuse terms of Eq. phong;
 *   - extensions: the distance-estimate march of Eq. distfract2, the bounding
 *     sphere, the specular term of Eq. phong, a normal from the four neighbouring
 *     pixels' hits, the component-wise square printed with Eq. dqjulia2, and the
 *     dense voxel grid of the paper's first prototype.
 *
 * Readings where the paper is silent or garbled are listed in the oracle source
 * next to the code that takes them.
 *
 * Pins (CPU tests, independent of these formulas): algebra identities, c = 0 closed
 * forms of the iteration, the render (ball, and the quadric of a general affine slice
 * with its origin and axis order) and the projection (union of shifted balls, least
 * potential over the fibre), the quaternion and complex reductions, symmetries, the
 * dual part as a derivative, brute-force marches, and for c != 0 the normal and shade
 * against the traced surface's own normal where the potential is smooth. Parity
 * unpinned: the normal where a stencil straddles a jump of the potential (no
 * independent value; the GPU is checked against this oracle only).
 */
#ifndef DQJ_ORACLE_H
#define DQJ_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DQJO_NORM_EUCLID8 = 0, DQJO_NORM_REALPART = 1 };

/* Same meaning as the product library's parameter record; an independent copy. */
typedef struct dqjo_params {
  uint32_t struct_size;
  double c[8];
  double slice_origin[8];
  double slice_axes[3][8];
  double box_min[3], box_max[3];
  double eye[3], target[3], up[3];
  double fov_y_deg;
  int32_t width, height, max_iter, march_steps, bisect_steps;
  double escape_radius;
  int32_t norm, precision, fp64_window;
  double normal_h;
  double light_dir[3];
  double k_ambient, k_diffuse;
  int32_t march;               /* 0: fixed steps, 1: distance-estimate steps */
  double de_hit_eps, de_min_step, de_max_step;
  int32_t algebra;             /* 0: a^2 + (ab + ba)e, 1: a^2 + b^2 e (printed form) */
  int32_t normal_mode;         /* 0: potential gradient, 1: four neighbouring pixels */
  double k_specular, shininess;    /* specular term of Eq. phong */
  double cull_radius;          /* bounding sphere about the origin, 0: none */
  int32_t fiber_count;         /* projection: 0 (slice), or F fibre offsets */
  int32_t fiber_reserved;
  const double *fiber;         /* F x 8 offsets in R^8 added to the slice point */
} dqjo_params;

/* ---- algebra (Appendix) ---- */
void dqjo_quat_mul(const double a[4], const double b[4], double out[4]);
void dqjo_quat_square_eq(const double q[4], double out[4]);   /* Eq. quatsq form */
void dqjo_dq_add(const double x[8], const double y[8], double out[8]);
void dqjo_dq_mul(const double x[8], const double y[8], double out[8]);
void dqjo_dq_square(const double z[8], double out[8]);        /* z*z via dqjo_dq_mul */

/* n updates z <- z^2 + c with no escape test (orbit state after n steps). */
void dqjo_orbit(const double z0[8], const double c[8], int32_t n, double out[8]);

/* Classify one point of R^8: returns 1 if inside (no escape within max_iter
 * updates), else 0. *m = escape index (1..max_iter) or max_iter when inside;
 * zfinal (may be NULL) = z_m; *norm2 (may be NULL) = ||z_m||^2 under p->norm. */
int32_t dqjo_classify(const dqjo_params *p, const double z0[8], int32_t *m,
                      double zfinal[8], double *norm2);

/* Batched classify over n points (row-major n x 8). Outputs may be NULL. */
/* Distance estimate 0.5 |z_m| ln|z_m| / |z'_m| of a point that escapes at m, with
 * |z'_{n+1}| = 2 |z_n| |z'_n|, |z'_0| = 1 (section "Ray-Marching", Eq. distfract,
 * Eq. distfract2). Returns 1 (and *de = 0) for an inside point. */
int32_t dqjo_distance(const dqjo_params *p, const double z0[8], int32_t *m, double *de);
void dqjo_classify_many(const dqjo_params *p, const double *pts, int64_t n,
                        uint8_t *inside, int32_t *m, double *norm2, double *zfinal);

/* Dense grid classification: the nx x ny x nz voxel centres
 * x_i = box_min + (i + 1/2)(box_max - box_min)/n of the box, each mapped through the
 * slice and classified. Voxel (i, j, k) is entry (k ny + j) nx + i. If idx is NULL every
 * voxel is classified and outputs are full grids; otherwise only the nidx listed voxel
 * indices, with outputs indexed by list position. inside: 1/0; m: escape index, 0 when
 * inside. Returns the total number of updates (the escape index, or max_iter when
 * inside, summed). Outputs may be NULL. */
uint64_t dqjo_classify_grid(const dqjo_params *p, int32_t nx, int32_t ny, int32_t nz,
                            const int64_t *idx, int64_t nidx, uint8_t *inside, int32_t *m,
                            int32_t nthreads);

/* World point -> R^8 through the slice. */
void dqjo_slice_map(const dqjo_params *p, const double x[3], double z0[8]);

/* Camera ray through pixel (i = column, j = row, row 0 top), clipped to the box.
 * Returns 1 if the ray meets the box (t0 <= t1, t0 >= 0), else 0. */
int32_t dqjo_ray(const dqjo_params *p, int32_t i, int32_t j, double o[3], double d[3],
                 double *t0, double *t1);

/* Smooth escape potential used for normals: ln(max(||z_m||^2, 1e-30)) * 2^-m. */
double dqjo_potential(const dqjo_params *p, const double x[3], int32_t *m);

/* Render. If pix is NULL all width*height pixels are rendered (index = j*width+i)
 * and outputs are full images; otherwise only the npix listed pixel indices are
 * rendered and outputs are indexed by list position. Any output may be NULL.
 *   mask: 1 hit / 0 miss; depth: ray parameter t (inf on miss); shade in [0,1];
 *   normal: 3 per pixel (0 on miss); first_hit: k* (-1 on miss);
 *   iters: DQ updates the method runs for the pixel (march up to and including
 *   the first inside sample, bisection, 6 normal samples).
 * Returns the total number of DQ updates. nthreads <= 0: OpenMP default. */
uint64_t dqjo_render(const dqjo_params *p, const int64_t *pix, int64_t npix,
                     uint8_t *mask, double *depth, double *shade, double *normal,
                     int32_t *first_hit, uint64_t *iters, int32_t nthreads);

/* Inside/outside classes of n points evenly spaced on [ta, tb] of pixel (i, j)'s
 * ray (n >= 2, both ends included). Returns the number of class changes. */
int32_t dqjo_scan_ray(const dqjo_params *p, int32_t i, int32_t j, double ta, double tb,
                      int32_t n, uint8_t *classes);

uint32_t dqjo_params_size(void);

/* Normal and shade (section "Lighting/Illumination", Eq. phong) at depth t on pixel
 * (i, j)'s ray, by the same steps as a render's hit. Returns 0 if the ray misses the box. */
int32_t dqjo_shade_at(const dqjo_params *p, int32_t i, int32_t j, double t, double normal[3],
                      double *shade);

#ifdef __cplusplus
}
#endif
#endif

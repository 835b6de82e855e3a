/*
 * dqj.h -- C ABI of the MI355X (gfx950) dual-quaternion Julia ray-march library.
 *
 * What the library computes (Kenwright, "Dual-Quaternion Julia Fractals"):
 *   - a dual quaternion zeta = q_r + q_d e is 8 reals [r0 r1 r2 r3 | d0 d1 d2 d3],
 *     slot 0 of each quaternion its scalar (Eq. quatsq squares its first slot as the
 *     scalar; Appendix, "Quaternion Operations" and "Dual-Quaternion Operations");
 *   - the iteration zeta_{n+1} = zeta_n^2 + c (Eq. dqjulia2), with
 *     (a + e b)^2 = a^2 + e (a b + b a) (the Appendix product rule with e^2 = 0);
 *   - escape when ||zeta||^2 > R^2 (strict), tested after every update; a point that
 *     has not escaped after max_iter updates is inside (section "Practical
 *     Considerations");
 *   - a 3D slice zeta_0 = O + X U + Y V + Z W through R^8 (section "Dimension
 *     Reduction");
 *   - per pixel, a ray clipped to a bounding box and marched in march_steps equal
 *     steps (section "Ray-Marching"); the first inside sample k* is refined by
 *     bisect_steps bisections of [t_{k*-1}, t_{k*}] (hit = final midpoint; k* = 0
 *     gives the box entry point); the normal is the normalised central difference
 *     (step normal_h) of the escape potential ln(||z_m||^2) 2^-m, m the escape
 *     index; shade = clamp(k_a + k_d max(0, n.l), 0, 1) (section
 *     "Lighting/Illumination", Eq. phong, ambient and diffuse terms).
 *
 * Conventions for every call:
 *   - Parameter records are read during the call and copied; the caller keeps
 *     ownership. Output buffers are DEVICE pointers owned by the caller; they must
 *     stay valid until the stream has executed the work (render calls) or until
 *     poll/wait reports a final status (serve calls).
 *   - Render calls validate synchronously, enqueue on the caller's HIP stream
 *     (NULL = the null stream) and return without waiting. A device fault shows up
 *     as DQJ_E_DEVICE on a later call.
 *   - No C++ exception crosses this boundary. On any non-OK status a description is
 *     available from dqj_last_error() on the same thread.
 *   - Images are H x W row-major, row 0 at the top, pixel (i, j) at index j*W + i.
 */
#ifndef DQJ_H
#define DQJ_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dqj_status;
enum {
  DQJ_OK = 0,
  DQJ_PENDING = 1,
  DQJ_E_INVALID = -1,      /* a parameter failed validation */
  DQJ_E_NOMEM = -2,        /* device or host allocation failed */
  DQJ_E_BUDGET = -3,       /* request alone exceeds the server's HBM budget */
  DQJ_E_QUEUE_FULL = -4,   /* server pending queue is full */
  DQJ_E_DEVICE = -5,       /* HIP runtime or kernel error */
  DQJ_E_TIMEOUT = -6,
  DQJ_E_CANCELLED = -7,
  DQJ_E_UNSUPPORTED = -8,  /* no gfx950 device, or a mode the library does not offer */
  DQJ_E_STATE = -9         /* call not valid in the object's current state */
};

/* Escape norm. EUCLID8 (default): sum of all 8 squares -- the series must stay
 * bounded in every component (section "Dual-Quaternion Julia Sets").
 * REALPART: squares of the real quaternion only -- the dual-number modulus
 * |a + b e| = |a| of the Introduction. */
enum { DQJ_NORM_EUCLID8 = 0, DQJ_NORM_REALPART = 1 };

/* Arithmetic of the render. FP32: every step in FP32. SPLIT: march in packed FP16, which
 * decides only escapes within its trust depth (N - ceil(N/4) updates, ceil(3N/8) for
 * the real-part norm: FP16 orbits near the boundary part from exact ones after some
 * updates); samples escaping later and
 * the FP16 crossing are re-checked in FP32, which also bisects, takes the normal and
 * shades; rays whose FP32 in/out test flips within fp64_window samples of the crossing
 * are re-done in FP64. Same accuracy bar as FP32. FP64: every step in FP64 on the GPU. */
enum { DQJ_PREC_FP32 = 0, DQJ_PREC_SPLIT = 1, DQJ_PREC_FP64 = 2 };

typedef struct dqj_params {
  uint32_t struct_size;        /* = sizeof(dqj_params); other values -> DQJ_E_INVALID */
  double c[8];                 /* Julia constant [r0..r3 | d0..d3] */
  double slice_origin[8];      /* O */
  double slice_axes[3][8];     /* U, V, W: world X, Y, Z -> R^8 */
  double box_min[3], box_max[3];   /* march region, box_min < box_max */
  double eye[3], target[3], up[3]; /* pinhole camera; up not parallel to target-eye */
  double fov_y_deg;            /* vertical field of view, (0, 180) */
  int32_t width, height;       /* 1..16384 */
  int32_t max_iter;            /* N, 1..4096 */
  int32_t march_steps;         /* S >= 1: S+1 samples t_k = t0 + k (t1-t0)/S */
  int32_t bisect_steps;        /* B >= 0 (0..64) */
  double escape_radius;        /* R > 0: escape iff ||z||^2 > R^2 (SPLIT: R^2 < 65504) */
  int32_t norm;                /* DQJ_NORM_* */
  int32_t precision;           /* DQJ_PREC_* */
  int32_t fp64_window;         /* SPLIT only: FP32 verify window +-w samples (1..8), default 2 */
  double normal_h;             /* central-difference step, > 0 */
  double light_dir[3];         /* direction towards the light (normalised by the library) */
  double k_ambient, k_diffuse;
  /* March mode (section "Ray-Marching"). FIXED: the S-step march above, then bisection.
   * DE: steps of the distance estimate 0.5 |z_m| ln|z_m| / |z'_m| (Eq. distfract2), with
   * |z'_{n+1}| = 2 |z_n| |z'_n| and |z'_0| = 1 (Eq. distfract; norms are the escape norm),
   * clamped to [de_min_step, de_max_step]; a hit when the estimate drops below de_hit_eps,
   * or, if a step lands inside the set, the bisection of that step; at most S steps.
   * DE renders run in FP32 through dqj_render only. */
  int32_t march;               /* DQJ_MARCH_FIXED (0) or DQJ_MARCH_DE (1) */
  double de_hit_eps;           /* DE: > 0, world units */
  double de_min_step;          /* DE: > 0 */
  double de_max_step;          /* DE: >= de_min_step */
  /* Algebra of the square (section "Dual-Quaternion Julia Sets"). DUAL: the square the
   * dual-quaternion product gives, (a + b e)^2 = a^2 + (ab + ba) e. COMPONENTWISE: the form
   * printed with Eq. dqjulia2, a^2 + b^2 e (its dual orbit does not depend on the point
   * when the slice keeps b_0 = 0). COMPONENTWISE is offered by dqj_classify_grid only;
   * renders return DQJ_E_UNSUPPORTED for it. */
  int32_t algebra;             /* DQJ_ALGEBRA_DUAL (0) or DQJ_ALGEBRA_COMPONENTWISE (1) */
  /* Normal estimate (paragraph "Lighting/Illumination"). POTENTIAL: central differences of
   * the escape potential ln(max(||z_m||^2, 1e-30)) 2^-m at p +- normal_h along each axis.
   * NEIGHBOUR4: from the hit points of the four neighbouring pixels (above, below, left,
   * right), n = normalize((P_right - P_left) x (P_up - P_down)) with one-sided differences
   * where a neighbour misses and -d where a whole pair misses, facing the eye; dqj_render
   * only (batches and the server return DQJ_E_UNSUPPORTED). */
  int32_t normal_mode;         /* DQJ_NORMAL_POTENTIAL (0) or DQJ_NORMAL_NEIGHBOUR4 (1) */
  /* Specular term of Eq. phong: k_specular * max(0, r . v)^shininess with
   * r = 2 n (n . l) - l and v = -d (towards the eye), added where n . l > 0. */
  double k_specular;           /* >= 0; 0 leaves the ambient + diffuse shade */
  double shininess;            /* >= 1 */
  /* Bounding sphere (section "Ray-Marching"): rays are clipped to the sphere of this
   * radius about the world origin as well as to the box, so rays that miss it are
   * discarded before any update. 0 disables the sphere. */
  double cull_radius;          /* >= 0 */
  /* Projection ("shadow") rendering, the second dimension reduction of paragraph
   * "Dimension Reduction": with fiber_count = F > 0, a world point x is inside when any of
   * the F points O + x U + y V + z W + fiber[f] is inside (f = 0..F-1; fiber holds F
   * offsets in R^8, row-major F x 8, host memory read during the call). The offsets
   * sample the directions the projection collapses, so the image is the shadow of the
   * set sampled at those fibre points. The potential of the normal is the least of the F
   * points' potentials. dqj_render, dqj_render_batch and batch plans (a batch holds
   * projection frames only, or none: DQJ_E_INVALID otherwise), FP32 fixed-step march with
   * the dual square; the server, the autotuner and other modes return DQJ_E_UNSUPPORTED.
   * 0: slice rendering. */
  int32_t fiber_count;         /* 0..32 */
  int32_t fiber_reserved;      /* 0 */
  const double *fiber;         /* fiber_count x 8 values; NULL when fiber_count = 0 */
} dqj_params;

enum { DQJ_MARCH_FIXED = 0, DQJ_MARCH_DE = 1 };
enum { DQJ_ALGEBRA_DUAL = 0, DQJ_ALGEBRA_COMPONENTWISE = 1 };
enum { DQJ_NORMAL_POTENTIAL = 0, DQJ_NORMAL_NEIGHBOUR4 = 1 };

/* Per-pixel ray flags written to dqj_frame_out.flags (bit set). */
enum {
  DQJ_FLAG_BOX = 1,       /* ray meets the box */
  DQJ_FLAG_HIT = 2,       /* a sample was inside */
  DQJ_FLAG_FP64 = 4,      /* SPLIT: ray was re-done in FP64 */
  DQJ_FLAG_FALLBACK = 8   /* normal fell back to -d (zero or non-finite gradient) */
};

typedef struct dqj_frame_out {
  uint32_t struct_size;     /* = sizeof(dqj_frame_out) */
  uint8_t *mask;            /* required: 1 hit, 0 miss */
  float *depth;             /* required: ray parameter t of the hit (distance), +inf on miss */
  float *shade;             /* required: [0, 1], 0 on miss */
  uint8_t *image8;          /* optional: floor(255 shade + 1/2) */
  float *normal;            /* optional: 3 floats per pixel, 0 on miss */
  int32_t *first_hit;       /* optional: k* or -1 */
  uint8_t *flags;           /* optional: DQJ_FLAG_* */
  unsigned long long *iters;/* optional, one counter: += DQ updates the method ran for the
                               frame (march through k*, bisection, 6 normal samples) */
} dqj_frame_out;

/* Render one frame (section "Ray-Marching" through "Lighting/Illumination").
 * precision FP32 and SPLIT are offered (FP64 through SPLIT's re-bisection only); the
 * fixed-step or distance-estimate march; slice rendering, or a projection when
 * params->fiber_count > 0 (paragraph "Dimension Reduction"). Stream-ordered: returns after
 * validation and the launch; errors of the kernels surface as DQJ_E_DEVICE later. */
dqj_status dqj_render(const dqj_params *params, const dqj_frame_out *out, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dqj_render with the same arguments,
 * outputs and results, except that it allocates nothing. dqj_render keeps its tile
 * counter, and for split renders the candidate and FP64 ray lists with the candidates'
 * chunk list, in device blocks it
 * allocates per (device, stream) on first use; this entry point keeps them instead in
 * one fixed device array of DQJ_NOALLOC_SCRATCH_BYTES per GPU, held from the library's
 * first call on that GPU until the process ends. The array bounds the split frames it
 * takes: precision SPLIT with width * height > DQJ_NOALLOC_MAX_SPLIT_PIXELS returns
 * DQJ_E_INVALID before any launch. Every call on one GPU shares that GPU's array (each
 * clears what it needs with a kernel of its own, never a memset), so calls that overlap
 * on one GPU -- on two streams, or from two threads -- race and must be serialised by
 * the caller; calls in one stream's order are safe. */
#define DQJ_NOALLOC_MAX_SPLIT_PIXELS 262144u
#define DQJ_NOALLOC_SCRATCH_BYTES (256u + 48u * DQJ_NOALLOC_MAX_SPLIT_PIXELS)
dqj_status dqj_render_noalloc(const dqj_params *params, const dqj_frame_out *out,
                              void *hip_stream);

/* Render n frames (params[i] -> outs[i]) in one persistent launch over a global
 * (frame, tile) queue. All frames must share precision, march and escape norm. A batch
 * of projection frames (fiber_count > 0, all of them) runs one launch with the frames'
 * blocks interleaved instead. */
dqj_status dqj_render_batch(const dqj_params *params, const dqj_frame_out *outs, int32_t n,
                            void *hip_stream);

/* Kernel choice for FP32 renders. REFILL: persistent waves whose lanes take the
 * next sample or ray as soon as theirs retires. DIRECT: one thread per pixel, the
 * method's steps in order, no refill (the simple yardstick). LOCKSTEP (the
 * distance-estimate march only): persistent waves that classify all lanes' current
 * points together, then advance each lane's ray by one point and refill finished
 * lanes with new rays. Batches take REFILL only. */
enum { DQJ_KERNEL_AUTO = 0, DQJ_KERNEL_REFILL = 1, DQJ_KERNEL_DIRECT = 2, DQJ_KERNEL_LOCKSTEP = 3 };

/* Work schedule of the persistent kernels (chosen by dqj_autotune, or by hand).
 * Any field 0 = library default. A schedule changes speed only: every schedule
 * gives bit-identical images. */
typedef struct dqj_schedule {
  uint32_t struct_size;        /* = sizeof(dqj_schedule) */
  int32_t kernel;              /* DQJ_KERNEL_* */
  int32_t tile_w, tile_h;      /* pixels per tile handed to one wave (tile_w*tile_h <= 4096) */
  int32_t waves_per_block;     /* 1..16 (block = 64 * waves_per_block threads) */
  int32_t blocks_per_cu;       /* persistent grid = CUs * blocks_per_cu, 1..32 */
} dqj_schedule;

/* Time each candidate schedule on the given representative frames (rendered into
 * outs as one batched launch per candidate, so outs are overwritten) and remember
 * the fastest for this workload shape (image size, max_iter, march and bisection
 * steps, precision, norm, slice kind, device). Renders and plans created later
 * without an explicit schedule use it. If cache_path (or the environment variable
 * DQJ_TUNE_CACHE) names a file, the choice is appended to it as a JSON line and the
 * file is read at the first schedule lookup of a later process. best (may be NULL)
 * receives the choice. Synchronous. */
dqj_status dqj_autotune(const dqj_params *params, const dqj_frame_out *outs, int32_t n,
                        const char *cache_path, dqj_schedule *best);

/* dqj_render with an explicit schedule (NULL = autotuned or default). */
dqj_status dqj_render_scheduled(const dqj_params *params, const dqj_frame_out *out,
                                const dqj_schedule *sched, void *hip_stream);

/* A batch captured once into a HIP graph and replayed: the parameter table stays
 * resident in device memory, each replay is one queue reset plus one persistent
 * kernel. sched may be NULL (autotune cache entry if present, else default). */
typedef struct dqj_batch_plan dqj_batch_plan;
dqj_status dqj_batch_plan_create(const dqj_params *params, const dqj_frame_out *outs, int32_t n,
                                 const dqj_schedule *sched, void *hip_stream,
                                 dqj_batch_plan **plan);
dqj_status dqj_batch_plan_launch(dqj_batch_plan *plan, void *hip_stream);
dqj_status dqj_batch_plan_destroy(dqj_batch_plan *plan);   /* waits for its work */

/* Classify n points of R^8 (device, row-major n x 8 floats for FP32 or doubles for
 * FP64; precision DQJ_PREC_FP32 or DQJ_PREC_FP64) with params->c, max_iter,
 * escape_radius and norm. escape_iter[i] = escape index 1..N, or 0 when inside;
 * final_norm2[i] = ||z_m||^2 as float. Test and debugging entry point. */
dqj_status dqj_classify_points(const void *pts_dev, int32_t n, int32_t precision,
                               const dqj_params *params, int32_t *escape_iter_dev,
                               float *final_norm2_dev, void *hip_stream);

/* Dense voxel-grid classification: the paper's first prototype (section "Ray-Marching",
 * the voxel-versus-ray-traced figure) as a throughput entry point. The nx x ny x nz voxel
 * centres x_i = box_min + (i + 1/2)(box_max - box_min)/n of params' box are mapped through
 * the slice and classified with params' c, max_iter, escape_radius, norm and algebra (the
 * camera, march and shading fields are validated but unused); precision must be
 * DQJ_PREC_FP32. Sizes 1..4096 per axis.
 * Outputs (device pointers, caller-owned, voxel (i, j, k) at (k ny + j) nx + i):
 *   mask_dev (required, u8): 1 inside, 0 outside;
 *   escape_dev (optional, i32): escape index 1..max_iter, 0 when inside;
 *   iters_dev (optional, one u64): updates run (escape index, or max_iter inside), added.
 * Stream-ordered; returns after the launch. Errors: DQJ_E_INVALID (sizes, NULL mask,
 * parameters), DQJ_E_UNSUPPORTED (precision), DQJ_E_DEVICE. */
dqj_status dqj_classify_grid(const dqj_params *params, int32_t nx, int32_t ny, int32_t nz,
                             uint8_t *mask_dev, int32_t *escape_dev,
                             unsigned long long *iters_dev, void *hip_stream);

/* ---- Request server (continuous batching) -------------------------------------
 * Requests of any size, Julia constant and max_iter are queued as they are
 * submitted, admitted first come first served while the device bytes their
 * framebuffers hold stay within the budget, and rendered in epochs: each epoch is
 * one persistent launch (replayed from a HIP graph captured per epoch slot) over
 * chunks of tiles taken from every active request, so work arriving while other
 * requests run joins the next epoch and overlaps with them on the device. Up to
 * `slots` epochs are in flight at once, each on its own stream. A request's result
 * is bit-identical to a dqj_render of the same parameters and precision.
 * Every dqj_serve_* call is thread-safe. */

typedef struct dqj_serve_config {
  uint32_t struct_size;        /* = sizeof(dqj_serve_config) */
  uint64_t hbm_budget_bytes;   /* framebuffer bytes of admitted requests at once (0: 8 GiB) */
  int32_t max_inflight;        /* admitted, unfinished requests at once (0: 64) */
  int32_t max_pending;         /* queued requests before submit returns DQJ_E_QUEUE_FULL (0: 4096) */
  int32_t precision;           /* DQJ_PREC_FP32 or DQJ_PREC_SPLIT; every request must match */
  int32_t norm;                /* escape norm; every request must match */
  int32_t slots;               /* epochs in flight at once, 1..8 (0: 3) */
  int32_t count_iters;         /* 1: kernels add executed updates to each request's iters */
  int64_t epoch_pixels;        /* pixels per epoch (0: 4 Mi); sizes the per-slot scratch */
  double epoch_work;           /* estimated DQ updates per epoch (0: 8e9) */
  dqj_schedule sched;          /* tile/wave schedule (struct_size 0: default) */
  int32_t policy;              /* DQJ_SERVE_FAIR (0): every active request gets a share of each
                                  epoch, the rest first come first served; DQJ_SERVE_OLDEST (1):
                                  epochs are filled oldest request first */
} dqj_serve_config;
enum { DQJ_SERVE_FAIR = 0, DQJ_SERVE_OLDEST = 1 };

typedef struct dqj_request_result {
  uint32_t struct_size;        /* = sizeof(dqj_request_result) */
  dqj_status status;           /* DQJ_PENDING until final: DQJ_OK, DQJ_E_CANCELLED, DQJ_E_DEVICE */
  double t_submit, t_admit, t_first_launch, t_done;   /* host steady clock (s); -1 if not yet */
  int32_t chunks;              /* launches the request's tiles were spread over */
} dqj_request_result;

typedef struct dqj_serve_stats {
  uint32_t struct_size;        /* = sizeof(dqj_serve_stats) */
  uint64_t submitted, admitted, completed, cancelled, failed, rejected, epochs;
  int32_t pending, active;
  uint64_t resident_bytes;
  double p50_latency_s, p99_latency_s, max_latency_s, mean_latency_s;  /* t_done - t_submit */
} dqj_serve_stats;

typedef struct dqj_server dqj_server;   /* opaque, library-owned */

/* Create a server on the current device (device memory for `slots` epochs is
 * allocated here). */
dqj_status dqj_serve_create(const dqj_serve_config *cfg, dqj_server **out);
/* Validate and queue a request. out holds caller-owned device buffers that must stay
 * valid until the request is final. DQJ_E_INVALID, DQJ_E_BUDGET (its framebuffer
 * bytes alone exceed the budget), DQJ_E_QUEUE_FULL, DQJ_E_STATE (server closing). */
dqj_status dqj_serve_submit(dqj_server *s, const dqj_params *params, const dqj_frame_out *out,
                            uint64_t *ticket);
/* DQJ_PENDING, or the request's final status; fills *res either way. */
dqj_status dqj_serve_poll(dqj_server *s, uint64_t ticket, dqj_request_result *res);
/* Wait up to timeout_ms (< 0: no limit) for the request to be final: its final
 * status, or DQJ_E_TIMEOUT (the request keeps running). */
dqj_status dqj_serve_wait(dqj_server *s, uint64_t ticket, int32_t timeout_ms,
                          dqj_request_result *res);
/* Cancel a pending or running request (its tiles already launched still finish). */
dqj_status dqj_serve_cancel(dqj_server *s, uint64_t ticket);
dqj_status dqj_serve_stats_get(dqj_server *s, dqj_serve_stats *out);
/* Cancel pending requests, wait for epochs in flight, free everything. */
dqj_status dqj_serve_destroy(dqj_server *s);

typedef struct dqj_device_info {
  uint32_t struct_size;
  char arch[64];               /* e.g. "gfx950:sramecc+:xnack-" */
  int32_t compute_units;
  int32_t clock_khz;           /* peak engine clock reported by the runtime */
  int32_t memory_clock_khz;
  uint64_t total_mem_bytes;
  double fp32_vector_peak_tflops;   /* 256 flop/clk/CU (packed) x CUs x clock */
  double fp32_unpacked_peak_tflops; /* 128 flop/clk/CU x CUs x clock */
} dqj_device_info;
dqj_status dqj_device_info_get(int32_t device, dqj_device_info *out);

const char *dqj_last_error(void);          /* thread-local text of the last non-OK status */
const char *dqj_status_str(dqj_status s);

#ifdef __cplusplus
}
#endif
#endif

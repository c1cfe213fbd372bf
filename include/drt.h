/*
 * drt.h -- C ABI of the dynamic-ray-tracing (DRT) hot path on one AMD Instinct MI355X.
 *
 * Dynamic Ray Tracing (Bilibashi, Vitucci, Degli-Esposti, "On Dynamic Ray Tracing and
 * Anticipative Channel Prediction for Dynamic Environments") takes the multipath of one
 * ray-tracing snapshot at t0 and extrapolates every ray analytically over future instants
 * t0 + dt while terminals and rigid bodies translate and rotate with constant velocity or
 * acceleration (Sec. II).  This library keeps a scene resident in device memory and, per
 * call, re-solves every ray's interaction points, its path length, delay, angles,
 * Doppler and field coefficient at each instant, and synthesises the time-variant
 * transfer function H(t, f) by summing the rays (Sec. II: "the total field, the
 * time-variant channel's transfer function, Doppler's shift frequencies, time delays").
 *
 * Conventions
 *   - every function returns an int status: DRT_OK (0) or a negative DRT_E_* code; on an
 *     error the detail text is available from drt_last_error() in the calling thread and
 *     out-parameters are left untouched;
 *   - no C++ exception crosses this boundary;
 *   - all host arrays passed in are borrowed for the duration of the call only (deep
 *     copied); all device buffers passed in are caller-owned, never freed by the library;
 *   - "device pointer" means memory allocated on the context's device (hipMalloc or a
 *     PyTorch CUDA tensor); "stream" is a hipStream_t passed as void* (NULL = the null
 *     stream); work is enqueued on it and the call returns without waiting;
 *   - floats are IEEE binary64 unless stated; vectors are in metres in one global frame;
 *     direction vectors must be unit length to 1e-9;
 *   - all calls are thread-safe on one context.
 */
#ifndef DRT_H
#define DRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct drt_ctx drt_ctx;

enum drt_status {
  DRT_OK = 0,
  DRT_E_INVAL = -1,        /* bad argument, index out of range, malformed ray */
  DRT_E_DEGENERATE = -2,   /* a ray is degenerate at t0 (see drt_load_scene) */
  DRT_E_NOMEM = -3,        /* device allocation failed or the HBM cap would be exceeded */
  DRT_E_ADMISSION = -4,    /* a request's footprint exceeds the HBM admission cap */
  DRT_E_NOTFOUND = -5,     /* unknown scene id or ticket */
  DRT_E_BUSY = -6,         /* scene still referenced by requests in flight */
  DRT_E_DEVICE = -7,       /* a HIP runtime call failed */
  DRT_E_INCONSISTENT = -8, /* ray_q0 disagrees with the t0 solve by more than 1e-6 m */
  DRT_E_CANCELLED = -9     /* a served request still queued when its context was destroyed */
};

/* Arithmetic of a call.  DRT_FP64: everything in binary64, gains and H complex128.
 * DRT_SPLIT: geometry (interaction points, path length, Doppler, carrier-phase reduction
 * f*L/c modulo one cycle, shadow-boundary distances of the wedge terms) in binary64; field
 * coefficients and angles in binary32 from those binary64 quantities; the per-sample phasor
 * work of H in binary32 / split binary16 on the matrix cores; gains complex64 and H complex64.  DRT_NAIVE32: geometry, gains, phase and H all in binary32 (for the
 * precision sweep only). */
enum drt_precision { DRT_FP64 = 0, DRT_SPLIT = 1, DRT_NAIVE32 = 2 };

enum drt_kind { DRT_R = 1, DRT_D = 2, DRT_S = 3 };   /* reflection, diffraction, scattering */
enum drt_pol { DRT_PERP = 0, DRT_PAR = 1 };          /* soft / TE, hard / TM */

#define DRT_MAX_INT 4

/* The dynamic environment database (Sec. II): geometry at t0 plus the rigid-body dynamics
 * of every object and terminal, and the interaction sequence of each t0 ray. */
typedef struct {
  double t0;                                   /* snapshot time [s] (metadata) */
  double tx_p[3], tx_v[3], tx_a[3];            /* eq. Taylor: position, velocity, acceleration */
  double rx_p[3], rx_v[3], rx_a[3];
  int32_t n_bodies;                            /* >= 1; body 0 is the static world */
  const double *body_O0;                       /* [nb][3] reference point on the rotation axis */
  const double *body_v0, *body_a;              /* [nb][3] translation velocity and acceleration */
  const double *body_axis;                     /* [nb][3] fixed unit rotation axis k */
  const double *body_w0, *body_wdot;           /* [nb] angular speed and acceleration about k */
  int32_t n_mat;
  const double *mat_eps_r, *mat_sigma;         /* [nm] relative permittivity, conductivity [S/m] */
  const uint8_t *mat_pec;                      /* [nm] 1 = perfect conductor */
  int32_t n_planes;
  const int32_t *plane_body, *plane_mat;       /* [np] */
  const double *plane_p0, *plane_n0;           /* [np][3] a point of the plane, unit normal */
  int32_t n_edges;
  const int32_t *edge_body;                    /* [ne] */
  const double *edge_a0, *edge_e0;             /* [ne][3] a point of the edge line, unit direction */
  const double *edge_t0, *edge_n0;             /* [ne][3] 0-face unit tangent (pointing away from the
                                                  edge) and 0-face outward unit normal */
  const double *edge_wedge_n;                  /* [ne] exterior wedge angle / pi */
  int32_t n_tiles;
  const int32_t *tile_body, *tile_alpha;       /* [nt] body, directive-lobe exponent 1..8 */
  const uint8_t *tile_model;                   /* [nt] 0 Lambertian, 1 directive */
  const double *tile_c0, *tile_n0;             /* [nt][3] centroid, outward unit normal */
  const double *tile_area, *tile_S, *tile_phase0;  /* [nt] dS [m^2], scattering coefficient, phase */
  int32_t n_rays;
  const uint8_t *ray_nint;                     /* [nr] 0..4 interactions (0 = line of sight) */
  const uint8_t *ray_kind, *ray_pol;           /* [nr][4] drt_kind, drt_pol per interaction */
  const int32_t *ray_prim;                     /* [nr][4] index into planes / edges / tiles */
  const double *ray_q0;                        /* optional [nr][4][3] t0 interaction points; NULL = skip */
  /* Bounds of the validity monitor (multipath lifetime, Sec. II); both optional. */
  const double *plane_facet;                   /* [np][3][3] the wall's facet at t0: corner, u, v, the
                                                  parallelogram corner + s u + w v, 0 <= s, w <= 1,
                                                  u and v in the plane; u = v = 0: unbounded wall;
                                                  NULL: every wall unbounded */
  const double *edge_zlim;                     /* [ne][2] the edge segment z_lo <= (X - a0) . e0 <= z_hi
                                                  (infinities allowed); NULL: every edge unbounded */
  /* Antennas (optional, both or neither): [4] = unit axis (x, y, z) and kind, 1 = half-wave
   * dipole along the axis (directivity 1.64; the antennas of Sec. IV-B).  With dipoles the
   * field coefficients are polarimetric: the transmitted vector pattern is carried through
   * every reflection (Fresnel perpendicular and parallel coefficients on the basis
   * e_perp = k_in x n, e_par = e_perp x k) and diffraction (UTD soft coefficient for the
   * component along e_beta = s x (e x s)/|e x s|, hard for the one along (e x s)/|e x s|), a
   * tile keeps the field, and the result is projected on the received pattern; the rays'
   * polarisation flags are then ignored.  Needs DRT_FP64 or DRT_SPLIT.  NULL, or kind 0 for
   * both: the scalar model with the flags. */
  const double *tx_ant, *rx_ant;
} drt_scene_desc;

/* t_j = t0 + j*dt, j = 0..n_steps-1. */
typedef struct { double dt; int32_t n_steps; } drt_time_grid;
/* f_k = f_c + (k - n_sub/2) * bandwidth / n_sub (integer division), k = 0..n_sub-1. */
typedef struct { double f_c, bandwidth; int32_t n_sub; } drt_freq_grid;

/* Caller-owned device outputs of drt_extrapolate, each [n_rays][n_steps] (time fastest);
 * any pointer may be NULL to skip that output.  gain is complex128 (interleaved re, im)
 * for DRT_FP64 and complex64 otherwise.  An instant where the ray's chain is inconsistent
 * (a reflection point outside the segment from its virtual receiver to its image, a
 * diffraction source or receiver on the edge line, a tile facing away from a terminal)
 * has valid = 0 and every other output 0; no NaN is ever written. */
typedef struct {
  double *L;                                   /* path length [m] */
  float *dop;                                  /* Doppler shift at f_c [Hz], > 0 when approaching */
  float *aod_az, *aod_el, *aoa_az, *aoa_el;    /* departure / arrival azimuth, elevation [rad] */
  void *gain;                                  /* field coefficient at f_c (no propagation phase) */
  uint8_t *valid;
  /* Validity monitor: in_bounds = valid and, on the geometry displaced to the instant, every
   * reflection point inside its wall's facet with both neighbouring vertices on the front
   * side (n . (P - Q) >= 0) and every diffraction point on its edge segment; first_out
   * ([n_rays]) = the first instant index with in_bounds = 0, n_steps if none. */
  uint8_t *in_bounds;
  int32_t *first_out;
  /* Kinematics of the interaction points (Sec. III-A.1 eqs. ref_point_velo and ref_point_acc,
   * App. B and C), each [n_rays][n_steps][4][3] binary64, interaction slots beyond the ray's
   * count zero: positions, velocities [m/s] and accelerations [m/s^2], exact time derivatives
   * of the re-solved points (computed as second-order jets in binary64 for every precision);
   * dop_rate ([n_rays][n_steps]) = -(f_c/c) d^2 L/dt^2 [Hz/s].  Written where the chain is
   * consistent (reflection parameters in (0, 1), diffraction source and receiver off the
   * edge line; scattering always), zero elsewhere. */
  double *q_pos, *q_vel, *q_acc;
  float *dop_rate;
} drt_ray_out;

typedef struct {
  uint32_t scene;
  int32_t n_rays;                              /* rays [0, n_rays) of the scene */
  drt_time_grid tg;
  drt_freq_grid fg;
  int32_t precision;                           /* DRT_SPLIT or DRT_FP64 */
  void *H;                                     /* device, [n_steps][n_sub] complex64 / complex128 */
} drt_request;

typedef struct {
  int32_t state;                               /* 0 queued, 1 running, 2 done, < 0 error status */
  double t_arrive, t_admit, t_done;            /* seconds on the library's monotonic clock */
} drt_req_stat;

/* Create a context on HIP device `device` (library lifetime management; no passage of the
 * paper defines it).  hbm_cap_bytes bounds the device memory the
 * context holds (resident scenes, scratch, in-flight requests); 0 = 90% of the device.
 * Three environment variables, read here, are tuning knobs: DRT_CFR_KERNEL (mfma16, the
 * default; mfma32; valu) picks the split ray-sum kernel, DRT_TARGET_WAVES (64 .. 2^24) the
 * number of waves it aims for, which sets how many ray groups share an instant, and
 * DRT_BATCH_SAMPLES (1e6 .. 1e13, default 4e9) the rays x instants x subcarriers one serving
 * batch may hold; a malformed value fails the call with DRT_E_INVAL. */
int drt_create(int device, uint64_t hbm_cap_bytes, drt_ctx **out);

/* Destroy a context: waits for the work already started (served batches, calls on caller
 * streams), cancels served requests still queued (DRT_E_CANCELLED; their H is not
 * written), frees every scene and scratch buffer.  Not a call of the paper's method: the
 * library's own lifetime management, as are drt_create and drt_strerror. */
int drt_destroy(drt_ctx *ctx);

/* Validate, pack and upload a scene (Sec. II's dynamic environment database plus the t0
 * rays).  Errors: DRT_E_INVAL (index out of range, n_int > 4, more than one diffraction
 * in a ray other than a two-edge ray (exactly two distinct edges, solved as the shortest path
 * over both edge lines), a scattering interaction that is not the ray's only one, non-unit
 * vectors);
 * DRT_E_DEGENERATE (at t0 a reflection's image line is parallel to its wall, i.e. the
 * denominator y_TX + y_RX of eq. ref_point vanishes, or a diffraction source/receiver
 * lies on the edge line, d_TX + d_RX = 0 in eq. diff_point); DRT_E_INCONSISTENT (ray_q0
 * given and farther than 1e-6 m from the t0 solve).  The scene stays resident until
 * drt_unload_scene. */
int drt_load_scene(drt_ctx *ctx, const drt_scene_desc *desc, uint32_t *scene_id);

/* Free a scene.  DRT_E_BUSY while served requests still reference it. */
int drt_unload_scene(drt_ctx *ctx, uint32_t scene_id);

/* Per-(ray, instant) extrapolation (Sec. III: reflection points by image and
 * back-tracking, diffraction points by the unfolded similar-triangle closed form,
 * scattering points carried rigidly with their body; App. A Doppler) for rays
 * [0, n_rays) over the time grid, field coefficients at carrier f_c.  Writes the
 * non-NULL members of *out on `stream`. */
int drt_extrapolate(drt_ctx *ctx, uint32_t scene, int32_t n_rays, const drt_time_grid *tg,
                    double f_c, int32_t precision, const drt_ray_out *out, void *stream);

/* Classes of paths a snapshot trace looks for. */
typedef struct {
  int32_t max_refl;           /* 0..3: paths of 1..max_refl reflections */
  int32_t max_refl_diff;      /* -1..2: paths of one diffraction and 0..max_refl_diff reflections
                                 (the edge at every position); -1: none */
  int32_t scattering;         /* 1: single diffuse scattering from every tile */
  int32_t los;                /* 1: the line of sight */
  int32_t double_diff;        /* 1: paths over two distinct edges (no reflection) */
} drt_trace_opts;

typedef struct {
  int32_t n_paths;            /* rays of the new scene */
  int32_t n_los, n_refl, n_diff, n_scat;
  int64_t candidates;         /* interaction sequences examined */
  int64_t geometric;          /* of which the interaction points exist (before obstruction) */
} drt_trace_info;

/* Snapshot ray trace at the instant t0 + t of `scene` (Sec. II: the conventional RT whose
 * rays DRT extrapolates, re-run at the end of each multipath lifetime T_C), by the image
 * method on every candidate interaction sequence of the classes in *opts, in binary64:
 * images and back-tracking for reflections (Sec. III-A.2), the unfolded closed form for the
 * diffraction point (Sec. III-B eq. diff_point).  A sequence is a path when every reflection
 * parameter lies in (0, 1), every reflection point lies in its wall's facet (walls without a
 * facet are unbounded) with both neighbouring vertices more than 1e-9 m in front of the wall,
 * the diffraction point lies on its edge segment with the directions to both neighbours in
 * the wedge's exterior (angle from the 0-face in [0, n pi]; for two edges, the points of
 * the shortest path over both edge lines, each so), a tile faces both terminals,
 * and no wall's facet (or unbounded wall) crosses any segment of the path more than 1e-7 m
 * from both of its ends.  Creates a new resident scene (*new_scene): the primitives, bodies
 * and terminals of `scene` carried to t0 + t (body reference points, velocities and angular
 * speeds advanced; primitive indices unchanged) and one ray per path, ordered by class (line
 * of sight; 1..max_refl reflections; one diffraction with 0, 1, 2 reflections, edge first to
 * edge last; two edges; scattering) and then by primitive indices.  Polarisation flags: perpendicular
 * for walls with |n_z| <= 0.5 and vertical edges (|e_z| > 0.5), parallel otherwise;
 * perpendicular for tiles.  Synchronous.  Errors: DRT_E_INVAL for options out of range or a
 * non-finite t; DRT_E_NOTFOUND; DRT_E_NOMEM. */
int drt_trace(drt_ctx *ctx, uint32_t scene, double t, const drt_trace_opts *opts,
              uint32_t *new_scene, drt_trace_info *info);

typedef struct {
  double threshold_db;        /* rays within this many dB of the strongest at a segment's first
                                 instant are the major ones (>= 0) */
  int32_t max_steps;          /* longest segment in instants (>= 1): paths that appear are only
                                 found by the next trace */
  int32_t min_steps;          /* shortest segment in instants, 1..max_steps */
} drt_refresh_opts;

/* Multipath lifetimes over the time grid (Sec. II: the extrapolation holds for a time T_C over
 * which no major path disappears; at its end the conventional trace is run again).  From
 * instant j = 0: trace `scene` at t0 + j dt (drt_trace with *topts), extrapolate the traced
 * scene over the next m = min(max_steps, n_steps - j) instants in binary64 with the validity
 * monitor, take as major the rays whose power |a|^2 at instant j lies within threshold_db of
 * the strongest, and end the segment at the first instant at which a major ray is out of
 * bounds (drt_ray_out first_out), clamped to [min_steps, m]; continue from there.  Writes,
 * for segment k < *n_segments: its first instant seg_start[k], its length seg_len[k] and the
 * resident scene seg_scene[k] traced at its start (the caller unloads them); the instants
 * of segment k are 0..seg_len[k]-1 of that scene's own time grid.  Synchronous.  Errors:
 * DRT_E_INVAL for bad options or more than max_segments segments (no scene is left
 * resident then), and those of drt_trace. */
int drt_segments(drt_ctx *ctx, uint32_t scene, const drt_time_grid *tg, double f_c,
                 const drt_trace_opts *topts, const drt_refresh_opts *ropts, int32_t max_segments,
                 int32_t *seg_start, int32_t *seg_len, uint32_t *seg_scene, int32_t *n_segments);

/* Copy the interaction sequences of a resident scene's rays into caller-owned host arrays
 * of `cap` rays ([cap] nint, [cap][4] kind, prim, pol; any may be NULL); *n_rays receives
 * the scene's ray count (the copy stops at cap). */
int drt_scene_rays(drt_ctx *ctx, uint32_t scene, int32_t cap, int32_t *n_rays, uint8_t *nint,
                   uint8_t *kind, int32_t *prim, uint8_t *pol);

/* Bins of the power profiles.  Instant j falls in time bin j / steps_per_bin; a Doppler
 * shift f_D in bin floor((f_D - dop_lo) / dop_step) and a delay tau in bin
 * floor((tau - delay_lo) / delay_step), counted only when that index lies in [0, n_dop) or
 * [0, n_delay).  Both divisions are correctly rounded binary64. */
typedef struct {
  double dop_lo, dop_step;          /* Hz; dop_step > 0 */
  double delay_lo, delay_step;      /* s; delay_step > 0 */
  int32_t steps_per_bin;            /* instants per time bin, >= 1 */
  int32_t n_dop, n_delay;           /* bins per time bin, >= 0 each */
  int32_t in_bounds_only;           /* 1: count only samples the validity monitor finds in bounds */
} drt_bins;

/* Caller-owned device outputs of drt_power_profiles, binary64, n_tb = ceil(n_steps /
 * steps_per_bin) time bins, row-major with the time bin slowest; any may be NULL. */
typedef struct {
  double *pdfp;                     /* [n_tb][n_dop] power-Doppler profile */
  double *pdp;                      /* [n_tb][n_delay] power-delay profile */
  double *total;                    /* [n_tb] power of every counted sample, in a bin or not */
} drt_power_out;

/* Power-Doppler profile (Sec. IV-A) and power-delay profile (Sec. IV-B) of rays [0, n_rays)
 * over the time grid: each (ray, instant) sample whose chain is consistent (and in bounds,
 * with in_bounds_only) adds its power |a|^2, a being its field coefficient at carrier f_c
 * (unit transmitted power, isotropic antennas), incoherently to the bin of its time and
 * Doppler shift, to the bin of its time and delay tau = L / c, and to its time bin's total.
 * The outputs are cleared and then accumulated on `stream` with binary64 atomic additions,
 * so the order of the additions, and the last bits of a sum, can differ between calls.
 * Errors: DRT_E_INVAL for steps_per_bin < 1, a step that is not > 0, negative bin counts
 * or a NULL output whose count is nonzero (total may always be NULL). */
int drt_power_profiles(drt_ctx *ctx, uint32_t scene, int32_t n_rays, const drt_time_grid *tg,
                       double f_c, int32_t precision, const drt_bins *bins,
                       const drt_power_out *out, void *stream);

/* Time-variant transfer function H[j][k] = sum_r a_r(t_j) exp(-j 2 pi f_k L_r(t_j) / c)
 * for rays [0, n_rays), written to the device buffer H ([n_steps][n_sub], interleaved
 * complex128 for DRT_FP64, complex64 otherwise) on `stream`.  Deterministic: the same
 * inputs give bitwise the same H whatever else runs on the device. */
int drt_cfr(drt_ctx *ctx, uint32_t scene, int32_t n_rays, const drt_time_grid *tg,
            const drt_freq_grid *fg, int32_t precision, void *H, void *stream);

/* drt_cfr for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments, kernels and result
 * as drt_cfr (bitwise), but the call's scratch (pose table, ray-sum records, partial sums)
 * is one static device array of 256 MiB per GPU, set up by drt_create and held until the
 * process ends; the call makes no hipMalloc, hipFree or other allocating call.  Errors:
 * DRT_E_NOMEM when the call needs more than 256 MiB of scratch (about n_rays x n_steps x 32 B
 * of records plus, for many rays, a few n_steps x n_sub x 8 B partial sums; the urban
 * workload of 5000 rays x 1000 instants x 1024 subcarriers needs 201 MB); those of drt_cfr.
 * Every call on one GPU, from any context or thread, uses that GPU's one array: calls on one
 * stream are ordered and safe, calls that overlap on one GPU (other streams, other threads)
 * race and give wrong results. */
int drt_cfr_noalloc(drt_ctx *ctx, uint32_t scene, int32_t n_rays, const drt_time_grid *tg,
                    const drt_freq_grid *fg, int32_t precision, void *H, void *stream);

/* The same H as drt_cfr in binary64, by a type-1 non-uniform FFT along the subcarrier grid
 * (per instant about R w + 5 M log2 M operations instead of R K): per instant, each ray's
 * coefficient c = a exp(-j 2 pi frac(f_c L / c)) is spread at x = frac(df L / c) onto a
 * periodic grid of M points (the smallest power of two >= 2K and >= 2w) with an exponential-of-
 * semicircle kernel of w points (w = ceil(-log10 eps) + 1, 2..16, shape 2.30 w), the grid
 * is Fourier transformed and divided by the kernel's transform.  eps (1e-15 .. 1e-1) is the
 * target error of each H[j][k] relative to sum_r |a_r(t_j)|.  H: device [n_steps][n_sub]
 * complex128, on `stream`.  Errors: DRT_E_INVAL for n_sub > 2048 or eps out of range; those
 * of drt_cfr.  Deterministic up to the order of the atomic additions into the grid. */
int drt_cfr_nufft(drt_ctx *ctx, uint32_t scene, int32_t n_rays, const drt_time_grid *tg,
                  const drt_freq_grid *fg, double eps, void *H, void *stream);

/* Serving: enqueue one channel-prediction request (Sec. IV-D: the predicted channel is to be
 * served ahead of time to the network that asks for it; a request is the H(t, f) of
 * drt_cfr over its own horizon, band and rays).  Non-blocking.  DRT_E_ADMISSION if
 * its device footprint alone exceeds the cap; otherwise it waits in the queue until a
 * batch slot and memory free up.  A worker thread keeps up to four batches in flight, each
 * on its own stream: a free slot takes the queue head and, FIFO, the split-precision
 * requests behind it (at most 64 per batch, about 4e9 samples of work beyond the first,
 * arena within the HBM budget) and runs them as one replay of the slot's captured graph
 * of fused kernels (poses, geometry per signature class, ray sum per matrix tile shape,
 * partial-sum reduction), each one launch over the work items of every request in the
 * batch, its grid set to the batch's item count.  Binary64 requests, and ray sums off the matrix-core path, run alone on a
 * slot.  Each request's H is bitwise the one drt_cfr gives for it.  req->H is borrowed
 * until drt_poll reports done or an error. */
int drt_submit(drt_ctx *ctx, const drt_request *req, uint64_t *ticket);

/* Non-blocking status of a ticket (Sec. IV-D, the serving side of channel prediction); a
 * ticket reported done or failed is forgotten afterwards (DRT_E_NOTFOUND on the next poll).
 * A request whose arena cannot fit in the HBM cap even with nothing else running fails with
 * DRT_E_NOMEM (memory held by idle batch slots and by the per-stream scratch of the calls
 * above is given back first), so that the requests queued behind it proceed. */
int drt_poll(drt_ctx *ctx, uint64_t ticket, drt_req_stat *stat);

/* Serving counters since the context was created. */
typedef struct {
  int64_t batches;            /* graph replays of the fused batch kernels */
  int64_t batched_requests;   /* requests served inside those batches */
  int64_t single_launches;    /* requests served alone on a slot */
  int32_t max_batch;          /* largest batch so far */
  int32_t slots;              /* batches that can be in flight at once (0 before the first submit) */
  int64_t failed_nomem;       /* requests failed with DRT_E_NOMEM: no room even with nothing running */
} drt_serving_stats;
int drt_serving_stats_get(drt_ctx *ctx, drt_serving_stats *out);

/* Seconds on the clock used by drt_req_stat. */
double drt_now(void);

/* Kernel timing (tracing aid).  While enabled, drt_extrapolate and drt_cfr record a
 * hipEvent pair around each kernel they launch, on the caller's stream (around the
 * back-to-back per-signature-class kernels of the geometry step together), so the figures
 * are device durations of those kernels alone.  drt_profile_read waits for the recorded
 * events and returns the totals since the last reset; index with enum drt_kernel_id.
 * launches counts kernels, so ms / launches is the mean duration of one kernel. */
enum drt_kernel_id { DRT_K_POSE = 0, DRT_K_GEOM = 1, DRT_K_CFR = 2, DRT_K_REDUCE = 3, DRT_K_COUNT = 4 };
typedef struct {
  double ms[DRT_K_COUNT];          /* summed device milliseconds per kernel */
  int64_t launches[DRT_K_COUNT];   /* number of launches timed */
} drt_profile;
int drt_profile_enable(drt_ctx *ctx, int on);
int drt_profile_read(drt_ctx *ctx, drt_profile *out, int reset);

/* Text of a status code, and the detail of the calling thread's last error (error
 * reporting of the library itself; no passage of the paper defines it). */
const char *drt_strerror(int status);
const char *drt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DRT_H */

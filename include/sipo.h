/*
 * sipo.h -- C ABI of the MI355X (gfx950) SiPO hot path.
 *
 * SiPO (Woo, Lee, Taylor: "Scale-invariant projection optimization in
 * tomographic volumetric additive manufacturing") designs projection patterns
 * by solving a Charnes-Cooper linear program with a matrix-free PDHG method
 * (Sec. 2.6-2.8).  This library provides the operators of that solve and the
 * solve itself as hand-written HIP kernels:
 *
 *   sipo_backproject   P^T, projection -> voxel        (Eq. 2-3)
 *   sipo_project       P,   voxel -> projection        (Sec. 2.3, adjoint of P^T)
 *   sipo_blur          K,   object-space PSF           (Eq. 1-3)
 *   sipo_regions       gel / band / exterior labels    (Sec. 2.2, Fig. 2a)
 *   sipo_active_rays   active-ray mask                 (Sec. 2.2, Fig. 2b)
 *   sipo_pdhg_solve    the LP of Eq. 19-24 / 32-37 / 40-45 by PDHG (Sec. 2.8)
 *   sipo_response      material response M and its inverse (Eq. 4-5)
 *   sipo_evaluate      scale-invariant metrics and post-scaling (Eq. 6-8, 25-28, 46)
 *
 * Conventions shared by every call
 *   - Array pointers named "device" are HIP device pointers owned by the
 *     caller; the library never frees them and never keeps them after the
 *     call returns.  Pointers named "host" are ordinary host memory.
 *   - Volume layout: [nz][n][n], x fastest (row r = y, column c = x).
 *     Sinogram layout: [n_angles][nz][n_bins], bin fastest (one detector row
 *     per angle and slice).  Elements are float (SIPO_F32) or double
 *     (SIPO_F64) as fixed by the plan; labels and masks are uint8.
 *   - Geometry: the n x n grid covers [-1,1]^2 with voxel centres
 *     -1 + (c + 1/2) 2/n; voxels with centre outside the unit disk (the vial)
 *     receive no dose.  n_bins detector bins cover [-1,1].  A view at angle t
 *     sends light along (cos t, sin t); the detector coordinate of (x, y) is
 *     s = -x sin t + y cos t.  Each (voxel, view) pair has two linear-
 *     interpolation taps at bins floor(u) and floor(u)+1, u = (s+1) n_bins/2
 *     - 1/2, weighted by the Beer-Lambert factor
 *     exp(-atten (x cos t + y sin t + sqrt(1 - s^2))).  Slices are independent
 *     (parallel beam perpendicular to the rotation axis z).
 *   - Every operator call is asynchronous on the given HIP stream (NULL =
 *     default stream).  sipo_pdhg_solve returns after its stream finishes,
 *     because its results are host data.
 *   - Every call returns a sipo_status.  Argument errors (null pointers, bad
 *     sizes, in == out where forbidden, workspace too small) are detected
 *     before anything is launched.  HIP failures return SIPO_E_DEVICE.
 *     sipo_last_error() gives a thread-local message for the last failure.
 *     No exception or abort crosses this boundary.
 */
#ifndef SIPO_H
#define SIPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SIPO_OK = 0,
    SIPO_E_INVALID = -1,      /* bad argument; nothing was launched          */
    SIPO_E_DEVICE = -2,       /* a HIP call failed                           */
    SIPO_E_WORKSPACE = -3,    /* caller workspace smaller than required      */
    SIPO_E_UNSUPPORTED = -4   /* valid request the library does not support  */
} sipo_status;

typedef enum { SIPO_F32 = 0, SIPO_F64 = 1 } sipo_dtype;

/* Object and projection domains (Sec. 2.2, Fig. 2). */
typedef struct {
    int32_t n;               /* grid is n x n per slice, n >= 1                 */
    int32_t nz;              /* slices along the rotation axis, nz >= 1         */
    int32_t n_angles;        /* views, >= 1                                     */
    int32_t n_bins;          /* detector bins per row (the paper uses n), >= 1  */
    const double *angles;    /* host, n_angles view angles in radians           */
    double atten;            /* Beer-Lambert coefficient per vial radius, >= 0  */
} sipo_geometry;

/* Separable object-space PSF K (Eq. 1-3): normalised 1D taps per axis. */
typedef struct {
    int32_t rx, ry, rz;      /* tap radii (0 .. SIPO_MAX_PSF_RADIUS); 2r+1 taps  */
    const double *kx;        /* host, 2rx+1 taps along x (NULL iff rx == 0 -> 1) */
    const double *ky;        /* host, 2ry+1 taps along y                        */
    const double *kz;        /* host, 2rz+1 taps along z                        */
} sipo_psf;

#define SIPO_MAX_PSF_RADIUS 8

/* A plan binds a geometry, an optional PSF and an element type, and holds the
 * device-side tables the kernels need: view sines and cosines, the view walk
 * order and opposite-view pairs, the staged cross ranges of the 3D projector
 * and, for single-slice plans, the work-item lists of the 2D kernels.  These
 * tables are the only device memory the library keeps (sipo_plan_autotune
 * allocates temporary arrays and frees them before it returns); they are
 * created with the plan on the current device, freed by sipo_plan_destroy,
 * and sipo_plan_device_bytes reports their size.  The plan must be used on
 * that device only.
 * psf == NULL means K = I.  Errors: NULL pointers, sizes < 1 or above 16384
 * (65535 views), non-finite angles or taps, PSF radius above
 * SIPO_MAX_PSF_RADIUS (SIPO_E_INVALID); allocation failure (SIPO_E_DEVICE). */
typedef struct sipo_plan_s *sipo_plan;

int sipo_plan_create(const sipo_geometry *geom, const sipo_psf *psf, sipo_dtype dtype,
                     sipo_plan *plan_out);
int sipo_plan_destroy(sipo_plan plan);

/* Device bytes of the plan's own tables (0 for a NULL plan). */
size_t sipo_plan_device_bytes(sipo_plan plan);

/* Operator workspace (matrix-free operators on caller-owned arrays, Sec. 2.8).
 * sipo_project, sipo_backproject, sipo_active_rays and sipo_evaluate need
 * scratch device memory beyond their inputs and outputs: a 128 KiB reduction
 * area, and for single-slice and 3D plans a z-contiguous copy of the volume
 * (and, in 3D, of the sinogram) that the projector kernels read and write.
 * The caller provides it once per plan: sipo_plan_workspace_size gives the
 * bytes (128 KiB + one volume + one sinogram in 3D; 128 KiB + one slice for
 * single-slice plans), and sipo_plan_set_workspace attaches a device buffer of
 * at least that size, 256-byte aligned, owned by the caller and kept until it
 * is replaced, detached (workspace == NULL) or the plan is destroyed.  Calls
 * that need it return SIPO_E_WORKSPACE while none is attached.  Every call on
 * the plan uses the same workspace, so calls on one plan must be ordered (one
 * stream, or streams the caller synchronises): calls that overlap race.
 * sipo_pdhg_solve and sipo_blur do not use it.  Errors of set_workspace:
 * misaligned pointer (SIPO_E_INVALID), too small (SIPO_E_WORKSPACE); nothing
 * is changed on error. */
size_t sipo_plan_workspace_size(sipo_plan plan);
int sipo_plan_set_workspace(sipo_plan plan, void *workspace, size_t bytes);

/* Times the plan's kernel variants that compute the same result with
 * different work splits (slices per projector thread, slices per blur
 * workgroup) on scratch arrays of the plan's shape and keeps the fastest for
 * later calls.  Optional: a plan starts from built-in defaults, and results
 * do not depend on the choice beyond rounding order.  Allocates and frees its
 * scratch; synchronous on stream.  Not thread-safe against concurrent use of
 * the same plan. */
int sipo_plan_autotune(sipo_plan plan, void *stream);

/* The work-split settings sipo_plan_autotune chooses among, so that a caller
 * can keep a tuning and restore it on a later plan of the same geometry, or
 * pin one variant.  They change speed, not results beyond rounding order. */
typedef struct {
    int32_t p3d_zc;     /* slices per 3D projector thread: 8 or 16 (FP64); 8, 16, 32 or 64
                           (FP32; 64 with the asynchronous projector only)                       */
    int32_t p3d_dma;    /* 1 = 3D projector with asynchronous LDS staging (FP32 only, and only
                           where the plan's staged ranges allow it)                             */
    int32_t p3d_skip;   /* asynchronous projector: lanes skip candidates outside their ray (0/1) */
    int32_t p3d_cm;     /* asynchronous projector: march steps per staged chunk, 1 or 2 (1 with
                           64 slices per thread)                                                */
    int32_t blur_zc;    /* slices per blur workgroup: 0 (whole columns), 8, 16 or 32 (<= nz)     */
    int32_t bp3d_zc;    /* slices per 3D backprojector thread: 4, 8 or 16 (FP64); 4, 8, 16 or
                           32 (FP32)                                                            */
} sipo_tuning;

/* Current settings of the plan (defaults, autotuned or set).  Errors: NULL
 * arguments (SIPO_E_INVALID). */
int sipo_plan_get_tuning(sipo_plan plan, sipo_tuning *out);

/* Applies settings to the plan; all fields are checked first and nothing is
 * changed on error (SIPO_E_INVALID for values outside the lists above,
 * SIPO_E_UNSUPPORTED for an asynchronous projector the plan cannot use).
 * Fields that do not apply to the plan (a 2D plan's projector settings, the
 * blur of a plan without a PSF) are stored and ignored.  Not thread-safe
 * against concurrent use of the same plan. */
int sipo_plan_set_tuning(sipo_plan plan, const sipo_tuning *t);

/* vol (+)= P^T sino: backprojection, the geometric part of the dose model
 * f = A^T g = K P^T g (Eq. 2-3).  sino: device [n_angles][nz][n_bins];
 * vol: device [nz][n][n].  accumulate != 0 adds to vol, else overwrites.
 * sino and vol must not overlap.  3D plans use the plan workspace. */
int sipo_backproject(sipo_plan plan, const void *sino, void *vol, int accumulate, void *stream);

/* sino (+)= P vol: forward projection, the exact transpose of
 * sipo_backproject (Sec. 2.3).  vol: device [nz][n][n];
 * sino: device [n_angles][nz][n_bins].  Must not overlap.  Single-slice and
 * 3D plans use the plan workspace. */
int sipo_project(sipo_plan plan, const void *vol, void *sino, int accumulate, void *stream);

/* out = K in: the plan's separable PSF with zero boundary ("same" size).
 * K is symmetric, so this is also K^T (Eq. 51).  in, out: device
 * [nz][n][n], in != out.  With psf == NULL this is a copy. */
int sipo_blur(sipo_plan plan, const void *in, void *out, void *stream);

/* Region labels (Sec. 2.2, Fig. 2a): labels[i] = 2 where f_target[i] != 0
 * inside the vial (gel); 1 where i is inside the vial, not gel, and either
 * within Euclidean centre distance band_width (voxel units, 3D distance) of a
 * gel voxel or inside the PSF's box support around a gel voxel (band); 0
 * otherwise (exterior).  band_width < 0 means band-free (every non-gel vial
 * voxel is band); otherwise 0 <= band_width <= SIPO_MAX_BAND_WIDTH.
 * f_target: device [nz][n][n] in the plan dtype; labels and scratch: device
 * uint8 [nz][n][n] (scratch contents are overwritten). */
#define SIPO_MAX_BAND_WIDTH 11.0
int sipo_regions(sipo_plan plan, const void *f_target, double band_width, uint8_t *labels,
                 uint8_t *scratch, void *stream);

/* Active rays (Sec. 2.2, Fig. 2b): act[j] = 1 where (P f_target)_j exceeds
 * 1e-6 times its maximum, else 0.  scratch_sino: device sinogram of the plan
 * dtype used for P f_target (left holding it); act: device uint8 sinogram.
 * Uses the plan workspace. */
int sipo_active_rays(sipo_plan plan, const void *f_target, void *scratch_sino, uint8_t *act,
                     void *stream);

/* ------------------------------------------------- response and metrics --- */
/* Richards material response (Eq. 4): M(f) = alpha + (k - alpha) / [1 + exp(-beta (f - f0))]^(1/gamma).
 * The paper prints no resin constants; callers supply them. */
typedef struct {
    double alpha, k, beta, gamma, f0;
} sipo_resin;

/* out = M(in) (inverse == 0) or out = M^-1(in) (inverse != 0, Eq. 5) for every
 * voxel of a plan-shaped volume.  in, out: device volumes (may be equal).
 * M^-1 is defined for alpha < m < k; other inputs give NaN.  Errors: resin with
 * k == alpha, beta == 0 or gamma <= 0 (SIPO_E_INVALID). */
int sipo_response(sipo_plan plan, const sipo_resin *resin, const void *in, void *out, int inverse, void *stream);

/* Metrics of a normalised dose D = A^T y (Sec. 2.5, 2.6.3, Sec. 3):
 *   DTVR = max_gel(D / f~_T) / min_gel(D / f~_T)          (Eq. 6, 8)
 *   DSR  = max_band D / min_gel(D / f~_T)                 (Eq. 8)
 *   PSR_f = min_gel D / max_band D                        (Eq. 46)
 *   alpha_f = <D, f_T>_w / <D, D>_w over the gel, f_T = f_crit f~_T   (Eq. 27)
 * and, when a resin is given, the response-domain calibration
 *   alpha_m = argmin_{alpha > 0} sum_gel w (M(alpha D) - m_T)^2      (Eq. 28)
 * with PSR_m (Eq. 46) and DTVR_m = max_gel(m/m_T) / min_gel(m/m_T) at m = M(alpha_m D).
 * Empty band: DSR, PSR_f and PSR_m are NaN.  min_gel(D / f~_T) = 0: DTVR and DSR are +inf. */
typedef struct {
    double dtvr, dsr, psr_f;
    double gel_ratio_min, gel_ratio_max, band_max, gel_min;
    double alpha_f;
    double alpha_m, psr_m, dtvr_m;   /* NaN without a resin */
    int64_t n_gel, n_band;
} sipo_metrics;

/* dose: device volume (plan dtype); labels: device uint8 volume; f_target_norm:
 * device volume of f~_T or NULL (then f_t_scalar everywhere on the gel); f_crit:
 * physical critical dose (f_T = f_crit f~_T); weights: device volume or NULL (1);
 * resin, m_target (device volume or NULL -> m_t_scalar): response-domain terms,
 * skipped when resin is NULL.  Uses the plan workspace; synchronous on stream. */
int sipo_evaluate(sipo_plan plan, const void *dose, const uint8_t *labels, const void *f_target_norm,
                  double f_t_scalar, double f_crit, const void *weights, const sipo_resin *resin,
                  const void *m_target, double m_t_scalar, sipo_metrics *out, void *stream);

/* sipo_evaluate for callers that cannot allocate device memory or attach a
 * plan workspace (tight serving loops, harnesses that forbid allocation):
 * same arguments, checks and results as sipo_evaluate, bit for bit, but the
 * reduction partials live in a fixed 65,600-byte device array inside the
 * library instead of the plan workspace, so no workspace needs to be attached
 * and the call allocates nothing.  Every GPU that runs the library holds its
 * own copy of the array until the process ends; the call looks up the current
 * device's copy on its first use there.  The reduction uses at most 1024
 * workgroups for any volume, so no size exceeds the array (a size that did
 * would return SIPO_E_INVALID before any launch).  Each call overwrites the
 * whole area it reads, so no state carries over between calls, but all calls
 * on one GPU share the array: calls that overlap in time on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * Synchronous on stream. */
int sipo_evaluate_noalloc(sipo_plan plan, const void *dose, const uint8_t *labels, const void *f_target_norm,
                          double f_t_scalar, double f_crit, const void *weights, const sipo_resin *resin,
                          const void *m_target, double m_t_scalar, sipo_metrics *out, void *stream);

/* ------------------------------------------------------------------ LP --- */
/* The unified LP (Eq. 19-24; Case 1 Eq. 32-37; Case 2 Eq. 40-45):
 *     minimise   w1 u + w2 v
 *     subject to D_i <= u        on band   (u = band_cap when u_free == 0)
 *                D_i <= v U_i    on gel    (v = 1 when v_free == 0)
 *                D_i >= L_i      on gel
 *                y >= 0 on active rays, y = 0 on masked rays, u, v >= 0
 * where D = K P^T y is the normalised dose.  General LP: u_free = v_free = 1,
 * L = U = normalised target.  Case 1: w = (1,0), v_free = 0, L/U = tolerance
 * bounds.  Case 2: w = (0,1), u_free = 0, band_cap = 1, L = U = normalised
 * target. */
typedef struct {
    sipo_plan plan;            /* geometry, PSF, dtype                              */
    const uint8_t *labels;     /* device [nz][n][n]: 0 ext, 1 band, 2 gel           */
    const uint8_t *act;        /* device sinogram mask, 1 = active ray              */
    const void *lo;            /* device per-voxel L (plan dtype) or NULL           */
    const void *hi;            /* device per-voxel U (plan dtype) or NULL           */
    double lo_scalar;          /* L on every gel voxel when lo == NULL              */
    double hi_scalar;          /* U on every gel voxel when hi == NULL              */
    int32_t u_free, v_free;    /* 1 = scalar is an LP variable                      */
    double w1, w2;             /* objective weights (>= 0)                          */
    double band_cap;           /* u when u_free == 0                                */
    void *y;                   /* device in/out sinogram: warm start, then y*       */
    void *lam_up;              /* device in/out [nz][n][n]: lambda1 (band), lambda2 (gel) */
    void *lam_lo;              /* device in/out [nz][n][n]: lambda3 (gel)           */
    double u0, v0;             /* warm-start scalars (ignored when fixed)           */
    void *dose_out;            /* device [nz][n][n] or NULL: D = K P^T y* on return */
} sipo_problem;

/* PLAIN: Chambolle-Pock steps with scalar tau = sigma = 0.9/||G|| (FP64 power
 * iteration), no restarts, max_iters iterations, then a KKT evaluation.
 * RESTARTED: reflected Halpern PDHG with diagonal (Pock-Chambolle) steps, a
 * primal weight, KKT termination checks on the PDHG output every
 * check_every iterations, adaptive restarts and Farkas infeasibility tests
 * (prior art: PDLP, and Halpern/restart schemes for PDHG on LPs). */
typedef enum { SIPO_PDHG_PLAIN = 0, SIPO_PDHG_RESTARTED = 1 } sipo_pdhg_mode;

typedef struct {
    int32_t mode;              /* sipo_pdhg_mode                                          */
    int32_t max_iters;         /* iteration budget (>= 1)                                 */
    int32_t check_every;       /* KKT/restart check period (restarted mode; >= 1)         */
    double tol;                /* relative KKT tolerance (restarted mode), e.g. 1e-4      */
    double tau, sigma;         /* plain mode: > 0 overrides the 0.9/||G|| steps           */
    int32_t power_iters;       /* plain mode: power iterations for ||G|| (e.g. 100)       */
    double eta;                /* restarted mode step factor (< 1), e.g. 0.95             */
    double infeas_tol;         /* restarted mode Farkas test tolerance, e.g. 1e-6         */
    int32_t use_graph;         /* 1 = capture the iteration block in a HIP graph          */
    int32_t profile;           /* 1 = time every iteration launch with HIP events on the
                                  solve's stream (per-phase totals in the result); cannot
                                  be combined with use_graph                              */
    double scalar_weight;      /* restarted mode: column weight of the free scalars u, v in
                                  the diagonal steps, as a multiple c >= 0 of the mean row
                                  sum of their rows (0 = plain Pock-Chambolle, weight 1):
                                  tau_u = w_u / |band|, band rows sigma = 1/(R + w_u); the
                                  step bound holds for any positive weight               */
    int32_t progress_every;    /* restarted mode: > 0 writes one line to stderr every this
                                  many KKT checks, per unfinished instance (iterations,
                                  relative residuals, restarts); 0 = silent (>= 0)        */
    int32_t tune_operators;    /* 1 = at setup, time the work splits on this solve's own
                                  data and run the fastest: for batched single-slice FP32
                                  instances the 2D pair's work shapes (tiles_2d); in
                                  restarted mode for 3D instances the masked operators'
                                  splits on each instance's own masks (projector 8 / 16 /
                                  32 slices per thread, work queue, fused or separate
                                  primal step, candidate skipping; backprojector 4 / 8 /
                                  16 slices and 1 / 2 / 4 / 8 view splits; blur 4 / 8
                                  slices per chunk; tens of ms at 256^3).  Backprojector
                                  tiles and view splits set summation orders, so a tuned
                                  solve is reproducible bit for bit only with the same
                                  picks (op_config and tiles_2d in the result; pass them
                                  back to repeat it).  0 = fixed rules                     */
    int32_t op_config[8];      /* restarted mode, 3D instances: a nonzero entry fixes that
                                  work split of the masked operators, as reported in the
                                  result's op_config (projector slices per thread 8 / 16 /
                                  32, the last FP32 only; backprojector slices per thread
                                  4 / 8 / 16; backprojector view splits 1..8; blur slices
                                  per chunk 4 / 8 / 16; the projector's work queue: -1 =
                                  one workgroup per switched-on tile, k = 1..16 = a
                                  persistent grid of k workgroups per CU, at most as many
                                  as fit, taking the tiles longest step list first; the
                                  primal step: 1 = fused into the projector's output where
                                  its march is unsplit, -1 = its own kernel; the
                                  projector's lanes: 1 = skip the LDS reads of candidates
                                  out of their ray's reach, -1 = read them, which changes
                                  no result; the projector's listed march steps per staged
                                  chunk, 1 or 2 (2 halves its barriers; 32 slices always
                                  take 1; 0: 2 when every switched-on workgroup fits on the
                                  device at once with the larger ring), which changes no
                                  result where the march is unsplit); passing a
                                  tuned result's op_config back repeats that solve bit for
                                  bit.  Zero entries are tuned or follow the fixed rules (no
                                  queue, fused)                                            */
    int32_t tiles_2d[3];       /* batched single-slice instances: a nonzero entry fixes that
                                  work shape of the 2D pair (the backprojector's tile width
                                  16 / 32 / 64 voxels, with 256 / width rows; views per
                                  staged batch 8 / 16 / 32; the projector's bundle of 32 /
                                  64 / 128 bins by 256 / bins views); shapes other than
                                  32, 16, 64 need FP32.  With tune_operators the others
                                  are timed on the batch at setup (FP32)                   */
} sipo_pdhg_options;

/* Phases of one PDHG iteration, for sipo_pdhg_result.phase_ms. */
typedef enum {
    SIPO_PHASE_PROJECT = 0,     /* P (forward projection of K z)                           */
    SIPO_PHASE_BACKPROJECT = 1, /* P^T (of the new y)                                      */
    SIPO_PHASE_BLUR = 2,        /* both applications of K                                  */
    SIPO_PHASE_TRANSPOSE = 3,   /* layout changes between the volume kernels               */
    SIPO_PHASE_PRIMAL = 4,      /* projected primal step on rays                           */
    SIPO_PHASE_DUAL = 5,        /* fused dual step on voxels with its reductions           */
    SIPO_PHASE_SCALARS = 6,     /* scalar (u, v) step and reduction finish                 */
    SIPO_NUM_PHASES = 7
} sipo_phase;

typedef enum {
    SIPO_OPTIMAL = 0, SIPO_PRIMAL_INFEASIBLE = 1, SIPO_ITER_LIMIT = 2, SIPO_NUMERICAL = 3
} sipo_solve_status;

typedef struct {
    int32_t status;            /* sipo_solve_status                                       */
    int32_t iters, restarts;
    double primal_obj, dual_obj;
    double rel_primal, rel_dual, rel_gap;   /* relative KKT residuals of the returned point */
    double u, v;               /* returned scalars                                        */
    double tau, sigma;         /* plain mode scalar steps                                 */
    double omega;              /* restarted mode final primal weight                      */
    double time_ms;            /* wall time of the whole call (setup, iterations, final
                                  evaluation and copies back into the caller's arrays)      */
    double loop_ms;            /* time on the solve's stream of the iteration loop alone:
                                  from the first iteration launch (after the first graph
                                  capture) to the end of the last iteration block and its
                                  KKT / restart / infeasibility check; 0 if no iteration
                                  ran.  iters / loop_ms is the steady iteration rate        */
    double phase_ms[SIPO_NUM_PHASES];       /* profile mode: summed launch durations          */
    int32_t phase_launches[SIPO_NUM_PHASES]; /* profile mode: launches timed per phase        */
    int32_t op_config[8];      /* restarted mode, 3D instance: the masked operators' work
                                  splits as run (projector slices per thread,
                                  backprojector slices per thread, backprojector view
                                  splits, blur slices per chunk, projector work queue,
                                  primal step, candidate skipping and listed steps per
                                  chunk as in the options; the last 0 without step lists);
                                  zeros otherwise                                          */
    int32_t tiles_2d[3];       /* batched single-slice instances: the 2D pair's work shapes
                                  as run (as in the options); zeros otherwise              */
} sipo_pdhg_result;

/* Bytes of device workspace sipo_pdhg_solve needs for these problems. */
size_t sipo_pdhg_workspace_size(const sipo_problem *probs, int32_t n_probs,
                                const sipo_pdhg_options *opts);

/* Solve n_probs independent LPs.  workspace: device buffer of at least
 * sipo_pdhg_workspace_size bytes (contents ignored on entry).  results: host
 * array of n_probs.  An infeasible LP is not an error: its status is
 * SIPO_PRIMAL_INFEASIBLE and lam_up / lam_lo then hold the certificate
 * (a dual ray lambda >= 0 with P K z >= 0 on active rays and positive
 * dual objective; Supp. 6.1).  In restarted mode the warm-start multipliers
 * are tested first: if max(lambda, 0) on the regions already passes the
 * Farkas test at infeas_tol (for example the multipliers of the h_min LP,
 * min u s.t. D <= u on band and D >= L on gel, handed to a Case-2 LP whose
 * band cap is below that minimum), the instance returns at once with status
 * SIPO_PRIMAL_INFEASIBLE, iters = 0, that ray as its certificate and y and the
 * scalars as passed in.  Zero multipliers (a cold start) never pass.  At every
 * check the same test runs, in this order, on max(d, 0) for d = lambda(t) -
 * lambda(z) (one step), lambda(t) - lambda(t at the previous check), lambda(t)
 * itself, and lambda(t) - lambda at the last restart; the first that passes is
 * returned as the certificate.  The test normalises the ray to unit dual
 * objective and accepts it when its reduced-cost violations (the most
 * negative P K z on active rays; the band, resp. weighted gel, sum of a free
 * u, resp. v) are at most infeas_tol.
 * Returns after the stream has finished. */
int sipo_pdhg_solve(const sipo_problem *probs, int32_t n_probs, const sipo_pdhg_options *opts,
                    void *workspace, size_t ws_bytes, sipo_pdhg_result *results, void *stream);

/* Thread-local text for the last non-OK return of this thread. */
const char *sipo_last_error(void);

/* Library version string. */
const char *sipo_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SIPO_H */

/*
 * hc.h -- C ABI of the MI355X (gfx950) batched homotopy-continuation tracker.
 *
 * The library tracks many independent solution paths x(t), t in [0,1], of a
 * polynomial homotopy H(x,t) on one GPU and returns each path's endpoint and
 * status.  The operations follow Chien et al., "GPU-Based Homotopy Continuation
 * for Minimal Problems in Computer Vision":
 *   - section 3, Eq. (1): H(x,t) = (1-t) G(x) + t F(x) from a start system G whose
 *     solutions are known to the target F (here with a unit-modulus gamma on G);
 *   - section 6 (parallel evaluations): coefficients interpolated linearly between
 *     a start and a target instance, with dH/dt from the same terms and the
 *     coefficient differences;
 *   - section 3, Eqs. (2)-(4) and the 4th-order Runge-Kutta remark: predictor from
 *     the Davidenko equation H_x dx/dt = -H_t (Eq. 3);
 *   - section 3, Eqs. (5)-(6): Newton corrector at t + dt;
 *   - section 6 (linear system solver): LU with partial pivoting on [H_x | rhs].
 *
 * Conventions for every call:
 *   - Functions return hc_status; a negative value is an error, and the message
 *     of the last error on the calling thread is available from hc_last_error().
 *     On error no output buffer is written.
 *   - A per-path failure is not an error: it is reported in status[].
 *   - The caller owns every buffer passed in; the library copies what it needs.
 *   - Complex numbers are interleaved (re, im) doubles: hc_c64.
 *   - A context is not thread-safe: one host thread drives it at a time.
 */
#ifndef HC_H
#define HC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HC_MAX_N 32 /* largest number of unknowns the GPU path handles */
/* Size of the fixed device workspace of hc_track_device_noalloc (per device). */
#define HC_NOALLOC_SCRATCH_BYTES (64u << 20)

typedef struct {
    double re, im;
} hc_c64;

typedef enum {
    HC_OK = 0,
    HC_E_INVALID = -1,     /* bad argument (null pointer, size, malformed system)  */
    HC_E_OOM = -2,         /* device or host allocation failed                     */
    HC_E_DEVICE = -3,      /* a HIP runtime call failed                            */
    HC_E_UNSUPPORTED = -4  /* valid request outside what the GPU path implements   */
} hc_status;

/* Per-path outcome, written to status[]. */
typedef enum {
    HC_T_SUCCESS = 0,       /* reached t = 1, refined, finite, residual <= eta_max  */
    HC_T_AT_INFINITY = 1,   /* ||x||_inf exceeded inf_bound                          */
    HC_T_MIN_STEP = 2,      /* step size fell below h_min                            */
    HC_T_MAX_STEPS = 3,     /* accepted + rejected steps reached max_steps           */
    HC_T_SINGULAR = 4,      /* exactly singular Jacobian during endpoint refinement  */
    HC_T_NONFINITE = 5,     /* non-finite data (coefficients, start point, tangent)  */
    HC_T_REFINE_FAILED = 6, /* reached t = 1 but the residual stayed above eta_max   */
    HC_T_SINGULAR_END = 7   /* end-game (opts.endgame): a finite endpoint at which
                               the path has cycle number >= 2 (a singular root); the
                               endpoint is the end-game's estimate, not refined     */
} hc_track_status;

typedef enum {
    HC_FP64 = 0,  /* complex FP64 for every step                                    */
    HC_MIXED = 1  /* complex FP32 tracking up to t = 1 - t_end (FP64 t and step
                     size), then FP64 to t = 1 and FP64 refinement; a path FP32
                     cannot finish is re-tracked in FP64 from its last point      */
} hc_precision;

typedef enum {
    HC_TOTAL_DEGREE = 0, /* H = (1-t) gamma G + t F(x; c(p)), G_i = x_i^d_i - 1,
                            d_i = degree of equation i; start points generated      */
    HC_PARAMETER = 1     /* H = F(x; (1-t) c(p0) + t c(p1)), start points supplied   */
} hc_homotopy_kind;

/* Per-path counters, written to info[] when it is not NULL (32 bytes). */
typedef struct {
    int32_t steps;       /* accepted steps                                   */
    int32_t rejects;     /* rejected steps                                   */
    int32_t newton_its;  /* corrector iterations while tracking              */
    int32_t refine_its;  /* Newton iterations of the FP64 endpoint refinement */
    int32_t escalated;   /* 1 if the path was tracked in FP64 after starting
                            otherwise: mixed mode's hand-over, or a re-tracking
                            by the crossing check or the end-game            */
    int32_t cycle;       /* end-game cycle number (winding number) of the
                            path at t = 1; 0 where no end-game converged     */
    double residual;     /* relative backward error max_i |F_i| / sum_k |c_k||m_k|
                            at the endpoint; NaN when t = 1 was not reached */
} hc_track_info;

/* A square polynomial family F(x; p): n equations in n unknowns.
 * Term k lies in equation term_eq[k] and is c_k * prod_j x_j^term_exp[k*n + j].
 * Its coefficient is affine in the parameters p (length n_params):
 *   c_k(p) = coef_const[k] + sum_{e = coef_rowptr[k]}^{coef_rowptr[k+1]-1} coef_val[e] * p[coef_col[e]].
 * coef_const may be NULL (all zero).  coef_rowptr == NULL selects the identity
 * map c = p (then n_params must equal n_terms and coef_col/coef_val are ignored).
 * The GPU path takes terms of total degree <= 8 (degree <= 2 for the dense
 * table layout, see hc_layout) and needs every equation of degree >= 1. */
typedef struct {
    int32_t n;
    int32_t n_terms;
    const int32_t *term_eq;   /* [n_terms]            */
    const int32_t *term_exp;  /* [n_terms * n]        */
    int32_t n_params;
    int32_t kind;             /* hc_homotopy_kind     */
    const hc_c64 *coef_const; /* [n_terms] or NULL    */
    const int32_t *coef_rowptr; /* [n_terms + 1] or NULL */
    const int32_t *coef_col;  /* [nnz]                */
    const hc_c64 *coef_val;   /* [nnz]                */
} hc_system_desc;

/* Tracking options.  hc_default_opts() fills the values the CPU reference is run
 * with; the paper itself prints no step-control constants. */
typedef struct {
    double h0;          /* first step size                                     (0.05)  */
    double h_min;       /* a rejected step below this fails the path           (1e-7)  */
    double h_max;       /* largest step                                        (0.1)   */
    double beta_inc;    /* growth factor after n_inc consecutive accepts       (2)     */
    double beta_dec;    /* factor applied on a rejected step                   (0.5)   */
    double tau64;       /* FP64 corrector: ||dx||_2 <= tau (1 + ||x||_2)      (1e-6)  */
    double tau32;       /* FP32 corrector tolerance in mixed mode              (3e-4)  */
    double pred_tol;    /* first correction above pred_tol (1 + ||x||_2)
                           rejects the step (prediction too far off)          (1e-2)  */
    double tau_refine;  /* refinement stops when ||dx||_2 <= tau_refine (1+||x||_2) (1e-14) */
    double inf_bound;   /* ||x||_inf above this: path at infinity             (1e7)   */
    double eta_max;     /* largest residual accepted at the endpoint          (1e-10) */
    double t_end;       /* mixed mode: FP64 tracking on [1 - t_end, 1]         (0)     */
    int32_t precision;  /* hc_precision                                        (FP64)  */
    int32_t n_inc;      /* accepted steps before the step grows                (5)     */
    int32_t max_newton; /* corrector iterations per step                       (3)     */
    int32_t max_steps;  /* accepted + rejected steps per path; counted afresh
                           from a hand-over to FP64 (mixed mode) or a
                           crossing-check restart                             (5000)  */
    int32_t max_refine; /* endpoint Newton iterations                          (10)    */
    int32_t steps_per_launch; /* steps per path per kernel launch, 0 = to the end;
                                 -1 = the autotuner's choice if one applies, else
                                 0 (hc_autotune with -1 also tries chunked
                                 launches)                                        (0)     */
    int32_t tracks_per_item;  /* paths per wavefront work item, 0 = autotuned  (0)     */
    int32_t lanes_per_path;   /* 1: one path per lane; 4 or 8: one row of [H_x | rhs]
                                 per lane, 4 or 8 lanes per path (dense tables);
                                 term lists take 16 (n <= 16) or 32; 64: one path
                                 per wavefront, one entry of H_x per lane (dense
                                 total-degree tables, 2 <= n <= 8, FP64 only: the
                                 short-latency layout the crossing check's and the
                                 end-game's re-tracking use); 0 = autotuned   (0)     */
    int32_t use_graph;        /* hc_track_device: capture the launch sequence in a
                                 hipGraph on the first call and replay it while the
                                 arguments stay the same (needs a non-null stream,
                                 steps_per_launch 0, endgame 0, profiling off)  (0)     */
    int32_t fp64_residual;    /* mixed mode: the FP32 pass's Newton corrector evaluates
                                 H(x, t) in FP64 at an FP64 point (dense tables: from
                                 the FP32 coefficients; term lists: from the FP64
                                 tables) and solves with the FP32 LU (iterative
                                 refinement)                                      (0)     */
    int32_t crossing_check;   /* mixed mode: after refinement, paths of one instance
                                 that ended on the same root (relative distance
                                 <= 1e-8) start over in FP64; instances above 8192
                                 paths take 16 more workspace bytes per path  (1)     */
    int32_t per_instance_start; /* 1: every instance has its own start system:
                                 start is [n_inst][n_start][n] and, for
                                 HC_PARAMETER, p_start [n_inst][n_params] (the
                                 second leg of a piecewise-linear parameter path
                                 starts from the first leg's endpoints);
                                 hc_track and hc_track_device only           (0)     */
    int32_t table_layout;     /* hc_layout of the evaluation tables: 0 (AUTO) = the
                                 system's own; the other layout runs on a copy of
                                 the system in that layout, made on first use (an
                                 allocation); HC_E_UNSUPPORTED if that layout
                                 cannot hold the system; 0 = autotuned        (0)     */
    /* Power-series end-game (not in the paper; Morgan, Sommese and Wampler, Numer.
     * Math. 63, 1992).  With s = 1 - t a path near t = 1 is a power series in
     * s^(1/c) for its cycle number c.  A path that fails inside the zone
     * [1 - eg_s0, 1] (MIN_STEP, MAX_STEPS) or reaches t = 1 without a regular
     * endpoint (REFINE_FAILED, SINGULAR) is re-tracked in FP64 from its start point
     * and sampled at s_k = eg_s0 eg_beta^k, k >= 1 (in the zone with corrector
     * tolerance eg_tau, eg_max_newton iterations, minimum step eg_h_min); the
     * samples are taken in projective coordinates y = (1, x) / (a . (1, x)) on the
     * fixed patch a_j = exp(2 pi i frac((j + 1)(sqrt 5 - 1) / 2)), j = 0..n; from
     * every three in a row c is estimated from the decay of their differences and
     * y(0) extrapolated by the quadratic in s^(1/c) through them.  The end-game has
     * converged when two successive estimates agree to eg_tol |y|_inf, or to
     * eg_tol_inf |y|_inf with y_0 below |y|_inf / inf_bound (a path to infinity).
     * A converged path then ends AT_INFINITY (|x|_inf > inf_bound), with the usual
     * FP64 refinement and classification from the estimate (c = 1), or
     * SINGULAR_END at the estimate (c >= 2); an unconverged one keeps its first
     * result.  Not available in the batch and server calls. */
    int32_t endgame;          /* 0 off; 1 on for failed paths; 2 on for every path
                                 that reaches the zone and met no non-finite value (0) */
    int32_t eg_max_newton;    /* corrector iterations per step in the zone     (5)     */
    int32_t eg_max_samples;   /* samples s_1 .. s_K, K <= 64                   (16)    */
    int32_t eg_max_cycle;     /* largest cycle number                          (8)     */
    double eg_s0;             /* the zone is [1 - eg_s0, 1]                    (0.1)   */
    double eg_beta;           /* sample ratio s_(k+1) / s_k                    (0.25)  */
    double eg_tol;            /* convergence of successive estimates          (1e-9)  */
    double eg_tol_inf;        /* the same for a path to infinity              (1e-3)  */
    double eg_tau;            /* corrector tolerance in the zone               (1e-8)  */
    double eg_h_min;          /* smallest step in the zone                     (1e-14) */
} hc_opts;

typedef struct hc_ctx hc_ctx;
typedef struct hc_system hc_system;

/* Fills *o with the defaults listed above. */
void hc_default_opts(hc_opts *o);

/* Message of the last error raised on the calling thread ("" if none).  The
 * pointer stays valid until the next hc_* call on the same thread. */
const char *hc_last_error(void);

/* Creates a context bound to HIP device `device`.  *out is owned by the caller
 * and released with hc_destroy.  Errors: HC_E_INVALID (no such device),
 * HC_E_DEVICE, HC_E_OOM. */
hc_status hc_create(int device, hc_ctx **out);

/* Frees the context, its workspace and every system still loaded in it. */
void hc_destroy(hc_ctx *ctx);

/* Validates and copies a system description (a0: the evaluation tables of
 * section 6, compiled once per family) and uploads its tables to the device.
 * *out stays owned by the context until hc_free_system or hc_destroy.
 * Errors: HC_E_INVALID (malformed description), HC_E_UNSUPPORTED (n > HC_MAX_N,
 * a term of degree > 8, an equation of degree 0), HC_E_OOM, HC_E_DEVICE. */
hc_status hc_load_system(hc_ctx *ctx, const hc_system_desc *desc, hc_system **out);

/* Evaluation-table layout of a loaded system. */
typedef enum {
    HC_LAYOUT_AUTO = 0,   /* dense tables for n <= 8 and degree <= 2, else term
                             lists                                                */
    HC_LAYOUT_DENSE = 1,  /* every monomial of degree <= 2 gets a table slot
                             (c, L, Q per equation); n <= 8                       */
    HC_LAYOUT_TERMS = 2   /* per equation the list of its own terms (section 6's
                             term tables): c x_a x_b for degree <= 2 and n <= 16,
                             else up to 8 factors per term; n <= HC_MAX_N (the
                             paper's largest Jacobian, 32 x 32, section 1)       */
} hc_layout;

/* hc_load_system with an explicit table layout (hc_load_system uses
 * HC_LAYOUT_AUTO).  Both layouts compute the same homotopy; the term lists do
 * work in proportion to the terms a system has, the dense tables to n^3.
 * Errors: as hc_load_system, and HC_E_UNSUPPORTED for HC_LAYOUT_DENSE with n > 8
 * or a term of degree > 2, or an unknown layout. */
hc_status hc_load_system_layout(hc_ctx *ctx, const hc_system_desc *desc, int32_t layout, hc_system **out);

/* Releases a loaded system. */
hc_status hc_free_system(hc_ctx *ctx, hc_system *sys);

/* Number of unknowns and Bezout number prod_i d_i (the number of total-degree
 * start points) of a loaded system. */
hc_status hc_system_dims(const hc_system *sys, int32_t *n, int64_t *bezout);

/* Start points first .. first+count-1 of the total-degree start system
 * G_i = x_i^d_i - 1 (section 3: start solutions known in closed form).  Point b
 * writes b in mixed radix (d_1, ..., d_n), x_1 least significant, digits j_i,
 * and sets x_i = exp(2 pi i j_i / d_i).  out: host [count][n]. */
hc_status hc_total_degree_start(const hc_system *sys, int64_t first, int64_t count, hc_c64 *out);

/* Tracks n_start paths for each of n_inst target instances (host buffers).
 *   start:    [n_start][n] start points ([n_inst][n_start][n] with
 *             opts.per_instance_start); NULL for HC_TOTAL_DEGREE (then n_start
 *             must not exceed the Bezout number and path b starts at point b)
 *   p_start:  [n_params] start parameters ([n_inst][n_params] with
 *             opts.per_instance_start; HC_PARAMETER only, else NULL)
 *   p_target: [n_inst][n_params] target parameters
 *   gamma:    [n_inst] start-system multipliers (HC_TOTAL_DEGREE; NULL = 1)
 *   opts:     NULL = hc_default_opts
 * For HC_PARAMETER the coefficients move linearly from c(p_start) to
 * c(p_target[i]) (section 6); start and p_start are required, gamma is ignored,
 * and the one-path-per-lane layout (lanes_per_path = 1, or n = 1) is not
 * available (HC_E_UNSUPPORTED).
 * Outputs: endpoints [n_inst][n_start][n], status [n_inst][n_start], and
 * info [n_inst][n_start] when info != NULL.  Blocks until done.
 * Errors: HC_E_INVALID, HC_E_UNSUPPORTED, HC_E_OOM, HC_E_DEVICE. */
hc_status hc_track(hc_ctx *ctx, const hc_system *sys,
                   const hc_c64 *start, int32_t n_start,
                   const hc_c64 *p_start, const hc_c64 *p_target, int32_t n_inst,
                   const hc_c64 *gamma, const hc_opts *opts,
                   hc_c64 *endpoints, int32_t *status, hc_track_info *info);

/* Same as hc_track, but every array argument is a device pointer on the
 * context's device, and the work is enqueued on `stream` (a hipStream_t; NULL =
 * the null stream).  Returns once the work is enqueued unless
 * opts->steps_per_launch > 0 or opts->endgame is on, which need host round
 * trips between launches.
 * The outputs are valid after the stream has been synchronised.  The library's
 * workspace is reused by the next call on the same context. */
hc_status hc_track_device(hc_ctx *ctx, const hc_system *sys,
                          const hc_c64 *start, int32_t n_start,
                          const hc_c64 *p_start, const hc_c64 *p_target, int32_t n_inst,
                          const hc_c64 *gamma, const hc_opts *opts,
                          hc_c64 *endpoints, int32_t *status, hc_track_info *info,
                          void *stream);

/* hc_track_device for callers that cannot allocate device memory: code under
 * hipGraph stream capture, tight serving loops, hosts that forbid hipMalloc.
 * Same arguments, results and stream semantics as hc_track_device, but the path
 * state, the per-instance coefficient tables and the launch counters live in a
 * fixed device array of HC_NOALLOC_SCRATCH_BYTES per device, held by the
 * library from load until the process ends; the call makes no hipMalloc,
 * hipFree or other allocation.  Workspace of one call, in bytes (each part
 * rounded up to 256): 256 + n_inst n_start (16 n + 40) [+ 16 n_inst n_start in
 * mixed precision with n_start > 8192] [+ 4 n_inst n_start for dense
 * total-degree tables with 2 <= n <= 8] + (n_inst + P) n T (16, + 8 in mixed
 * precision), where T is the system's table slots per equation and P is 0 for
 * total degree, 1 for HC_PARAMETER (n_inst with per_instance_start); the
 * dense n = 8 batch of 512 x 256 paths takes about 27 MB.
 * Every call on a device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (two streams, two contexts, two
 * threads) race and corrupt each other's paths -- serialise them.  Kernels clear
 * what must start at zero themselves, so back-to-back calls on one stream are
 * safe.  Differences from hc_track_device: opts->use_graph is ignored (capture
 * the call instead), profiling is not recorded, the end-game (opts->endgame) is
 * not available, and a table_layout other than the system's own is served only
 * if hc_autotune or an earlier call already made that copy.
 * Errors: as hc_track_device; HC_E_UNSUPPORTED when the workspace exceeds
 * HC_NOALLOC_SCRATCH_BYTES (the message gives both sizes) or the table layout
 * would need a new copy. */
hc_status hc_track_device_noalloc(hc_ctx *ctx, const hc_system *sys,
                                  const hc_c64 *start, int32_t n_start,
                                  const hc_c64 *p_start, const hc_c64 *p_target, int32_t n_inst,
                                  const hc_c64 *gamma, const hc_opts *opts,
                                  hc_c64 *endpoints, int32_t *status, hc_track_info *info,
                                  void *stream);

/* Batched complex linear solves A_k x_k = b_k, k < batch (section 6, "Linear
 * System Solver": one fused kernel factors the augmented matrix [A_k | b_k] by
 * LU with partial pivoting, which carries out the triangular solve with L on
 * the way, and back-substitutes with the cached U).  The solver the path
 * trackers use, on its own: one system per group of 4, 8, 16 or 32 lanes (the
 * smallest >= n), one row per lane.
 *   n:      1..32
 *   fp32:   1: complex FP32 data and arithmetic (interleaved float pairs);
 *           0: complex FP64 (hc_c64)
 *   A:      [batch][n][n] row-major, element (i, j) of system k at k n^2 + i n + j
 *   b, x:   [batch][n]; x may not alias A or b
 *   info:   [batch] or NULL: 1 where a pivot is zero (x then holds inf/NaN), else 0
 * Device pointers on the context's device; enqueued on `stream` (NULL = the null
 * stream), outputs valid after it has been synchronised.  Allocates nothing.
 * Errors: HC_E_INVALID (n outside 1..32, batch < 0, a NULL array with
 * batch > 0), HC_E_DEVICE. */
hc_status hc_solve_batched_device(hc_ctx *ctx, int32_t n, int64_t batch, int32_t fp32, const void *A,
                                  const void *b, void *x, int32_t *info, void *stream);

/* Batched evaluation of a dense quadratic system and its Jacobian, FP32: the
 * evaluation step every tracking stage runs (section 3, Eq. (3)-(4): the
 * predictor and corrector need H and H_x; section 6: evaluation in parallel),
 * here of the target system F alone, at n_pts points of each of n_inst
 * instances.  Two engines compute the same numbers:
 *   HC_EVAL_ROWS (0): one Jacobian row per lane on the vector ALUs, the
 *       coefficients read from LDS (the trackers' own evaluation);
 *   HC_EVAL_MFMA (1): per instance, the n^2 x (n + 1) complex matrix of the
 *       rows' coefficients times the points' (x, 1) as FP32 matrix-core tiles
 *       (v_mfma_f32_16x16x4_f32; 16 points per wavefront), F by Euler's
 *       identity from the rows.
 *   sys:      a dense-table system (HC_LAYOUT_DENSE), 1 <= n <= 8
 *   p_target: device [n_inst][n_params] (hc_c64): each instance's coefficients
 *             or parameters, as in hc_track_device
 *   x:        device [n_inst][n_pts][n] complex FP32 (interleaved float pairs)
 *   F:        device [n_inst][n_pts][n] complex FP32: F_r(x)
 *   J:        device [n_inst][n_pts][n][n] complex FP32: dF_r / dx_a at r n + a
 *   repeat:   >= 1; every point is evaluated this many times and the outputs are
 *             one evaluation's (more than 1 only to time the arithmetic apart
 *             from the memory traffic)
 * Enqueued on `stream` (NULL = the null stream); the coefficient tables are
 * built in a context buffer (allocated or grown on first use).  Errors:
 * HC_E_INVALID (NULL arguments, negative sizes, n_pts > 2^30, repeat < 1, unknown engine),
 * HC_E_UNSUPPORTED (term-list system, n > 8), HC_E_DEVICE. */
enum { HC_EVAL_ROWS = 0, HC_EVAL_MFMA = 1 };
hc_status hc_eval_dense_device(hc_ctx *ctx, const hc_system *sys, const hc_c64 *p_target, int32_t n_inst,
                               const float *x, int32_t n_pts, int32_t engine, int32_t repeat, float *F,
                               float *J, void *stream);

/* Duplicate marking of a point set (the merge step of monodromy, which the paper
 * uses to compute its start systems, section 7): keep[i] = 1 unless an earlier
 * point j < i lies within the relative tolerance,
 *   max_k |x_ik - x_jk| <= tol max(1, |x_i|_inf, |x_j|_inf),
 * else 0.  Every point is compared with all earlier ones (not only the kept
 * ones): the two differ only where duplicates chain (a ~ b ~ c with a, c apart).
 *   points: device [count][n] (hc_c64), n in 1..64;  keep: device [count].
 * Enqueued on `stream` (NULL = the null stream); allocates nothing.
 * Errors: HC_E_INVALID, HC_E_DEVICE. */
hc_status hc_distinct_device(hc_ctx *ctx, int32_t n, int64_t count, const hc_c64 *points, double tol,
                             int32_t *keep, void *stream);

/* Diagnostic: the measured vector FMA rate of the context's device in TFLOP/s
 * (2 FLOP per FMA), the check of the peak the trackers' ALU roofline is quoted
 * against.  Every lane of 8 wavefronts per SIMD runs 16 independent FMA chains
 * on registers; fp64 = 1 times FP64 FMAs, fp64 = 0 plain FP32 FMAs (one value
 * per lane and instruction, as in the trackers: the library is built without
 * packed FP32).  Synchronous on the null stream; allocates and frees ~4 MB of
 * device memory.  Errors: HC_E_INVALID (NULL ctx or tflops), HC_E_DEVICE. */
hc_status hc_measure_vector_peak(hc_ctx *ctx, int32_t fp64, double *tflops);

/* One job of a batch: a loaded system, its start points and instances, and its
 * output buffers, with the meaning and layout of the hc_track arguments.  All
 * pointers are device pointers. */
typedef struct {
    const hc_system *sys;
    const hc_c64 *start;      /* [n_start][n] or NULL (total degree)          */
    int32_t n_start;
    int32_t n_inst;
    const hc_c64 *p_start;    /* [n_params] (HC_PARAMETER) or NULL           */
    const hc_c64 *p_target;   /* [n_inst][n_params]                          */
    const hc_c64 *gamma;      /* [n_inst] or NULL                            */
    hc_c64 *endpoints;        /* [n_inst][n_start][n]                        */
    int32_t *status;          /* [n_inst][n_start]                           */
    hc_track_info *info;      /* [n_inst][n_start] or NULL                   */
} hc_job;

/* Tracks every path of n_jobs jobs that may differ in system, n (2..HC_MAX_N),
 * table layout, kind, path count and instance count, with one persistent
 * kernel per table kind, homotopy kind and precision pass: its wavefronts pop
 * work items (job, instance, range of paths) from a device queue until it is
 * empty, larger n first.  Options are shared (opts->steps_per_launch must be 0
 * or -1, lanes_per_path 0, table_layout 0, per_instance_start 0).  With
 * opts->use_graph and a non-null stream, the launch sequence is captured in a
 * hipGraph on the first call and replayed by later calls with the same jobs
 * array contents, options, stream and systems (profiling off): the inputs may
 * change in place between calls, the job list may not.  Enqueued on `stream`;
 * outputs valid after the stream is synchronised.  Each job's results equal
 * those of hc_track_device on that job alone.
 * Errors: HC_E_INVALID, HC_E_UNSUPPORTED (n = 1, steps_per_launch > 0,
 * lanes_per_path = 1, per_instance_start), HC_E_OOM, HC_E_DEVICE. */
hc_status hc_track_batch_device(hc_ctx *ctx, int32_t n_jobs, const hc_job *jobs, const hc_opts *opts,
                                void *stream);

/* Autotuner: runs hc_track_device with each candidate work decomposition on
 * these inputs, times it with HIP events on `stream`, and writes the fastest
 * into *best (other fields copied from opts).  Candidates: the evaluation-table
 * layout (the system's own, and the other one where it can hold the system),
 * lanes per path (one row of [H_x | rhs] per lane, or one path per lane for
 * dense total-degree tables), paths per wavefront work item, and, when
 * opts->steps_per_launch is -1, steps per launch (0, 64, 512).  The choice is
 * remembered in the context under the workload's shape (device architecture,
 * table layout, homotopy kind, n, term count, degrees, precision, n_start,
 * n_inst) and used by later calls that leave table_layout, lanes_per_path and
 * tracks_per_item at 0 (steps_per_launch only where the call passes -1), on
 * any system of that shape.  When the environment variable HC_TUNE_CACHE named
 * a file at hc_create, the context loaded it then and hc_autotune rewrites it
 * with every choice made so far.  The output buffers hold the last trial's
 * results.  Errors: as hc_track_device; HC_E_INVALID if the cache file cannot
 * be written. */
hc_status hc_autotune(hc_ctx *ctx, const hc_system *sys, const hc_c64 *start, int32_t n_start,
                      const hc_c64 *p_start, const hc_c64 *p_target, int32_t n_inst, const hc_c64 *gamma,
                      const hc_opts *opts, hc_c64 *endpoints, int32_t *status, hc_track_info *info,
                      void *stream, hc_opts *best);

/* Writes every autotuner choice of the context to the text file `path`, one
 * per line ("<key> -> <layout> <lanes_per_path> <tracks_per_item>
 * <steps_per_launch>").  Errors: HC_E_INVALID (NULL argument, file not
 * writable). */
hc_status hc_tune_save(hc_ctx *ctx, const char *path);

/* Merges the choices stored in `path` (as written by hc_tune_save) into the
 * context; entries of another device architecture never match this device's
 * keys.  *n_loaded (may be NULL) receives the number of entries read.  Errors:
 * HC_E_INVALID (NULL argument, file not readable, a malformed line: then
 * nothing is merged). */
hc_status hc_tune_load(hc_ctx *ctx, const char *path, int32_t *n_loaded);

/* ---- serving: continuous batching of solve requests (host buffers) ---------- */

typedef struct hc_server hc_server;

typedef struct {
    int32_t max_inflight;       /* batches on the device at once, each with its own
                                   stream and workspace                      (3)     */
    int32_t max_batch_requests; /* requests per batch                        (64)    */
    int64_t hbm_budget;         /* device bytes for the requests in flight   (8 GiB) */
    hc_opts opts;               /* tracking options of every request (mixed precision) */
} hc_server_opts;

/* A start set (start points and start parameters) kept on the server's device
 * (hc_server_add_start_set). */
typedef struct hc_start_set hc_start_set;

/* One solve request: the hc_track arguments in host memory.  Inputs are copied
 * at submission; outputs are written when the request completes. */
typedef struct {
    const hc_system *sys;       /* loaded on the server's device (n >= 2)    */
    int32_t n_start;
    int32_t n_inst;
    const hc_c64 *start;        /* [n_start][n] or NULL (total degree)      */
    const hc_c64 *p_start;      /* [n_params] (HC_PARAMETER) or NULL        */
    const hc_c64 *p_target;     /* [n_inst][n_params]                       */
    const hc_c64 *gamma;        /* [n_inst] or NULL                         */
    hc_c64 *endpoints;          /* [n_inst][n_start][n]                     */
    int32_t *status;            /* [n_inst][n_start]                        */
    hc_track_info *info;        /* [n_inst][n_start] or NULL                */
    const hc_start_set *start_set; /* or NULL; when set, the request tracks from
                                   this resident set: start and p_start must be
                                   NULL and n_start the set's count         */
} hc_request;

typedef struct {
    int64_t submitted, completed, batches, tracks_completed;
    int64_t latencies;          /* completed requests submitted since the last reset */
    int64_t peak_bytes;         /* largest device footprint admitted at once         */
    double wall_s;              /* seconds since creation or the last reset          */
    double mean_ms, p50_ms, p99_ms, max_ms;  /* submission -> completion latency     */
} hc_server_stats;

/* Fills *o with the defaults listed above. */
void hc_server_default_opts(hc_server_opts *o);

/* Starts a server on ctx's device: a dispatcher thread forms batches from the
 * pending requests (first come first served, admitted while the device bytes of
 * the batches in flight stay within hbm_budget; a request larger than the budget
 * runs alone) and tracks each batch with hc_track_batch_device on a free slot, so
 * batches overlap on the device; a completion thread copies results out.  A
 * request's results equal those of tracking it alone.  The context must outlive
 * the server.  Errors: HC_E_INVALID, HC_E_UNSUPPORTED (opts.steps_per_launch > 0
 * or lanes_per_path = 1), HC_E_OOM, HC_E_DEVICE. */
hc_status hc_server_create(hc_ctx *ctx, const hc_server_opts *opts, hc_server **out);

/* Uploads start points [n_start][n] (and, for HC_PARAMETER, the start
 * parameters p_start [n_params]) of `sys` once; requests that name the returned
 * set track from them without copying them (resident start sets: the serving
 * loop's solve requests of one family share them).  The set lives on the
 * device until hc_server_destroy.  Thread-safe.  Errors: HC_E_INVALID (NULL
 * argument, n_start < 1, no p_start for a parameter homotopy, system on another
 * device), HC_E_OOM, HC_E_DEVICE. */
hc_status hc_server_add_start_set(hc_server *srv, const hc_system *sys, const hc_c64 *start, int32_t n_start,
                                  const hc_c64 *p_start, const hc_start_set **out);

/* Queues a request; *ticket identifies it.  Thread-safe.  The output buffers
 * must stay valid until the request completes.  Errors: HC_E_INVALID,
 * HC_E_UNSUPPORTED (n = 1), HC_E_OOM. */
hc_status hc_server_submit(hc_server *srv, const hc_request *req, int64_t *ticket);

/* *done = 1 once the request's outputs are written.  Returns the request's error
 * if it failed.  Thread-safe. */
hc_status hc_server_poll(hc_server *srv, int64_t ticket, int32_t *done);

/* Blocks until the request completes, then forgets the ticket.  Thread-safe. */
hc_status hc_server_wait(hc_server *srv, int64_t ticket);

/* Counters and latency percentiles since creation or the last reset. */
hc_status hc_server_get_stats(hc_server *srv, hc_server_stats *out);
hc_status hc_server_reset_stats(hc_server *srv);

/* Finishes every submitted request, stops the threads and frees the server. */
hc_status hc_server_destroy(hc_server *srv);

/* Event timings of the last hc_track / hc_track_device call on a context with
 * profiling switched on.  The times come from HIP events recorded on the stream
 * the kernels ran on; a "stage" is one evaluation of [H_x | rhs] plus one LU solve
 * for one path (inactive lanes are not counted). */
typedef struct {
    float ms_prep;          /* kernel-table preparation                     */
    float ms_init;          /* path-state initialisation                    */
    float ms_track_fp32;    /* mixed-mode tracking launches                 */
    float ms_track_fp64;    /* FP64 tracking launches                       */
    float ms_refine;        /* endpoint refinement and classification       */
    int32_t launches_fp32;
    int32_t launches_fp64;
    float ms_crossing;      /* mixed mode: crossing check, FP64 re-tracking of
                               crossed paths and their refinement           */
    int64_t stages_fp32;    /* stages run in FP32                           */
    int64_t stages_fp64;    /* stages run in FP64 (with the default lanes_per_path,
                               mixed mode runs the FP64 stages of its escalated
                               paths inside its own launches)                 */
} hc_profile;

/* Switches event timing and stage counting on (enable != 0) or off for the
 * following calls on this context.  It adds a few events and one atomic per
 * finished path; the kernels are the same. */
hc_status hc_set_profiling(hc_ctx *ctx, int32_t enable);

/* Waits for the events of the last profiled call and fills *out.  Errors:
 * HC_E_INVALID if no profiled call has been made on the context. */
hc_status hc_last_profile(hc_ctx *ctx, hc_profile *out);

/* Homogenised term tables in the form section 6 describes: each entry (an H_i
 * or a Jacobian entry) is a sum of K terms s * c[a] * x[m_1] * ... * x[m_M],
 * where x[n] is an auxiliary variable equal to 1 (pads terms of lower degree)
 * and missing terms have s = 0.  Input: n_entries polynomials in n variables,
 * entry e holding terms entry_ptr[e] .. entry_ptr[e+1]-1, term t being
 * scalar[t] * c[coef[t]] * prod_j x_j^exp[t*n + j].  K and M must be at least
 * the largest term count and degree.  Output out[e][k][2 + M] = (s, a, m_1..m_M),
 * 0-based indices, variables in ascending order; host memory.
 * Errors: HC_E_INVALID. */
hc_status hc_homogenize(int32_t n, int32_t n_entries, const int32_t *entry_ptr,
                        const int32_t *scalar, const int32_t *coef, const int32_t *exp,
                        int32_t K, int32_t M, int32_t *out);

#ifdef __cplusplus
}
#endif

#endif /* HC_H */

// hc_internal.h -- declarations shared by the host library (hc_api.cpp) and the
// gfx950 kernels (hc_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hc.h"

namespace hcx {

constexpr int kMaxN = HC_MAX_N;
constexpr int kMaxTermDeg = 8;  // factors per term-list slot (general-degree kinds)

// Terms of one dense quadratic equation in n unknowns: 1, x_1..x_n, x_a x_b (a <= b).
__host__ __device__ constexpr int dense_terms(int n) { return 1 + n + n * (n + 1) / 2; }

// Position of x_a x_b (a <= b) inside an equation's dense term list.
__host__ __device__ constexpr int quad_slot(int n, int a, int b)
{
    return 1 + n + a * n - a * (a - 1) / 2 + (b - a);
}

// Track status codes inside the SoA state: the public hc_track_status values
// (>= 0) are final; these two mean "still going".
constexpr int kRunning = -1;  // between launches or at the FP32/FP64 hand-over
constexpr int kReached = -2;  // at t = 1, waiting for refinement
constexpr int kDone = -3;     // refined; a re-tracking pass leaves it alone
constexpr int kRetrack = -4;  // endpoint coincides with another: start over in FP64
// Path state field `escal`: 0 while a path is tracked in the precision it
// started in; after a hand-over to FP64 (mixed precision) or a restart of the
// crossing check, 1 + the path's steps + rejects at that moment, so the FP64
// tracking gets the whole step budget again.
__host__ __device__ inline int steps_used(int steps, int rejects, int escal)
{
    return steps + rejects - (escal > 0 ? escal - 1 : 0);
}

// Largest n_start whose crossing check keeps the instance's projections in LDS;
// larger instances go through global memory (launch_dedup_big).
constexpr int kDedupMax = 8192;

// Mixed precision on the group trackers: 1 = a failed FP32 path goes on in FP64
// inside the same launch; 0 = it goes back to RUNNING and a second (FP64) launch
// takes it over.
#ifndef HC_INLINE_ESCALATION
#define HC_INLINE_ESCALATION 1
#endif
constexpr bool kInlineEsc = HC_INLINE_ESCALATION != 0;
constexpr double kCrossTol = 1e-8;  // endpoints this close (relative inf-norm) are one root

// Structure-of-arrays path state in HBM, path index fastest (coalesced when the
// lanes of a wavefront hold consecutive paths).  x is FP64 in both precisions.
struct TrackState {
    double *xr, *xi;   // [n][total]
    double *t, *h;     // [total]
    int *succ, *steps, *rejects, *nits, *status, *escal;  // [total]
};

// Per-instance coefficients in the layout the dense kernels read ("kernel
// tables"): for each equation i the dense term list as interleaved complex, with
// the coefficient of x_a^2 stored doubled (it enters dF_i/dx_a twice).
struct PrepArgs {
    int n, T, n_inst, n_params, n_slots;    // n_slots = n * T
    const int *slot_ptr;      // [n_slots + 1] CSR: terms feeding each slot
    const int *slot_term;     // [nnz_slot]
    const int *slot_mult;     // [nnz_slot] 1 or 2
    const double *term_const; // [n_terms][2] or null
    const int *map_ptr;       // [n_terms + 1] or null (identity)
    const int *map_col;
    const double *map_val;    // [nnz][2]
    const double *params;     // [n_inst][n_params][2]
    double *out64;            // [n_inst][n_slots][2]
    float *out32;             // [n_inst][n_slots][2] or null
};

struct InitArgs {
    int n, n_start;
    long long total;
    unsigned deg2;            // bit i: equation i has degree 2 (else 1)
    const int *eqdeg;         // or [n] equation degrees (any degree; overrides deg2)
    const double *start;      // [n_start][n][2] (per instance: [n_inst][n_start][n][2]) or
                              // null (total-degree points)
    int start_per_inst;       // start holds one set of start points per instance
    double h0;
    TrackState s;
    int retrack;              // only reset paths marked kRetrack, in FP64 (escal = 1)
};

// Crossing check after refinement (mixed mode): per instance, a SUCCESS endpoint
// equal to another one (relative inf-norm distance <= tol) is marked kRetrack;
// every other path kDone.
struct DedupArgs {
    int n, n_start, n_inst;
    long long total;
    double tol;
    const double *endpoints;  // [total][n][2]
    const int *status;        // [total] final statuses
    TrackState s;
    double *proj;             // [total][2] workspace of instances above kDedupMax paths, else null
};

struct TrackArgs {
    int n;                    // unknowns (the persistent tracker dispatches on it)
    const void *coef;         // [n_inst][n][T][2] in the tracking precision
    const void *coef0;        // parameter homotopy: start tables [n][T][2], else null
    long long coef0_stride;   // elements between instances' start tables (0: one shared)
    const double *coef64;     // group tracker in mixed mode: FP64 tables for the FP64 stage
    const double *coef0_64;   //   and the FP64 start tables of a parameter homotopy
    const double *gamma;      // [n_inst][2] or null (gamma = 1)
    unsigned deg2;
    int n_start, items_per_inst, tracks_per_item, n_items;
    long long total;          // n_inst * n_start: stride of the SoA arrays
    double t_final;           // 1, or 1 - t_end for the FP32 pass (lane tracker)
    double t_switch;          // group tracker, mixed mode: FP32 -> FP64 at this t (1 - t_end)
    double tau64;             // group tracker, mixed mode: tolerance of the FP64 stage
    int launch_steps;         // steps per path in this launch, 0 = unlimited
    int escalate;             // lane tracker's FP32 pass: failures go back to RUNNING for FP64
    int ir;                   // FP32 pass: FP64 right-hand side in Newton stages
    double h0, h_min, h_max, beta_inc, beta_dec, tau, pred_tol, inf2;
    int n_inc, max_newton, max_steps;
    TrackState s;
    unsigned *n_suspended;    // paths left RUNNING by launch_steps
    unsigned *head;           // k_track_grp: next work item (zeroed before each launch)
    const void *vars;         // term-list layout: [n][n_tslots] slot variables (16-bit a | b << 8,
                              //   or 64-bit factor bytes for the general-degree kinds)
    int n_tslots;             // term-list layout: slots per equation
    const int *sdeg;          // general-degree kinds: [n_tslots] largest degree of each slot
    const int *eqdeg;         // general-degree kinds: [n] degree of each equation
    unsigned long long *stage_count;  // or null: stages of active lanes, summed (lane tracker:
                                      // one counter; group tracker: [FP32, FP64] stages)
};

struct RefineArgs {
    const double *coef;       // FP64 kernel tables
    const double *gamma;
    unsigned deg2;
    int n_start;
    long long total;
    int max_refine;
    double tau_refine, inf2, eta_max;
    int eg_cycle;             // end-game pass: info.cycle = the path's cycle number (kept in succ)
    int singular_end;         // end-game pass: a finite endpoint within the bound ends
                              //   HC_T_SINGULAR_END whatever its residual
    TrackState s;
    double *endpoints;        // [total][n][2]
    int *status;              // [total]
    hc_track_info *info;      // [total] or null
    int n;                    // term-list layout: unknowns,
    int n_tslots;             //   slots per equation
    const void *vars;         //   the slots' variables
    const int *sdeg;          //   and, general degree, the slots' degrees
};

// Power-series end-game (hc_endgame.hip).  Candidates are compacted into
// list[0 .. *count); per candidate the last three samples of the path in
// projective coordinates (n + 1 complex values each) and the previous estimate
// live in ring / prev, and cls records the outcome: 0 pending or failed, 1 a
// finite estimate with cycle number 1 (to be refined), 2 a finite estimate with
// cycle number >= 2, 3 classified at infinity (written out at once).
constexpr int kEgMaxSamples = 64;
struct EgArgs {
    int n;
    long long total;
    TrackState s;
    int mode;                 // 1: failed paths; 2: every path that reached the zone
    double s0;
    int *list;                // [total] capacity
    unsigned *count;          // candidates found by k_eg_select
    int m;                    // candidates (host copy of *count) for the sampling kernels
    double *ring;             // [3][m][n + 1][2]
    double *prev;             // [m][n + 1][2]
    int *cls;                 // [m]
    int *have_prev;           // [m]
    int k;                    // sample index (>= 1)
    double t_k;               // 1 - s_k
    double beta, tol, tol_inf, inf_bound;
    int max_cycle;
    double *endpoints;        // outputs, for paths classified at infinity
    int *status;
    hc_track_info *info;
};
// Marks candidates kRetrack (and appends them to list), every other path kDone.
hipError_t launch_eg_select(const EgArgs &a, hipStream_t st);
// Takes sample k of every candidate that reached t_k and updates its estimate.
hipError_t launch_eg_sample(const EgArgs &a, hipStream_t st);
// Candidates of class `cls` go to refinement (kReached), all others kDone.
hipError_t launch_eg_mark(const EgArgs &a, int cls, hipStream_t st);

hipError_t launch_prep(const PrepArgs &a, hipStream_t st);
hipError_t launch_init(const InitArgs &a, hipStream_t st);
// fp32 selects the complex-FP32 tracker, else complex FP64.
hipError_t launch_track(int n, bool fp32, const TrackArgs &a, int waves_per_block, hipStream_t st);
// One entry of the persistent tracker's device work queue.
struct QueueItem {
    int job;   // index into the jobs' TrackArgs
    int inst;  // instance within the job
    int tb;    // first path
    int tend;  // one past the last path
};

// Persistent tracker over a work queue (group layout, n in 2..8): n_waves
// wavefronts pop items by atomicAdd on *head (zeroed by the caller).
hipError_t launch_track_queue(bool fp32, bool param, const TrackArgs *jobs, const QueueItem *items, int n_items,
                              unsigned *head, int n_waves, hipStream_t st);
int queue_waves(bool fp32, bool param);
// Sets count 32-bit words to value (graph-safe replacement for hipMemsetAsync).
hipError_t launch_fill_u32(unsigned *p, unsigned value, int count, hipStream_t st);

// G lanes per path (one row of [H_x | rhs] per lane); G = group_lanes(n).
// Persistent grid of resident wavefronts popping a.n_items work items from a.head
// (which must be zero at launch).
hipError_t launch_track_group(int n, bool fp32, const TrackArgs &a, hipStream_t st);
int group_lanes(int n);
// FP64 refinement of dense systems with 2 <= n <= 8 in the group layout: one job
// (many = false, *a read on the host) or count jobs (a in device memory);
// max_total = the largest path count of the jobs.
hipError_t launch_refine_group(int n, const RefineArgs *a, int count, long long max_total, bool many, hipStream_t st);

// Term-list layout (hc_terms_impl.h): kind tk = 5, 3 or 0 (degree <= 2,
// n <= 10, 14 or 16), 1 (any degree <= 8, n <= 16), 4 (any degree <= 8,
// n <= 18), 2 (any degree <= 8, n <= 20) or 6 (any degree <= 8, n <= 32); 16
// lanes per path for kinds 0, 1, 3 and 5, 32 for kinds 2, 4 and 6.
constexpr int kTermKindCount = 7;
constexpr int term_kind_lanes(int tk) { return tk == 2 || tk == 4 || tk == 6 ? 32 : 16; }
constexpr bool term_kind_general(int tk) { return tk == 1 || tk == 2 || tk == 4 || tk == 6; }
// Mixed precision on a term-list kind: escalation inside the FP32 launch (as on
// the dense tables) or in a second, FP64 launch.  Without the FP64 stage in its
// loop every term-list FP32 kernel fits 3 wavefronts per SIMD (168 VGPRs, 0-9
// spilled, FP32-sized LDS slices) instead of 2, which outweighs the second
// launch (4-view batch: 754 -> 559 ms per step; 3-view 104 -> 96 ms; trifocal
// -3.5%).  g16 keeps it inline: the 5-point batch is small for the device and
// lost 7% with a second launch.  Single-call tracking only: the batch tracker
// escalates inline on every kind.
constexpr bool term_kind_inline_esc(int tk) { return tk == 1; }
// The kind with the smallest solver that holds a term-list system.
constexpr int term_kind_for(int max_deg, int n)
{
    return n > 20         ? 6
           : max_deg <= 2 ? (n <= 10 ? 5 : n <= 14 ? 3 : n <= 16 ? 0 : n <= 18 ? 4 : 2)
                          : (n <= 16 ? 1 : n <= 18 ? 4 : 2);
}
hipError_t launch_track_terms(int tk, bool fp32, const TrackArgs &a, hipStream_t st);
hipError_t launch_track_queue_terms(int tk, bool fp32, bool param, const TrackArgs *jobs, const QueueItem *items,
                                    int n_items, unsigned *head, int n_waves, hipStream_t st);
int queue_waves_terms(int tk, bool fp32, bool param);
hipError_t launch_refine_terms(int tk, const RefineArgs &a, hipStream_t st);
hipError_t launch_refine_terms_many(int tk, const RefineArgs *a, int count, long long max_total, hipStream_t st);

// Fixed device workspace of hc_track_device_noalloc (hc_scratch.hip): one
// kScratchBytes array per device, its address looked up once per device by
// scratch_init (hc_create); scratch_ptr returns it (null before scratch_init).
constexpr size_t kScratchBytes = (size_t)HC_NOALLOC_SCRATCH_BYTES;
hipError_t scratch_init(int device);
void *scratch_ptr(int device);

// One path per wavefront, one Jacobian entry per lane (hc_wave.hip): dense
// total-degree tables, 2 <= n <= 8, FP64.  The RUNNING paths below a.t_final
// are compacted into list ([a.total] capacity; *count is cleared first) and
// `waves` wavefronts track them, one path each while there are no more.
hipError_t launch_track_wave(int n, const TrackArgs &a, int *list, unsigned *count, int waves, hipStream_t st);

// Duplicate marking of count points of n complex entries (hc_distinct.hip).
hipError_t launch_distinct(int n, long long count, const double *pts, double tol, int *keep, hipStream_t st);

// Batched FP32 evaluation of a dense quadratic system (tables as the trackers
// read them) and its Jacobian at n_pts points of each instance.
struct EvalArgs {
    int n, n_inst, n_pts, repeat;
    const float *tab;         // [n_inst][n][T][2] FP32 kernel tables
    const float *x;           // [n_inst][n_pts][n][2]
    float *F;                 // [n_inst][n_pts][n][2]
    float *J;                 // [n_inst][n_pts][n][n][2]: J[r][a] = dF_r / dx_a
};
// engine 0: one Jacobian row per lane (vector ALUs); 1: matrix cores
hipError_t launch_eval(const EvalArgs &a, int engine, hipStream_t st);

// Measured vector FMA rate (hc_peak.hip), TFLOP/s.
hipError_t measure_peak_fma(bool fp64, double *tflops, hipStream_t st);

// Standalone batched complex solves (hc_lu.hip): n <= 32, systems of one size.
hipError_t launch_lu_solve(int n, long long batch, bool fp32, const void *A, const void *b, void *x, int *info,
                           hipStream_t st);

// Per-kind entry points (one source file per kind).
template <int TK>
hipError_t launch_track_terms_k(bool fp32, const TrackArgs &a, hipStream_t st);
template <int TK>
hipError_t launch_track_queue_terms_k(bool fp32, bool param, const TrackArgs *jobs, const QueueItem *items,
                                      int n_items, unsigned *head, int n_waves, hipStream_t st);
template <int TK>
int queue_waves_terms_k(bool fp32, bool param);
template <int TK>
hipError_t launch_refine_terms_k(const RefineArgs *a, int count, long long max_total, bool many, hipStream_t st);
hipError_t launch_refine(int n, const RefineArgs &a, hipStream_t st);
hipError_t launch_dedup(const DedupArgs &a, hipStream_t st);
// The crossing check of one job whose instances have more than kDedupMax paths
// (a.proj must hold a.total complex values).
hipError_t launch_dedup_big(const DedupArgs &a, hipStream_t st);
// Batch API: one launch per step over many jobs (argument arrays in device memory).
hipError_t launch_prep_many(const PrepArgs *a, int count, long long max_work, hipStream_t st);
hipError_t launch_init_many(const InitArgs *a, int count, long long max_total, hipStream_t st);
// Jobs above kDedupMax paths per instance are skipped: launch_dedup_big each.
hipError_t launch_dedup_many(const DedupArgs *a, int count, int max_inst, int max_start, hipStream_t st);
// max_items: the largest n_inst * ceil(n_start / 64) of the jobs (n = 1), max_total
// the largest path count (2 <= n <= 8)
hipError_t launch_refine_many(int n, const RefineArgs *a, int count, long long max_items, long long max_total,
                              hipStream_t st);

}  // namespace hcx

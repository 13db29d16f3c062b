// hc_kernels.hip -- gfx950 kernels of the batched homotopy-continuation tracker.
//
// Layout and mapping (one path per lane, "64 tracks per wavefront"):
//   * A wavefront owns a work item = (instance, range of start points).  All 64
//     lanes work on the same instance, so every coefficient read is wavefront-
//     uniform: the coefficients are fetched with scalar loads into SGPRs and fed
//     straight into the VALU FMAs (no LDS traffic, no per-lane copies).
//   * Each lane holds one path's whole working set in VGPRs: the point, the RK4
//     accumulator and the n x (n+1) augmented matrix [H_x | rhs], factored by
//     partial-pivot LU entirely in registers.
//   * Every loop iteration performs exactly one "stage" for every lane: evaluate
//     H_x and one right-hand side at the lane's own (x, t), then solve.  What the
//     stage means (RK4 node 1..4, or a Newton correction) is per-lane state, so
//     lanes at different phases of different steps never diverge in the
//     expensive part.  A lane whose path ends takes the next start point of the
//     work item (lane refill), so short paths do not idle the lane.
//   * Path state between launches lives in HBM as structure-of-arrays.
//
// Method (Chien et al., section 3 and section 6): H = (1-t) gamma G + t F with
// G_i = x_i^d_i - 1; tangent from H_x dx/dt = -H_t (Eq. 3); classic RK4
// predictor; Newton corrector at t + h (Eqs. 5-6); LU with partial pivoting on
// the augmented matrix [H_x | rhs], back substitution with U.
#include "hc_device.h"

namespace hcx {

// ---------------------------------------------------------------- evaluation

// Builds the augmented matrix [H_x | rhs] at (x, t) for the total-degree
// homotopy H = (1-t) gamma G + t F, G_i = x_i^d_i - 1 (d_i in {1, 2}):
//   H_x = t F_x + (1-t) gamma diag(G'),
//   rhs = -H_t = -(F - gamma G)      for a predictor stage (Eq. 3),
//   rhs = -H   = -((1-t) gamma G + t F) for a corrector stage (Eq. 6).
// F is a dense quadratic in the kernel-table layout: per equation the constant,
// the n linear coefficients L and the upper-triangular quadratic coefficients q
// (q_aa doubled), so dF_i/dx_j = L_j + sum_a q_(j,a) x_a.  F itself comes from
// Euler's identity for polynomials of degree <= 2:
//   F_i = c_i + (L_i . x + x . J_i) / 2,
// which reuses the Jacobian row instead of re-summing the monomials.
template <int N, typename R>
__device__ __forceinline__ void build_td(tbl_ptr<R> cf, cx<R> gam, unsigned deg2,
                                         const cx<R> (&x)[N], R t, bool pred,
                                         cx<R> (&A)[N][N + 1])
{
    constexpr int T = dense_terms(N);
    const R omt = R(1) - t;
#pragma unroll
    for (int i = 0; i < N; i++) {
        const tbl_ptr<R> c = cf + 2 * T * i;
        cx<R> Lx = {R(0), R(0)};
#pragma unroll
        for (int j = 0; j < N; j++) {
            cx<R> L = ldc(c, 1 + j);
            A[i][j] = L;
            Lx = cfma(L, x[j], Lx);
        }
#pragma unroll
        for (int a = 0; a < N; a++) {
#pragma unroll
            for (int b = a; b < N; b++) {
                cx<R> q = ldc(c, quad_slot(N, a, b));
                if (a == b) {
                    A[i][a] = cfma(q, x[a], A[i][a]);
                } else {
                    A[i][a] = cfma(q, x[b], A[i][a]);
                    A[i][b] = cfma(q, x[a], A[i][b]);
                }
            }
        }
        cx<R> s = Lx;
#pragma unroll
        for (int j = 0; j < N; j++) s = cfma(x[j], A[i][j], s);
        cx<R> c0 = ldc(c, 0);
        cx<R> F = {fma(R(0.5), s.re, c0.re), fma(R(0.5), s.im, c0.im)};

        const bool d2 = (deg2 >> i) & 1u;
        cx<R> G, dG;
        if (d2) {
            G = cmul(x[i], x[i]);
            G.re -= R(1);
            dG = {R(2) * x[i].re, R(2) * x[i].im};
        } else {
            G = {x[i].re - R(1), x[i].im};
            dG = {R(1), R(0)};
        }
        const cx<R> gG = cmul(gam, G);
        const cx<R> gdG = cmul(gam, dG);
#pragma unroll
        for (int j = 0; j < N; j++) A[i][j] = cscale(t, A[i][j]);
        A[i][i].re = fma(omt, gdG.re, A[i][i].re);
        A[i][i].im = fma(omt, gdG.im, A[i][i].im);
        const cx<R> Ht = {F.re - gG.re, F.im - gG.im};
        const cx<R> H = {fma(t, F.re, omt * gG.re), fma(t, F.im, omt * gG.im)};
        A[i][N].re = pred ? -Ht.re : -H.re;
        A[i][N].im = pred ? -Ht.im : -H.im;
    }
}

// ---------------------------------------------------------------- linear solve

// Gaussian elimination with partial pivoting on the augmented matrix [A | b]
// held in registers (section 6): the pivot of column k is the row r >= k with
// the largest |Re| + |Im| (lowest row on ties); the row interchange is done with
// per-lane selects since each lane pivots its own matrix; eliminating below the
// pivot also transforms b, and back substitution with the cached U and the
// pivot reciprocals gives x.  Returns true if some pivot is exactly zero.
template <int N, typename R>
__device__ __forceinline__ bool lu_solve(cx<R> (&A)[N][N + 1], cx<R> (&x)[N])
{
    bool sing = false;
    cx<R> inv[N];
#pragma unroll
    for (int k = 0; k < N; k++) {
        R best = abs1(A[k][k]);
        int p = k;
#pragma unroll
        for (int r = k + 1; r < N; r++) {
            const R v = abs1(A[r][k]);
            const bool g = v > best;
            best = g ? v : best;
            p = g ? r : p;
        }
        sing |= (best == R(0));
#pragma unroll
        for (int r = k + 1; r < N; r++) {
            const bool s = (p == r);
#pragma unroll
            for (int c = k; c <= N; c++) {
                const cx<R> u = A[k][c], w = A[r][c];
                A[k][c].re = s ? w.re : u.re;
                A[k][c].im = s ? w.im : u.im;
                A[r][c].re = s ? u.re : w.re;
                A[r][c].im = s ? u.im : w.im;
            }
        }
        inv[k] = crecip(A[k][k]);
#pragma unroll
        for (int r = k + 1; r < N; r++) {
            const cx<R> l = cmul(A[r][k], inv[k]);
#pragma unroll
            for (int c = k + 1; c <= N; c++) A[r][c] = cfms(l, A[k][c], A[r][c]);
        }
    }
#pragma unroll
    for (int k = N - 1; k >= 0; k--) {
        cx<R> s = A[k][N];
#pragma unroll
        for (int c = k + 1; c < N; c++) s = cfms(A[k][c], x[c], s);
        x[k] = cmul(s, inv[k]);
    }
    return sing;
}

// ---------------------------------------------------------------- tracker

template <int N, typename R>
__global__ __launch_bounds__(256) void k_track(const TrackArgs a)
{
    constexpr int T = dense_terms(N);
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int item = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * wpb + wib);
    if (item >= a.n_items) return;
    const int inst = item / a.items_per_inst;
    const int tb = (item - inst * a.items_per_inst) * a.tracks_per_item;
    const int tend = min(tb + a.tracks_per_item, a.n_start);
    const R *__restrict__ cf = static_cast<const R *>(a.coef) + (size_t)inst * N * T * 2;
    cx<R> gam = {R(1), R(0)};
    if (a.gamma) gam = {R(a.gamma[2 * inst]), R(a.gamma[2 * inst + 1])};
    const long long gbase = (long long)inst * a.n_start;
    const long long total = a.total;
    const TrackState S = a.s;
    const R tau = R(a.tau), pred_tol = R(a.pred_tol);

    int trk = -1;
    long long g = 0;
    cx<R> x[N], xe[N], acc[N];
#pragma unroll
    for (int j = 0; j < N; j++) x[j] = xe[j] = acc[j] = {R(1), R(0)};
    double t = 0.0, h = 0.0, te = 0.0, hu = 0.0, tn = 0.0;
    int phase = 0, nit = 0, succ = 0, steps = 0, rejects = 0, nits = 0, lsteps = 0, escal = 0;
    unsigned lstages = 0;  // stages of the current path in this launch (profiling)
    int next = tb;

    auto save = [&](int st) {
#pragma unroll
        for (int j = 0; j < N; j++) {
            S.xr[j * total + g] = (double)x[j].re;
            S.xi[j * total + g] = (double)x[j].im;
        }
        S.t[g] = t;
        S.h[g] = h;
        S.succ[g] = succ;
        S.steps[g] = steps;
        S.rejects[g] = rejects;
        S.nits[g] = nits;
        S.escal[g] = escal;
        S.status[g] = st;
        if (a.stage_count) atomicAdd(a.stage_count, (unsigned long long)lstages);
        lstages = 0;
        trk = -1;
    };
    auto finish = [&](int st) {
        if (a.escalate && st != HC_T_AT_INFINITY) {
            // FP32 could not finish this path: hand it to FP64 from the last
            // accepted point with a fresh step size.
            escal = steps + rejects + 1;
            h = a.h0;
            succ = 0;
            st = kRunning;
        }
        save(st);
    };
    auto start_step = [&]() {
        if (steps_used(steps, rejects, escal) >= a.max_steps) {
            finish(HC_T_MAX_STEPS);
            return;
        }
        const double rem = a.t_final - t;
        if (h >= rem) {
            hu = rem;
            tn = a.t_final;
        } else {
            hu = h;
            tn = t + h;
        }
        phase = 0;
#pragma unroll
        for (int j = 0; j < N; j++) xe[j] = x[j];
        te = t;
    };
    auto refill = [&]() {
        for (;;) {
            const unsigned long long need = ballot(trk < 0);
            if (need == 0ull || next >= tend) break;
            const int cand = next + lanes_below(need);
            next += __popcll(need);
            if (trk < 0 && cand < tend) {
                const long long gg = gbase + cand;
                // still going, not yet at this pass's end time, and (in the FP32
                // pass) not already handed over to FP64
                if (S.status[gg] == kRunning && S.t[gg] < a.t_final && !(a.escalate && S.escal[gg])) {
                    trk = cand;
                    g = gg;
#pragma unroll
                    for (int j = 0; j < N; j++) x[j] = {R(S.xr[j * total + g]), R(S.xi[j * total + g])};
                    t = S.t[g];
                    h = S.h[g];
                    succ = S.succ[g];
                    steps = S.steps[g];
                    rejects = S.rejects[g];
                    nits = S.nits[g];
                    escal = S.escal[g];
                    lsteps = 0;
                    start_step();
                }
            }
        }
    };
    auto end_of_step = [&]() {
        if (a.launch_steps > 0 && lsteps >= a.launch_steps) {
            atomicAdd(a.n_suspended, 1u);
            save(kRunning);
        } else {
            start_step();
        }
    };

    refill();
    while (ballot(trk >= 0) != 0ull) {
        const bool act = trk >= 0;
        const bool pred = phase < 4;
        // Re-derive the table pointer each stage: otherwise the compiler hoists
        // every (loop-invariant) coefficient load out of the loop and parks the
        // whole table in VGPRs.  Streamed per stage, the loads stay scalar.
        const R *cfs = cf;
        asm volatile("" : "+s"(cfs));
        cx<R> A[N][N + 1];
        build_td<N, R>(as_table(cfs), gam, a.deg2, xe, R(te), pred, A);
        cx<R> dx[N];
        const bool sing = lu_solve<N, R>(A, dx);

        if (act) {
            lstages++;
            bool reject = false, accept = false;
            if (phase < 4) {
                bool dx_ok = true;
#pragma unroll
                for (int j = 0; j < N; j++) dx_ok = dx_ok && finite(dx[j]);
                if (sing) {
                    reject = true;
                } else if (phase == 0 && !dx_ok) {
                    finish(HC_T_NONFINITE);
                } else {
                    const R half = R(0.5 * hu), full = R(hu);
                    if (phase == 0) {
#pragma unroll
                        for (int j = 0; j < N; j++) {
                            acc[j] = dx[j];
                            xe[j] = {fma(half, dx[j].re, x[j].re), fma(half, dx[j].im, x[j].im)};
                        }
                        te = t + 0.5 * hu;
                    } else if (phase == 1 || phase == 2) {
                        const R c = phase == 1 ? half : full;
#pragma unroll
                        for (int j = 0; j < N; j++) {
                            acc[j] = {fma(R(2), dx[j].re, acc[j].re), fma(R(2), dx[j].im, acc[j].im)};
                            xe[j] = {fma(c, dx[j].re, x[j].re), fma(c, dx[j].im, x[j].im)};
                        }
                        te = phase == 1 ? t + 0.5 * hu : tn;
                    } else {
                        const R sixth = R(hu / 6.0);
#pragma unroll
                        for (int j = 0; j < N; j++) {
                            acc[j] = {acc[j].re + dx[j].re, acc[j].im + dx[j].im};
                            xe[j] = {fma(sixth, acc[j].re, x[j].re), fma(sixth, acc[j].im, x[j].im)};
                        }
                        te = tn;
                        nit = 0;
                        if (a.max_newton <= 0) reject = true;
                    }
                    phase++;
                }
            } else {
                if (sing) {
                    reject = true;
                } else {
                    R nd = R(0), nx = R(0);
#pragma unroll
                    for (int j = 0; j < N; j++) {
                        xe[j] = {xe[j].re + dx[j].re, xe[j].im + dx[j].im};
                        nd += abs2(dx[j]);
                        nx += abs2(xe[j]);
                    }
                    nd = sqrt(nd);
                    nx = sqrt(nx);
                    nit++;
                    nits++;
                    if (nit == 1 && !(nd <= pred_tol * (R(1) + nx)))
                        reject = true;
                    else if (nd <= tau * (R(1) + nx))
                        accept = true;
                    else if (nit >= a.max_newton)
                        reject = true;
                }
            }
            if (accept) {
                R big = R(0);
#pragma unroll
                for (int j = 0; j < N; j++) {
                    x[j] = xe[j];
                    big = fmax(big, abs2(x[j]));
                }
                t = tn;
                steps++;
                lsteps++;
                if (++succ >= a.n_inc) {
                    h = fmin(h * a.beta_inc, a.h_max);
                    succ = 0;
                }
                if (!((double)big <= a.inf2))
                    finish(isnan(big) ? HC_T_NONFINITE : HC_T_AT_INFINITY);
                else if (t >= a.t_final)
                    save(a.t_final >= 1.0 ? kReached : kRunning);
                else
                    end_of_step();
            } else if (reject) {
                rejects++;
                lsteps++;
                succ = 0;
                h *= a.beta_dec;
                if (h < a.h_min)
                    finish(HC_T_MIN_STEP);
                else
                    end_of_step();
            }
        }
        refill();
    }
}

// ---------------------------------------------------------------- init (a1)

__device__ __forceinline__ void init_body(const InitArgs &a, long long g)
{
    if (g >= a.total) return;
    const long long b = g % a.n_start;
    const TrackState S = a.s;
    if (a.retrack && S.status[g] != kRetrack) return;
    if (a.start) {
        const long long sb = a.start_per_inst ? g : b;  // g = instance * n_start + b
        for (int j = 0; j < a.n; j++) {
            S.xr[j * a.total + g] = a.start[(sb * a.n + j) * 2];
            S.xi[j * a.total + g] = a.start[(sb * a.n + j) * 2 + 1];
        }
    } else {
        // total-degree start point b: mixed-radix digits over (d_1..d_n), x_1
        // least significant, digit k of equation j giving the root of unity
        // exp(2 pi i k / d_j); with d_j in {1, 2} (deg2 mask) they are +-1.
        long long r = b;
        for (int j = 0; j < a.n; j++) {
            double vr = 1.0, vi = 0.0;
            if (a.eqdeg) {
                const int d = a.eqdeg[j];
                const long long k = r % d;
                r /= d;
                if (2 * k == d) {
                    vr = -1.0;
                } else if (k != 0) {
                    sincospi(2.0 * (double)k / (double)d, &vi, &vr);
                }
            } else if ((a.deg2 >> j) & 1u) {
                vr = (r & 1) ? -1.0 : 1.0;
                r >>= 1;
            }
            S.xr[j * a.total + g] = vr;
            S.xi[j * a.total + g] = vi;
        }
    }
    S.t[g] = 0.0;
    S.h[g] = a.h0;
    S.succ[g] = 0;
    if (!a.retrack) {
        S.steps[g] = 0;
        S.rejects[g] = 0;
        S.nits[g] = 0;
    }
    // a restarted path tracks in FP64 with a fresh step budget
    S.escal[g] = a.retrack ? 1 + S.steps[g] + S.rejects[g] : 0;
    S.status[g] = kRunning;
}

__global__ void k_init(const InitArgs a) { init_body(a, (long long)blockIdx.x * blockDim.x + threadIdx.x); }

// One launch for many jobs (batch API): job blockIdx.y, its blocks along x.
__global__ void k_init_many(const InitArgs *a)
{
    init_body(a[blockIdx.y], (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------- crossing check

// One block per instance.  Two paths of one instance that end on the same root
// have crossed (one jumped onto the other's path); both start over in FP64.
// A complex projection of every SUCCESS endpoint is kept in LDS and compared
// first; candidates are then compared in full.
template <int C>
struct k_dedup_tag {
    static constexpr int cap = C;
};

// A complex projection of a SUCCESS endpoint (NaN for any other status): the
// cheap first comparison of the crossing check.
__device__ __forceinline__ cx<double> dedup_proj(const DedupArgs &a, long long g)
{
    cx<double> p = {NAN, NAN};
    if (a.status[g] == HC_T_SUCCESS) {
        p = {0.0, 0.0};
        for (int j = 0; j < a.n; j++) {
            const cx<double> w = {cos(1.3 * j + 0.4), sin(2.1 * j + 0.9)};  // fixed generic weights
            p = cfma(w, cx<double>{a.endpoints[(g * a.n + j) * 2], a.endpoints[(g * a.n + j) * 2 + 1]}, p);
        }
    }
    return p;
}

// Full comparison of two endpoints whose projections are close: relative
// inf-norm distance within a.tol.
__device__ __forceinline__ bool dedup_same(const DedupArgs &a, long long g, long long h)
{
    double dmax = 0.0, cmax = 0.0;
    for (int j = 0; j < a.n; j++) {
        const double xr = a.endpoints[(g * a.n + j) * 2], xi = a.endpoints[(g * a.n + j) * 2 + 1];
        const double yr = a.endpoints[(h * a.n + j) * 2], yi = a.endpoints[(h * a.n + j) * 2 + 1];
        dmax = fmax(dmax, sqrt((xr - yr) * (xr - yr) + (xi - yi) * (xi - yi)));
        cmax = fmax(cmax, sqrt(yr * yr + yi * yi));
    }
    return dmax <= a.tol * fmax(1.0, cmax);
}

__device__ __forceinline__ bool dedup_near(cx<double> pb, cx<double> pc)
{
    return fabs(pc.re - pb.re) + fabs(pc.im - pb.im) <= 1e-6 * (1.0 + sqrt(abs2(pb)));
}

// CAP: LDS entries of the block (the launcher picks the smallest of 64, 1024 and
// kDedupMax that holds every instance it covers, so small instances do not tie
// up 128 KB of LDS per block).  Instances above CAP paths are left to
// k_dedup_big (this body returns without touching them).
template <int CAP>
__device__ __forceinline__ void dedup_body(const DedupArgs &a, int inst)
{
    __shared__ cx<double> proj[CAP];
    if (inst >= a.n_inst || a.n_start > CAP) return;
    const long long g0 = (long long)inst * a.n_start;
    const TrackState S = a.s;
    for (int b = threadIdx.x; b < a.n_start; b += blockDim.x) proj[b] = dedup_proj(a, g0 + b);
    __syncthreads();
    for (int b = threadIdx.x; b < a.n_start; b += blockDim.x) {
        const long long g = g0 + b;
        bool dup = false;
        if (a.status[g] == HC_T_SUCCESS) {
            const cx<double> pb = proj[b];
            for (int c = 0; c < a.n_start && !dup; c++)
                if (c != b && dedup_near(pb, proj[c])) dup = dedup_same(a, g, g0 + c);
        }
        S.status[g] = dup ? kRetrack : kDone;
    }
}

template <int CAP>
__global__ __launch_bounds__(256) void k_dedup(const DedupArgs a) { dedup_body<CAP>(a, blockIdx.x); }

template <int CAP>
__global__ __launch_bounds__(256) void k_dedup_many(const DedupArgs *a)
{
    dedup_body<CAP>(a[blockIdx.y], blockIdx.x);
}

// Instances with more than kDedupMax paths: every path's projection goes to
// a.proj in global memory (k_dedup_proj, one thread per path), then each thread
// of k_dedup_big compares its path with all of its instance's projections,
// staged through LDS one tile at a time (one block per 256 paths of an
// instance, the instance's blocks consecutive).
constexpr int kDedupTile = 1024;

__global__ __launch_bounds__(256) void k_dedup_proj(const DedupArgs a)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < a.total) reinterpret_cast<cx<double> *>(a.proj)[g] = dedup_proj(a, g);
}

__global__ __launch_bounds__(256) void k_dedup_big(const DedupArgs a)
{
    __shared__ cx<double> tile[kDedupTile];
    const int nb = (a.n_start + 255) / 256;  // path blocks per instance
    const int b = (int)(blockIdx.x % nb) * blockDim.x + threadIdx.x;
    const long long g0 = (long long)(blockIdx.x / nb) * a.n_start;
    const long long g = g0 + b;
    const bool mine = b < a.n_start && a.status[g] == HC_T_SUCCESS;
    const cx<double> *proj = reinterpret_cast<const cx<double> *>(a.proj);
    const cx<double> pb = mine ? proj[g] : cx<double>{NAN, NAN};
    bool dup = false;
    for (int c0 = 0; c0 < a.n_start; c0 += kDedupTile) {
        const int m = min(kDedupTile, a.n_start - c0);
        __syncthreads();
        for (int j = threadIdx.x; j < m; j += blockDim.x) tile[j] = proj[g0 + c0 + j];
        __syncthreads();
        for (int j = 0; mine && !dup && j < m; j++)
            if (c0 + j != b && dedup_near(pb, tile[j])) dup = dedup_same(a, g, g0 + c0 + j);
    }
    if (b < a.n_start) a.s.status[g] = dup ? kRetrack : kDone;
}

// The block's LDS capacity and size for instances of up to max_start paths
// (above kDedupMax: the largest block, which leaves those instances to
// k_dedup_big).
template <typename L>
static hipError_t dedup_dispatch(int max_start, L launch)
{
    if (max_start <= 64) return launch(k_dedup_tag<64>{}, 64);
    if (max_start <= 1024) return launch(k_dedup_tag<1024>{}, 256);
    return launch(k_dedup_tag<kDedupMax>{}, 256);
}

hipError_t launch_dedup_big(const DedupArgs &a, hipStream_t st)
{
    if (a.total == 0 || a.n_inst == 0) return hipSuccess;
    if (!a.proj) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dedup_proj, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, st, a);
    const long long blocks = (long long)((a.n_start + 255) / 256) * a.n_inst;
    hipLaunchKernelGGL(k_dedup_big, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_dedup(const DedupArgs &a, hipStream_t st)
{
    if (a.total == 0 || a.n_inst == 0) return hipSuccess;
    if (a.n_start > kDedupMax) return launch_dedup_big(a, st);
    return dedup_dispatch(a.n_start, [&](auto tag, int threads) {
        hipLaunchKernelGGL(k_dedup<decltype(tag)::cap>, dim3((unsigned)a.n_inst), dim3(threads), 0, st, a);
        return hipGetLastError();
    });
}

// ---------------------------------------------------------------- prep (a0/a2)

// One thread per (instance, kernel-table slot): the slot's coefficient is the sum
// over the terms mapped to it of mult * c_k(p), c_k(p) = const_k + sum val * p.
__device__ __forceinline__ void prep_body(const PrepArgs &a, long long gid)
{
    if (gid >= (long long)a.n_inst * a.n_slots) return;
    const int inst = (int)(gid / a.n_slots);
    const int s = (int)(gid % a.n_slots);
    const double *p = a.params + (size_t)inst * a.n_params * 2;
    double re = 0.0, im = 0.0;
    for (int e = a.slot_ptr[s]; e < a.slot_ptr[s + 1]; e++) {
        const int k = a.slot_term[e];
        double cr = 0.0, ci = 0.0;
        if (a.term_const) {
            cr = a.term_const[2 * k];
            ci = a.term_const[2 * k + 1];
        }
        if (a.map_ptr) {
            for (int m = a.map_ptr[k]; m < a.map_ptr[k + 1]; m++) {
                const int col = a.map_col[m];
                const double vr = a.map_val[2 * m], vi = a.map_val[2 * m + 1];
                const double pr = p[2 * col], pi = p[2 * col + 1];
                cr += vr * pr - vi * pi;
                ci += vr * pi + vi * pr;
            }
        } else {
            cr += p[2 * k];
            ci += p[2 * k + 1];
        }
        const double m = (double)a.slot_mult[e];
        re += m * cr;
        im += m * ci;
    }
    a.out64[2 * gid] = re;
    a.out64[2 * gid + 1] = im;
    if (a.out32) {
        a.out32[2 * gid] = (float)re;
        a.out32[2 * gid + 1] = (float)im;
    }
}

__global__ void k_prep(const PrepArgs a) { prep_body(a, (long long)blockIdx.x * blockDim.x + threadIdx.x); }

__global__ void k_prep_many(const PrepArgs *a)
{
    prep_body(a[blockIdx.y], (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------- refine (a8)

// Relative backward error max_i |F_i(x)| / sum_k |c_k| |m_k(x)| from the FP64
// kernel tables (q_aa holds twice the x_a^2 coefficient).
template <int N>
__device__ double residual_dense(tbl_ptr<double> cf, const cx<double> (&x)[N])
{
    constexpr int T = dense_terms(N);
    double eta = 0.0;
    for (int i = 0; i < N; i++) {
        const tbl_ptr<double> c = cf + 2 * T * i;
        cx<double> F = ldc(c, 0);
        double den = sqrt(abs2(F));
#pragma unroll
        for (int j = 0; j < N; j++) {
            const cx<double> L = ldc(c, 1 + j);
            F = cfma(L, x[j], F);
            den += sqrt(abs2(L)) * sqrt(abs2(x[j]));
        }
#pragma unroll
        for (int p = 0; p < N; p++) {
#pragma unroll
            for (int q = p; q < N; q++) {
                cx<double> cq = ldc(c, quad_slot(N, p, q));
                if (p == q) cq = {0.5 * cq.re, 0.5 * cq.im};
                const cx<double> m = cmul(x[p], x[q]);
                F = cfma(cq, m, F);
                den += sqrt(abs2(cq)) * sqrt(abs2(m));
            }
        }
        const double num = sqrt(abs2(F));
        const double e = den > 0.0 ? num / den : (num == 0.0 ? 0.0 : INFINITY);
        if (!(e <= eta)) eta = e;
    }
    return eta;
}

template <int N>
__device__ __forceinline__ void refine_body(const RefineArgs &a, int block)
{
    // one wavefront per (instance, 64 consecutive paths): the instance, and so the
    // table address, is wavefront-uniform and the tables come in by scalar loads
    constexpr int T = dense_terms(N);
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int item = __builtin_amdgcn_readfirstlane(block * (blockDim.x >> 6) + wib);
    if (a.total == 0) return;
    const int per_inst = (a.n_start + 63) / 64;
    const int inst = item / per_inst;
    const int b = (item - inst * per_inst) * 64 + lane;
    if ((long long)inst * a.n_start >= a.total) return;
    const bool valid = b < a.n_start;
    const long long g = (long long)inst * a.n_start + (valid ? b : 0);
    const double *cf = a.coef + (size_t)inst * N * T * 2;
    cx<double> gam = {1.0, 0.0};
    if (a.gamma) gam = {a.gamma[2 * inst], a.gamma[2 * inst + 1]};
    const TrackState S = a.s;
    int st = valid ? S.status[g] : HC_T_SUCCESS;
    const bool done = st == kDone;  // final from an earlier pass: nothing to write
    cx<double> x[N];
#pragma unroll
    for (int j = 0; j < N; j++) x[j] = {S.xr[j * a.total + g], S.xi[j * a.total + g]};
    int rits = 0;
    double resid = NAN;
    bool act = valid && st == kReached;
    for (int it = 0; it < a.max_refine; it++) {
        if (ballot(act) == 0ull) break;
        const double *cfs = cf;
        asm volatile("" : "+s"(cfs));
        cx<double> A[N][N + 1];
        build_td<N, double>(as_table(cfs), gam, a.deg2, x, 1.0, false, A);
        cx<double> dx[N];
        const bool sing = lu_solve<N, double>(A, dx);
        if (act) {
            if (sing) {
                st = HC_T_SINGULAR;
                act = false;
            } else {
                double nd = 0.0, nx = 0.0;
#pragma unroll
                for (int j = 0; j < N; j++) {
                    x[j] = {x[j].re + dx[j].re, x[j].im + dx[j].im};
                    nd += abs2(dx[j]);
                    nx += abs2(x[j]);
                }
                rits++;
                if (sqrt(nd) <= a.tau_refine * (1.0 + sqrt(nx))) act = false;
            }
        }
    }
    if (!valid || done) return;
    if (st == kReached) {
        bool fin = true;
        double big = 0.0;
#pragma unroll
        for (int j = 0; j < N; j++) {
            fin = fin && finite(x[j]);
            big = fmax(big, abs2(x[j]));
        }
        if (!fin) {
            st = HC_T_NONFINITE;
        } else {
            resid = residual_dense<N>(as_table(cf), x);
            if (big > a.inf2)
                st = HC_T_AT_INFINITY;
            else if (a.singular_end)
                st = HC_T_SINGULAR_END;
            else if (!(resid <= a.eta_max))
                st = HC_T_REFINE_FAILED;
            else
                st = HC_T_SUCCESS;
        }
    } else if (st < 0) {
        st = HC_T_MAX_STEPS;  // unreachable after a full run: every path ends
    }
#pragma unroll
    for (int j = 0; j < N; j++) {
        a.endpoints[(g * N + j) * 2] = x[j].re;
        a.endpoints[(g * N + j) * 2 + 1] = x[j].im;
    }
    a.status[g] = st;
    if (a.info) {
        hc_track_info inf;
        inf.steps = S.steps[g];
        inf.rejects = S.rejects[g];
        inf.newton_its = S.nits[g];
        inf.refine_its = rits;
        inf.escalated = S.escal[g] != 0 ? 1 : 0;
        inf.cycle = a.eg_cycle ? S.succ[g] : 0;
        inf.residual = resid;
        a.info[g] = inf;
    }
}

template <int N>
__global__ __launch_bounds__(256) void k_refine(const RefineArgs a) { refine_body<N>(a, blockIdx.x); }

template <int N>
__global__ __launch_bounds__(256) void k_refine_many(const RefineArgs *a) { refine_body<N>(a[blockIdx.y], blockIdx.x); }

// ---------------------------------------------------------------- launchers

__global__ void k_fill_u32(unsigned *p, unsigned value, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

hipError_t launch_fill_u32(unsigned *p, unsigned value, int count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((count + 255) / 256), dim3(256), 0, st, p, value, count);
    return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs &a, hipStream_t st)
{
    const long long n = (long long)a.n_inst * a.n_slots;
    if (n == 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_init(const InitArgs &a, hipStream_t st)
{
    if (a.total == 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(k_init, dim3((unsigned)((a.total + bs - 1) / bs)), dim3(bs), 0, st, a);
    return hipGetLastError();
}

template <int N>
static hipError_t launch_track_n(bool fp32, const TrackArgs &a, int wpb, hipStream_t st)
{
    const int blocks = (a.n_items + wpb - 1) / wpb;
    if (fp32)
        hipLaunchKernelGGL((k_track<N, float>), dim3(blocks), dim3(64 * wpb), 0, st, a);
    else
        hipLaunchKernelGGL((k_track<N, double>), dim3(blocks), dim3(64 * wpb), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_track(int n, bool fp32, const TrackArgs &a, int wpb, hipStream_t st)
{
    if (a.n_items == 0) return hipSuccess;
    switch (n) {
    case 1: return launch_track_n<1>(fp32, a, wpb, st);
    case 2: return launch_track_n<2>(fp32, a, wpb, st);
    case 3: return launch_track_n<3>(fp32, a, wpb, st);
    case 4: return launch_track_n<4>(fp32, a, wpb, st);
    case 5: return launch_track_n<5>(fp32, a, wpb, st);
    case 6: return launch_track_n<6>(fp32, a, wpb, st);
    case 7: return launch_track_n<7>(fp32, a, wpb, st);
    case 8: return launch_track_n<8>(fp32, a, wpb, st);
    default: return hipErrorInvalidValue;
    }
}

template <int N>
static hipError_t launch_refine_n(const RefineArgs &a, hipStream_t st)
{
    const long long n_inst = a.total / a.n_start;
    const long long items = n_inst * ((a.n_start + 63) / 64);
    hipLaunchKernelGGL(k_refine<N>, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Many jobs: blocks = the largest job's block count along x, one job per y.
hipError_t launch_prep_many(const PrepArgs *a, int count, long long max_work, hipStream_t st)
{
    if (count == 0 || max_work == 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep_many, dim3((unsigned)((max_work + 255) / 256), (unsigned)count), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_init_many(const InitArgs *a, int count, long long max_total, hipStream_t st)
{
    if (count == 0 || max_total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_many, dim3((unsigned)((max_total + 255) / 256), (unsigned)count), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_dedup_many(const DedupArgs *a, int count, int max_inst, int max_start, hipStream_t st)
{
    if (count == 0 || max_inst == 0) return hipSuccess;
    return dedup_dispatch(max_start, [&](auto tag, int threads) {
        hipLaunchKernelGGL(k_dedup_many<decltype(tag)::cap>, dim3((unsigned)max_inst, (unsigned)count), dim3(threads),
                           0, st, a);
        return hipGetLastError();
    });
}

template <int N>
static hipError_t launch_refine_many_n(const RefineArgs *a, int count, long long max_items, hipStream_t st)
{
    hipLaunchKernelGGL(k_refine_many<N>, dim3((unsigned)((max_items + 3) / 4), (unsigned)count), dim3(256), 0, st, a);
    return hipGetLastError();
}

// One path per lane for n = 1; 2 <= n <= 8 refine in the group layout
// (hc_track_group.hip), whose registers hold one row per lane instead of the
// whole n x (n + 1) system.
hipError_t launch_refine_many(int n, const RefineArgs *a, int count, long long max_items, long long max_total,
                              hipStream_t st)
{
    if (count == 0 || max_items == 0) return hipSuccess;
    if (n == 1) return launch_refine_many_n<1>(a, count, max_items, st);
    return launch_refine_group(n, a, count, max_total, true, st);
}

hipError_t launch_refine(int n, const RefineArgs &a, hipStream_t st)
{
    if (a.total == 0) return hipSuccess;
    if (n == 1) return launch_refine_n<1>(a, st);
    return launch_refine_group(n, &a, 1, a.total, false, st);
}

}  // namespace hcx

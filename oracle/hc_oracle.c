/*
 * hc_oracle.c -- plain FP64 CPU homotopy-continuation path tracker (the ORACLE).
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's CPU
 * baseline call it; the product path never does, and it shares no code, header,
 * table or constant with the HIP path.  It is deliberately plain: naive monomial
 * sums, textbook LU, one track at a time, complex double throughout.
 *
 * What it computes, following Chien et al., "GPU-Based Homotopy Continuation for
 * Minimal Problems in Computer Vision":
 *   - section 3, Eq. (1): the linear homotopy H(x,t) = (1-t) G(x) + t F(x), t in [0,1],
 *     with a random unit-modulus gamma on the start system (reading: the gamma trick,
 *     which the paper does not print) -- H = (1-t) gamma G + t F, G_i = x_i^d_i - 1;
 *   - section 6 (parallel evaluations): parameter homotopies whose coefficients are
 *     linear interpolations of the start and target coefficients, c(t) = (1-t)c0 + t c1,
 *     with dH/dt obtained from the same terms with coefficients c1 - c0;
 *   - section 3, Eq. (3): the Davidenko equation H_x dx/dt = -H_t gives the tangent;
 *   - section 3 (text after Eq. (4)): a 4th-order Runge-Kutta predictor built from that
 *     tangent (reading: the classic tableau, nodes 0, 1/2, 1/2, 1, weights 1/6,1/3,1/3,1/6);
 *   - section 3, Eqs. (5)-(6): Newton correction at t + dt;
 *   - section 3 ("a number of small steps"): adaptive step size (constants are ours);
 *   - section 6 (linear system solver): LU with partial pivoting of the augmented
 *     matrix [A b], so the forward substitution happens during the factorization and
 *     the back substitution uses U.
 * Readings where the paper is silent are the ones listed with the opts below.
 *
 * Parity-pinned by tests/test_oracle_*.py against library routines, closed forms,
 * resultants, brute force and planted roots.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_MAXN 64

/* ---- problem description ------------------------------------------------ */

typedef struct {
    int n;               /* unknowns = equations                               */
    int n_terms;         /* number of terms over all equations                 */
    const int *term_eq;  /* [n_terms]    equation of term k                    */
    const int *term_exp; /* [n_terms*n]  exponent of x_j in term k             */
} orc_system;

enum { ORC_TOTAL_DEGREE = 0, ORC_LINEAR = 1 };

typedef struct {
    const orc_system *S;
    int kind;            /* ORC_TOTAL_DEGREE or ORC_LINEAR                      */
    const cplx *c0;      /* LINEAR: start coefficients [n_terms]                */
    const cplx *c1;      /* target coefficients [n_terms]                       */
    cplx gamma;          /* TOTAL_DEGREE: multiplies the start system           */
    int deg[ORC_MAXN];   /* TOTAL_DEGREE: degree d_i of equation i              */
} orc_homotopy;

/* Step-control constants and tolerances (the paper gives none). */
typedef struct {
    double h0, h_min, h_max;     /* first step, failure threshold, cap              */
    double beta_inc, beta_dec;   /* growth after n_inc accepted steps, shrink on reject */
    double tau;                  /* Newton: ||dx||_2 <= tau (1 + ||x||_2)          */
    double pred_tol;             /* first correction: ||dx_1||_2 <= pred_tol (1 + ||x||_2),
                                    else the prediction was too far off: reject the step */
    double tau_refine;           /* endpoint refinement stop test, same form        */
    double inf_bound;            /* ||x||_inf above this => path at infinity        */
    double eta_max;              /* relative backward error accepted at t = 1       */
    int n_inc, max_newton, max_steps, max_refine;
} orc_opts;

typedef struct {
    int steps;       /* accepted steps                       */
    int rejects;     /* rejected steps                       */
    int newton_its;  /* corrector iterations while tracking  */
    int refine_its;  /* Newton iterations of the refinement  */
    double residual; /* relative backward error at the end   */
} orc_info;

enum {
    ORC_SUCCESS = 0, ORC_AT_INFINITY = 1, ORC_MIN_STEP = 2, ORC_MAX_STEPS = 3,
    ORC_SINGULAR = 4, ORC_NONFINITE = 5, ORC_REFINE_FAILED = 6,
    ORC_SINGULAR_END = 7   /* the end-game's estimate of a singular endpoint        */
};

/* ---- small helpers -------------------------------------------------------- */

static cplx ipow(cplx z, int e)
{
    cplx r = 1.0;
    for (int i = 0; i < e; i++) r *= z;
    return r;
}

static double norm2(int n, const cplx *v)
{
    double s = 0.0;
    for (int j = 0; j < n; j++) s += creal(v[j]) * creal(v[j]) + cimag(v[j]) * cimag(v[j]);
    return sqrt(s);
}

static double norminf(int n, const cplx *v)
{
    double m = 0.0;
    for (int j = 0; j < n; j++) {
        double a = cabs(v[j]);
        if (!(a <= m)) m = a; /* NaN propagates */
    }
    return m;
}

static int all_finite(int n, const cplx *v)
{
    for (int j = 0; j < n; j++)
        if (!isfinite(creal(v[j])) || !isfinite(cimag(v[j]))) return 0;
    return 1;
}

/* ---- evaluation (definition of F and its Jacobian) ------------------------ */

/* m_k(x) = prod_j x_j^e_kj */
static cplx monomial(const orc_system *S, int k, const cplx *x)
{
    const int *e = S->term_exp + (size_t)k * S->n;
    cplx m = 1.0;
    for (int j = 0; j < S->n; j++) m *= ipow(x[j], e[j]);
    return m;
}

/* d m_k / d x_j = e_kj x_j^(e_kj - 1) prod_{l != j} x_l^e_kl */
static cplx monomial_dx(const orc_system *S, int k, const cplx *x, int j)
{
    const int *e = S->term_exp + (size_t)k * S->n;
    if (e[j] == 0) return 0.0;
    cplx m = (double)e[j] * ipow(x[j], e[j] - 1);
    for (int l = 0; l < S->n; l++)
        if (l != j) m *= ipow(x[l], e[l]);
    return m;
}

/* F_i(x) = sum_{k in eq i} c_k m_k(x);  J_ij = sum_{k in eq i} c_k dm_k/dx_j.
 * F or J may be NULL.  J is row-major n x n. */
void orc_eval_system(const orc_system *S, const cplx *c, const cplx *x, cplx *F, cplx *J)
{
    int n = S->n;
    if (F) for (int i = 0; i < n; i++) F[i] = 0.0;
    if (J) for (int i = 0; i < n * n; i++) J[i] = 0.0;
    for (int k = 0; k < S->n_terms; k++) {
        int i = S->term_eq[k];
        if (F) F[i] += c[k] * monomial(S, k, x);
        if (J)
            for (int j = 0; j < n; j++) J[i * n + j] += c[k] * monomial_dx(S, k, x, j);
    }
}

/* d_i = largest total degree among the terms of equation i */
void orc_degrees(const orc_system *S, int *deg)
{
    for (int i = 0; i < S->n; i++) deg[i] = 0;
    for (int k = 0; k < S->n_terms; k++) {
        int d = 0;
        for (int j = 0; j < S->n; j++) d += S->term_exp[(size_t)k * S->n + j];
        if (d > deg[S->term_eq[k]]) deg[S->term_eq[k]] = d;
    }
}

/* H, H_x (row-major) and H_t at (x, t); any output may be NULL.
 *   TOTAL_DEGREE: H = (1-t) gamma G + t F, G_i = x_i^d_i - 1, H_t = F - gamma G.
 *   LINEAR:       H = F(x; (1-t) c0 + t c1),        H_t = F(x; c1 - c0).       */
void orc_homotopy_eval(const orc_homotopy *Hm, const cplx *x, double t, cplx *H, cplx *Hx, cplx *Ht)
{
    const orc_system *S = Hm->S;
    int n = S->n;
    if (Hm->kind == ORC_TOTAL_DEGREE) {
        cplx F[ORC_MAXN], J[ORC_MAXN * ORC_MAXN];
        orc_eval_system(S, Hm->c1, x, F, J);
        for (int i = 0; i < n; i++) {
            cplx G = ipow(x[i], Hm->deg[i]) - 1.0;
            cplx dG = (double)Hm->deg[i] * ipow(x[i], Hm->deg[i] - 1);
            if (H) H[i] = (1.0 - t) * Hm->gamma * G + t * F[i];
            if (Ht) Ht[i] = F[i] - Hm->gamma * G;
            if (Hx)
                for (int j = 0; j < n; j++)
                    Hx[i * n + j] = t * J[i * n + j] + (i == j ? (1.0 - t) * Hm->gamma * dG : 0.0);
        }
    } else {
        int T = S->n_terms;
        cplx *ct = malloc(sizeof(cplx) * (size_t)T);
        cplx *dc = malloc(sizeof(cplx) * (size_t)T);
        for (int k = 0; k < T; k++) {
            ct[k] = (1.0 - t) * Hm->c0[k] + t * Hm->c1[k];
            dc[k] = Hm->c1[k] - Hm->c0[k];
        }
        orc_eval_system(S, ct, x, H, Hx);
        if (Ht) orc_eval_system(S, dc, x, Ht, NULL);
        free(ct);
        free(dc);
    }
}

/* ---- dense linear solve ------------------------------------------------------ */

/* Solve A x = b (A row-major n x n) by Gaussian elimination with partial pivoting
 * on the augmented matrix [A b]: eliminating below each pivot also transforms b,
 * and back substitution with U finishes the solve.  Pivot = the row with the
 * largest |Re a| + |Im a| in the column, the lowest row index on ties.
 * Returns 0, or 1 if some pivot is exactly zero (x is then left untouched). */
int orc_lu_solve(int n, const cplx *A, const cplx *b, cplx *x)
{
    cplx M[ORC_MAXN][ORC_MAXN + 1];
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < n; j++) M[i][j] = A[i * n + j];
        M[i][n] = b[i];
    }
    for (int k = 0; k < n; k++) {
        int p = k;
        double best = fabs(creal(M[k][k])) + fabs(cimag(M[k][k]));
        for (int r = k + 1; r < n; r++) {
            double v = fabs(creal(M[r][k])) + fabs(cimag(M[r][k]));
            if (v > best) { best = v; p = r; }
        }
        if (best == 0.0) return 1;
        if (p != k)
            for (int c = k; c <= n; c++) { cplx tmp = M[k][c]; M[k][c] = M[p][c]; M[p][c] = tmp; }
        cplx inv = 1.0 / M[k][k];
        for (int r = k + 1; r < n; r++) {
            cplx l = M[r][k] * inv;
            for (int c = k + 1; c <= n; c++) M[r][c] -= l * M[k][c];
        }
    }
    for (int k = n - 1; k >= 0; k--) {
        cplx s = M[k][n];
        for (int c = k + 1; c < n; c++) s -= M[k][c] * x[c];
        x[k] = s / M[k][k];
    }
    return 0;
}

/* ---- predictor / corrector pieces --------------------------------------------- */

/* Tangent dx/dt at (x,t): solve H_x v = -H_t  (Eq. 3).  Returns 1 on a zero pivot. */
static int tangent(const orc_homotopy *Hm, const cplx *x, double t, cplx *v)
{
    int n = Hm->S->n;
    cplx Hx[ORC_MAXN * ORC_MAXN], Ht[ORC_MAXN], rhs[ORC_MAXN];
    orc_homotopy_eval(Hm, x, t, NULL, Hx, Ht);
    for (int i = 0; i < n; i++) rhs[i] = -Ht[i];
    return orc_lu_solve(n, Hx, rhs, v);
}

/* Newton update at (x,t): solve H_x d = -H  (Eqs. 5-6).  Returns 1 on a zero pivot. */
static int newton_delta(const orc_homotopy *Hm, const cplx *x, double t, cplx *d)
{
    int n = Hm->S->n;
    cplx Hx[ORC_MAXN * ORC_MAXN], H[ORC_MAXN], rhs[ORC_MAXN];
    orc_homotopy_eval(Hm, x, t, H, Hx, NULL);
    for (int i = 0; i < n; i++) rhs[i] = -H[i];
    return orc_lu_solve(n, Hx, rhs, d);
}

/* One classic RK4 step of dx/dt = v(x,t) from (x,t) over hu, the last node at tn
 * (tn = t + hu, or the exact end point when the step was clipped to it).
 * xs receives x + hu/6 (k1 + 2 k2 + 2 k3 + k4).  Returns 1 if a solve failed, and 2
 * if the first tangent (at the accepted point) came out non-finite from a regular
 * matrix: non-finite data, which no smaller step can cure. */
static int rk4_step(const orc_homotopy *Hm, const cplx *x, double t, double hu, double tn, cplx *xs)
{
    int n = Hm->S->n;
    cplx k1[ORC_MAXN], k2[ORC_MAXN], k3[ORC_MAXN], k4[ORC_MAXN], y[ORC_MAXN];
    double tm = t + 0.5 * hu;
    if (tangent(Hm, x, t, k1)) return 1;
    if (!all_finite(n, k1)) return 2;
    for (int j = 0; j < n; j++) y[j] = x[j] + (0.5 * hu) * k1[j];
    if (tangent(Hm, y, tm, k2)) return 1;
    for (int j = 0; j < n; j++) y[j] = x[j] + (0.5 * hu) * k2[j];
    if (tangent(Hm, y, tm, k3)) return 1;
    for (int j = 0; j < n; j++) y[j] = x[j] + hu * k3[j];
    if (tangent(Hm, y, tn, k4)) return 1;
    for (int j = 0; j < n; j++) xs[j] = x[j] + (hu / 6.0) * (k1[j] + 2.0 * k2[j] + 2.0 * k3[j] + k4[j]);
    return 0;
}

/* ---- endpoint refinement and classification ------------------------------------ */

/* Relative backward error: max_i |F_i(x)| / sum_{k in eq i} |c_k| |m_k(x)|. */
double orc_residual(const orc_system *S, const cplx *c, const cplx *x)
{
    double num[ORC_MAXN], den[ORC_MAXN];
    cplx F[ORC_MAXN];
    orc_eval_system(S, c, x, F, NULL);
    for (int i = 0; i < S->n; i++) { num[i] = cabs(F[i]); den[i] = 0.0; }
    for (int k = 0; k < S->n_terms; k++) den[S->term_eq[k]] += cabs(c[k]) * cabs(monomial(S, k, x));
    double eta = 0.0;
    for (int i = 0; i < S->n; i++) {
        double e = den[i] > 0.0 ? num[i] / den[i] : (num[i] == 0.0 ? 0.0 : INFINITY);
        if (!(e <= eta)) eta = e;
    }
    return eta;
}

/* Newton on F = H(., 1) until ||dx||_2 <= tau_refine (1 + ||x||_2) or max_refine
 * iterations, then classify the endpoint. */
static int refine_endpoint(const orc_homotopy *Hm, const orc_opts *o, cplx *x, orc_info *info)
{
    const orc_system *S = Hm->S;
    int n = S->n;
    cplx F[ORC_MAXN], J[ORC_MAXN * ORC_MAXN], rhs[ORC_MAXN], d[ORC_MAXN];
    for (int it = 0; it < o->max_refine; it++) {
        orc_eval_system(S, Hm->c1, x, F, J);
        for (int i = 0; i < n; i++) rhs[i] = -F[i];
        if (orc_lu_solve(n, J, rhs, d)) return ORC_SINGULAR;
        for (int j = 0; j < n; j++) x[j] += d[j];
        info->refine_its++;
        if (norm2(n, d) <= o->tau_refine * (1.0 + norm2(n, x))) break;
    }
    if (!all_finite(n, x)) return ORC_NONFINITE;
    info->residual = orc_residual(S, Hm->c1, x);
    if (norminf(n, x) > o->inf_bound) return ORC_AT_INFINITY;
    if (!(info->residual <= o->eta_max)) return ORC_REFINE_FAILED;
    return ORC_SUCCESS;
}

/* ---- one path ------------------------------------------------------------------- */

/* The step loop of section 3 from (x, *t) up to t_final: per step an RK4 prediction
 * to t + h, then at most max_newton Newton corrections at t + h; accept when the
 * correction is below tau (1 + ||x||_2), else halve h.  The last step is clipped
 * to land exactly on t_final.  x, *t, *h, *succ and info carry the path's state
 * from one call to the next.  Returns -1 once t_final is reached, else the
 * failure status. */
static int track_segment(const orc_homotopy *Hm, const orc_opts *o, double tau, int max_newton, double h_min,
                         cplx *x, double *t_io, double *h_io, int *succ_io, double t_final,
                         orc_info *info)
{
    int n = Hm->S->n;
    cplx xs[ORC_MAXN], d[ORC_MAXN];
    double t = *t_io, h = *h_io;
    int succ = *succ_io, status = -1;

    while (t < t_final) {
        if (info->steps + info->rejects >= o->max_steps) { status = ORC_MAX_STEPS; break; }
        double hu, tn;
        if (h >= t_final - t) { hu = t_final - t; tn = t_final; }   /* land exactly on t_final */
        else                  { hu = h;           tn = t + h; }

        int converged = 0;
        int bad = rk4_step(Hm, x, t, hu, tn, xs);
        if (bad == 2) { status = ORC_NONFINITE; break; }
        if (!bad) {
            for (int it = 0; it < max_newton; it++) {
                if (newton_delta(Hm, xs, tn, d)) break;
                info->newton_its++;
                for (int j = 0; j < n; j++) xs[j] += d[j];
                double nd = norm2(n, d), nx = norm2(n, xs);
                if (it == 0 && !(nd <= o->pred_tol * (1.0 + nx))) break;
                if (nd <= tau * (1.0 + nx)) { converged = 1; break; }
            }
        }
        if (converged) {
            for (int j = 0; j < n; j++) x[j] = xs[j];
            t = tn;
            info->steps++;
            if (++succ >= o->n_inc) { h = fmin(h * o->beta_inc, o->h_max); succ = 0; }
            if (norminf(n, x) > o->inf_bound) { status = ORC_AT_INFINITY; break; }
        } else {
            info->rejects++;
            succ = 0;
            h *= o->beta_dec;
            if (h < h_min) { status = ORC_MIN_STEP; break; }
        }
    }
    *t_io = t;
    *h_io = h;
    *succ_io = succ;
    return status;
}

/* Track x(t) from x0 at t = 0 to t = 1 (section 3), then refine at t = 1.
 * Returns the status; *t_end = the t the path stopped at. */
static int track_one_t(const orc_homotopy *Hm, const orc_opts *o, const cplx *x0, cplx *x_out,
                       orc_info *info, double *t_end)
{
    int n = Hm->S->n;
    cplx x[ORC_MAXN];
    double t = 0.0, h = o->h0;
    int succ = 0, status = -1;
    memset(info, 0, sizeof(*info));
    info->residual = NAN;
    for (int j = 0; j < n; j++) x[j] = x0[j];
    if (!all_finite(n, x)) status = ORC_NONFINITE;
    if (status < 0) status = track_segment(Hm, o, o->tau, o->max_newton, o->h_min, x, &t, &h, &succ, 1.0, info);
    if (status < 0) status = refine_endpoint(Hm, o, x, info);
    for (int j = 0; j < n; j++) x_out[j] = x[j];
    *t_end = t;
    return status;
}

int orc_track_one(const orc_homotopy *Hm, const orc_opts *o, const cplx *x0, cplx *x_out, orc_info *info)
{
    double t;
    return track_one_t(Hm, o, x0, x_out, info, &t);
}

/* ---- power-series end-game ------------------------------------------------------ */

/* The paper does not treat singular endpoints (section 2 only warns that the number
 * of solutions HC reports needs checking).  This follows the published power-series
 * end-game of Morgan, Sommese and Wampler ("A power series method for computing
 * singular solutions to nonlinear analytic systems", Numer. Math. 63, 1992):
 * near t = 1, with s = 1 - t, a path has a convergent fractional power series
 * x(s) = sum_j a_j s^(j/c) whose cycle number c >= 1 makes x analytic in
 * sigma = s^(1/c) (meromorphic, for a path that goes to infinity).  The series is
 * taken of the point in projective coordinates on a fixed patch,
 * y(s) = (1, x(s)) / (a . (1, x(s))), which stays bounded at infinity (y_0 -> 0)
 * as well as at finite endpoints.  The path is sampled at the geometric points
 * s_k = s0 beta^k, c is estimated from the decay of successive sample differences
 * (|y_k - y_(k+1)| ~ s_k^(1/c)), and y(0) is extrapolated from the last three
 * samples by the quadratic through them in sigma; x = y_(1..n) / y_0.  Readings
 * (the constants are ours): samples from k = 1 on, tracked with a tighter
 * corrector (eg->tau, eg->max_newton) and a smaller minimum step (eg->h_min: the
 * steps shrink with s there) inside the zone [1 - s0, 1]; the end-game has
 * converged when two successive estimates of y agree to eg->tol |y|_inf, or to
 * eg->tol_inf |y|_inf with an estimated y_0 below |y|_inf / inf_bound (the affine
 * tracker's bound on |x|: a path to infinity, whose y_0 -> 0 needs no more digits
 * to be told from a finite endpoint); the
 * patch is a_j = exp(2 pi i frac((j + 1) phi)), phi = (sqrt 5 - 1) / 2 (the
 * golden-ratio Weyl sequence, j = 0..n), fixed so that both sides of a
 * comparison use the same one. */
typedef struct {
    double s0;        /* zone [1 - s0, 1]                                          */
    double beta;      /* sample ratio s_(k+1) = beta s_k                            */
    double tol;       /* successive estimates this close (relative): converged     */
    double tol_inf;   /* ... this close, with y_0 below |y|_inf / inf_bound: at infinity */
    double tau;       /* corrector tolerance inside the zone                       */
    double h_min;     /* smallest step inside the zone                              */
    int max_newton;   /* corrector iterations per step inside the zone             */
    int max_samples;  /* samples s_1 .. s_max_samples                              */
    int max_cycle;    /* largest cycle number considered                           */
    int every;        /* 1: every path that reaches the zone takes the end-game    */
} orc_eg_opts;

/* Cycle number and extrapolated x(0) from three samples y0, y1, y2 taken at s,
 * beta s, beta^2 s.  Returns 0 and sets *c, E; 1 if the samples do not decay. */
static int eg_estimate(int n, const cplx *y0, const cplx *y1, const cplx *y2, double beta, int max_cycle,
                       int *c, cplx *E)
{
    cplx d[ORC_MAXN + 1];
    for (int j = 0; j < n; j++) d[j] = y0[j] - y1[j];
    double d1 = norminf(n, d);
    for (int j = 0; j < n; j++) d[j] = y1[j] - y2[j];
    double d2 = norminf(n, d);
    if (d2 == 0.0) {              /* the path has stopped moving: x(0) = y2 */
        *c = 1;
        for (int j = 0; j < n; j++) E[j] = y2[j];
        return 0;
    }
    if (!(d2 < d1)) return 1;     /* not decaying (yet), or heading to infinity */
    /* d2 / d1 ~ beta^(1/c) */
    double cr = log(beta) / log(d2 / d1);
    int ci = (int)floor(cr + 0.5);
    if (ci < 1) ci = 1;
    if (ci > max_cycle) ci = max_cycle;
    *c = ci;
    /* the samples sit at sigma0, q sigma0, q^2 sigma0 with q = beta^(1/c); the
     * lines through consecutive pairs meet sigma = 0 at R_a, R_b, and the quadratic
     * through all three at (R_b - q^2 R_a) / (1 - q^2) */
    double q = pow(beta, 1.0 / ci);
    for (int j = 0; j < n; j++) {
        cplx ra = (y1[j] - q * y0[j]) / (1.0 - q);
        cplx rb = (y2[j] - q * y1[j]) / (1.0 - q);
        E[j] = (rb - q * q * ra) / (1.0 - q * q);
    }
    return 0;
}

/* y = (1, x) / (a . (1, x)) on the end-game's patch (n + 1 entries). */
static void eg_project(int n, const cplx *x, cplx *y)
{
    const double phi = 0.5 * (sqrt(5.0) - 1.0);
    cplx den = 0.0;
    for (int j = 0; j <= n; j++) {
        double f = (j + 1) * phi;
        f -= floor(f);
        den += cexp(I * (2.0 * 3.14159265358979323846 * f)) * (j == 0 ? 1.0 : x[j - 1]);
    }
    y[0] = 1.0 / den;
    for (int j = 0; j < n; j++) y[j + 1] = x[j] / den;
}

/* End-game of one path from its start point x0: tracked like orc_track_one up to
 * t = 1 - s0, then sampled at s_1, s_2, ... as above.  Returns -1 and sets x_out
 * (= y_(1..n) / y_0 of the estimate, infinite entries for y_0 = 0), *cycle when
 * two successive estimates agree; else the status at which the path stopped (a
 * tracking failure, or ORC_MIN_STEP when max_samples were not enough), with x_out
 * the last point tracked.  info counts this run's steps. */
static int endgame_one(const orc_homotopy *Hm, const orc_opts *o, const orc_eg_opts *eg, const cplx *x0,
                       cplx *x_out, orc_info *info, int *cycle)
{
    int n = Hm->S->n, m = Hm->S->n + 1;
    cplx x[ORC_MAXN], y[3][ORC_MAXN + 1], E[ORC_MAXN + 1], Ep[ORC_MAXN + 1];
    double t = 0.0, h = o->h0, s = eg->s0;
    int succ = 0, have_prev = 0, status;
    memset(info, 0, sizeof(*info));
    info->residual = NAN;
    for (int j = 0; j < n; j++) x[j] = x0[j];
    if (!all_finite(n, x)) return ORC_NONFINITE;
    status = track_segment(Hm, o, o->tau, o->max_newton, o->h_min, x, &t, &h, &succ, 1.0 - s, info);
    for (int k = 1; status < 0 && k <= eg->max_samples; k++) {
        s *= eg->beta;
        status = track_segment(Hm, o, eg->tau, eg->max_newton, eg->h_min, x, &t, &h, &succ, 1.0 - s, info);
        if (status >= 0) break;
        memmove(y[0], y[1], sizeof(y[0]) * 2);
        eg_project(n, x, y[2]);
        if (k < 3) continue;
        int c;
        if (eg_estimate(m, y[0], y[1], y[2], eg->beta, eg->max_cycle, &c, E)) {
            have_prev = 0;
            continue;
        }
        if (have_prev) {
            cplx diff[ORC_MAXN + 1];
            for (int j = 0; j < m; j++) diff[j] = E[j] - Ep[j];
            double dn = norminf(m, diff), en = norminf(m, E);
            /* settled on a finite point, or on y_0 = 0 as closely as the affine
             * bound |x| <= inf_bound can tell (a path to infinity) */
            if (dn <= eg->tol * en || (dn <= eg->tol_inf * en && cabs(E[0]) * o->inf_bound <= en)) {
                for (int j = 0; j < n; j++) x_out[j] = E[j + 1] / E[0];
                *cycle = c;
                return -1;
            }
        }
        for (int j = 0; j < m; j++) Ep[j] = E[j];
        have_prev = 1;
    }
    for (int j = 0; j < n; j++) x_out[j] = x[j];
    return status < 0 ? ORC_MIN_STEP : status;
}

/* A path that stopped with `status` at t_end gets the end-game when it failed in
 * the zone [1 - s0, 1] or reached t = 1 without a regular endpoint; with
 * eg->every, every path that reached the zone and met no non-finite value. */
static int eg_candidate(const orc_eg_opts *eg, int status, double t_end)
{
    if (eg->every) return status != ORC_NONFINITE && t_end >= 1.0 - eg->s0;
    if (status == ORC_REFINE_FAILED || status == ORC_SINGULAR) return 1;
    return (status == ORC_MIN_STEP || status == ORC_MAX_STEPS) && t_end >= 1.0 - eg->s0;
}

/* orc_track_one, and for an end-game candidate the end-game from the start point.
 * If the end-game converges, its estimate E is classified: above inf_bound (y_0 ->
 * 0) ORC_AT_INFINITY; cycle number 1 (the path ends at a point where it is
 * analytic in s) the usual refinement and classification at t = 1 from E; cycle
 * number >= 2 (a singular endpoint: Newton would only converge linearly) the
 * endpoint is E itself, status ORC_SINGULAR_END, with its residual.  If it does
 * not converge the first result stands.  info counts the steps of both runs;
 * *cycle = the cycle number (0 without a converged end-game). */
static int track_one_eg(const orc_homotopy *Hm, const orc_opts *o, const orc_eg_opts *eg, const cplx *x0,
                        cplx *x_out, orc_info *info, int *cycle)
{
    int n = Hm->S->n;
    double t_end;
    *cycle = 0;
    int st = track_one_t(Hm, o, x0, x_out, info, &t_end);
    if (!eg || !eg_candidate(eg, st, t_end)) return st;
    cplx E[ORC_MAXN];
    orc_info ie;
    int c = 0;
    if (endgame_one(Hm, o, eg, x0, E, &ie, &c) >= 0) return st;
    info->steps += ie.steps;
    info->rejects += ie.rejects;
    info->newton_its += ie.newton_its;
    info->refine_its = 0;
    info->residual = NAN;
    *cycle = c;
    for (int j = 0; j < n; j++) x_out[j] = E[j];
    if (!(norminf(n, E) <= o->inf_bound)) return ORC_AT_INFINITY;
    if (c == 1) return refine_endpoint(Hm, o, x_out, info);
    info->residual = orc_residual(Hm->S, Hm->c1, E);
    return ORC_SINGULAR_END;
}

/* Start point of track b of the total-degree start system G_i = x_i^d_i - 1:
 * write b in mixed radix (d_1, ..., d_n), x_1 least significant, digit j_i, and
 * take x_i = exp(2 pi i j_i / d_i). */
void orc_total_degree_start(int n, const int *deg, long long b, cplx *x)
{
    for (int i = 0; i < n; i++) {
        int j = (int)(b % deg[i]);
        b /= deg[i];
        if (j == 0) x[i] = 1.0;
        else if (2 * j == deg[i]) x[i] = -1.0;
        else x[i] = cexp(I * (2.0 * 3.14159265358979323846 * j / deg[i]));
    }
}

/* ---- batch driver (all host cores) ------------------------------------------------ */

typedef struct {
    const orc_system *S;
    int kind;
    const cplx *c0, *c1, *gamma, *start;
    int n_start, n_inst;
    const orc_opts *o;
    const orc_eg_opts *eg; /* NULL: no end-game */
    cplx *endpoints;
    int *status;
    orc_info *info;
    int *cycle;          /* [n_inst][n_start] or NULL */
    long long next;      /* shared work counter */
    pthread_mutex_t lock;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *B = (batch_job *)arg;
    int n = B->S->n;
    long long total = (long long)B->n_inst * B->n_start;
    orc_homotopy Hm;
    Hm.S = B->S;
    Hm.kind = B->kind;
    Hm.c0 = B->c0;
    orc_degrees(B->S, Hm.deg);
    for (;;) {
        pthread_mutex_lock(&B->lock);
        long long w = B->next++;
        pthread_mutex_unlock(&B->lock);
        if (w >= total) break;
        int inst = (int)(w / B->n_start);
        long long trk = w % B->n_start;
        Hm.c1 = B->c1 + (size_t)inst * B->S->n_terms;
        Hm.gamma = B->gamma ? B->gamma[inst] : 1.0;
        cplx x0[ORC_MAXN];
        if (B->start) memcpy(x0, B->start + (size_t)trk * n, sizeof(cplx) * n);
        else orc_total_degree_start(n, Hm.deg, trk, x0);
        orc_info inf;
        int cyc = 0;
        int st = track_one_eg(&Hm, B->o, B->eg, x0, B->endpoints + (size_t)w * n, &inf, &cyc);
        B->status[w] = st;
        if (B->info) B->info[w] = inf;
        if (B->cycle) B->cycle[w] = cyc;
    }
    return NULL;
}

/* Track n_start paths for each of n_inst target instances.
 *   c1:    [n_inst][n_terms] target coefficients
 *   c0:    [n_terms] start coefficients (LINEAR only)
 *   gamma: [n_inst] (TOTAL_DEGREE only; NULL = 1)
 *   start: [n_start][n] start points, or NULL for the total-degree start points
 *   eg:    end-game options, or NULL for none (then every path is orc_track_one's)
 * Outputs endpoints [n_inst][n_start][n], status and (optional) info and cycle
 * [n_inst][n_start].  Uses n_threads POSIX threads.  Returns 0, or -1 on bad input. */
int orc_track_batch_eg(const orc_system *S, int kind, const cplx *c0, const cplx *c1,
                       const cplx *gamma, const cplx *start, int n_start, int n_inst,
                       const orc_opts *o, const orc_eg_opts *eg, int n_threads,
                       cplx *endpoints, int *status, orc_info *info, int *cycle)
{
    if (!S || S->n < 1 || S->n > ORC_MAXN || n_start < 0 || n_inst < 0) return -1;
    if (kind == ORC_LINEAR && !c0) return -1;
    if (kind == ORC_LINEAR && !start) return -1;
    if (eg && (eg->max_samples < 0 || !(eg->beta > 0.0 && eg->beta < 1.0) || eg->max_cycle < 1)) return -1;
    batch_job B;
    B.S = S; B.kind = kind; B.c0 = c0; B.c1 = c1; B.gamma = gamma; B.start = start;
    B.n_start = n_start; B.n_inst = n_inst; B.o = o; B.eg = eg; B.cycle = cycle;
    B.endpoints = endpoints; B.status = status; B.info = info;
    B.next = 0;
    pthread_mutex_init(&B.lock, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    for (int i = 0; i < n_threads; i++) pthread_create(&th[i], NULL, batch_worker, &B);
    for (int i = 0; i < n_threads; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&B.lock);
    return 0;
}

/* orc_track_batch_eg without the end-game. */
int orc_track_batch(const orc_system *S, int kind, const cplx *c0, const cplx *c1,
                    const cplx *gamma, const cplx *start, int n_start, int n_inst,
                    const orc_opts *o, int n_threads,
                    cplx *endpoints, int *status, orc_info *info)
{
    return orc_track_batch_eg(S, kind, c0, c1, gamma, start, n_start, n_inst, o, NULL, n_threads,
                              endpoints, status, info, NULL);
}

/* ---- pieces exposed for the pins ------------------------------------------------------ */

static void make_homotopy(orc_homotopy *Hm, const orc_system *S, int kind, const cplx *c0,
                          const cplx *c1, cplx gamma)
{
    Hm->S = S; Hm->kind = kind; Hm->c0 = c0; Hm->c1 = c1; Hm->gamma = gamma;
    orc_degrees(S, Hm->deg);
}

/* H, H_x, H_t at (x, t); gamma passed as (re, im). */
void orc_homotopy_eval_flat(const orc_system *S, int kind, const cplx *c0, const cplx *c1,
                            double gre, double gim, const cplx *x, double t,
                            cplx *H, cplx *Hx, cplx *Ht)
{
    orc_homotopy Hm;
    make_homotopy(&Hm, S, kind, c0, c1, gre + I * gim);
    orc_homotopy_eval(&Hm, x, t, H, Hx, Ht);
}

/* Integrate dx/dt = -H_x^{-1} H_t from t = 0 to 1 with n_steps equal RK4 steps and no
 * corrector (used to check the order of the predictor).  Returns 1 on a zero pivot. */
int orc_rk4_fixed(const orc_system *S, int kind, const cplx *c0, const cplx *c1,
                  double gre, double gim, const cplx *x0, int n_steps, cplx *x_out)
{
    orc_homotopy Hm;
    make_homotopy(&Hm, S, kind, c0, c1, gre + I * gim);
    int n = S->n;
    cplx x[ORC_MAXN], xs[ORC_MAXN];
    for (int j = 0; j < n; j++) x[j] = x0[j];
    double h = 1.0 / n_steps;
    for (int s = 0; s < n_steps; s++) {
        double t = s * h;
        double tn = (s + 1 == n_steps) ? 1.0 : (s + 1) * h;
        if (rk4_step(&Hm, x, t, tn - t, tn, xs)) return 1;
        for (int j = 0; j < n; j++) x[j] = xs[j];
    }
    for (int j = 0; j < n; j++) x_out[j] = x[j];
    return 0;
}

/* The end-game's estimator on its own: cycle number and extrapolated value from
 * three samples of an m-vector at s, beta s, beta^2 s.  Returns 1 if the samples
 * do not decay. */
int orc_eg_extrapolate(int m, const cplx *y0, const cplx *y1, const cplx *y2, double beta, int max_cycle,
                       int *c, cplx *E)
{
    if (m < 1 || m > ORC_MAXN + 1) return 1;
    return eg_estimate(m, y0, y1, y2, beta, max_cycle, c, E);
}

/* Plain Newton on H(., t) from x0 for `iters` iterations; norms[k] = ||dx_k||_2. */
int orc_newton_trace(const orc_system *S, int kind, const cplx *c0, const cplx *c1,
                     double gre, double gim, const cplx *x0, double t, int iters,
                     double *norms, cplx *x_out)
{
    orc_homotopy Hm;
    make_homotopy(&Hm, S, kind, c0, c1, gre + I * gim);
    int n = S->n;
    cplx x[ORC_MAXN], d[ORC_MAXN];
    for (int j = 0; j < n; j++) x[j] = x0[j];
    for (int k = 0; k < iters; k++) {
        if (newton_delta(&Hm, x, t, d)) return 1;
        for (int j = 0; j < n; j++) x[j] += d[j];
        norms[k] = norm2(n, d);
    }
    for (int j = 0; j < n; j++) x_out[j] = x[j];
    return 0;
}

// hc_wave.hip -- a latency-oriented FP64 tracker for dense quadratic total-degree
// systems (n <= 8): one path per wavefront, one entry of the n x n Jacobian per
// lane.
//
// The group trackers put one path on G lanes (one matrix row per lane) so a
// wavefront carries 64 / G paths: the right shape for throughput, but a lone
// path's stage is then a long chain per lane (its whole row build, the pivot
// chain, the back substitution), about 5 us.  Passes that track only a few
// paths -- the crossing check's re-tracking from t = 0, the end-game's samples --
// are bound by exactly that chain.  Here lane (i, j) = (lane >> 3, lane & 7)
// holds H_x[i][j]: building it is n multiply-adds per lane, the right-hand side
// row i a reduction over the 8 lanes of the row (Euler's identity for the
// quadratic part, as in the group trackers), and each elimination step of the
// LU with partial pivoting (section 6: the augmented matrix, then back
// substitution with U) is one multiply-add per lane after a pivot search over
// column k (readlane of the 8 candidates) and an exchange of the pivot row and
// the multipliers' column across lanes (ds_bpermute, readlane).  The path state (x, t, h, counters) is uniform
// across the wavefront; every lane takes the same decisions.
//
// Same stage machine, step control and statuses as the group trackers (RK4
// predictor, Newton corrector with the first-correction guard, growth after
// n_inc accepts, clipping to t_final), so its paths follow the oracle's within
// rounding.
#include "hc_device.h"

namespace hcx {

namespace {

template <int N>
struct WaveLds {
    cx<double> u[N][N + 1]; // rows of U in pivot order, then back substitution
};

// Orders this wavefront's LDS accesses around it in program order only: a
// wavefront's LDS instructions execute in issue order, so the back substitution
// reads the rows of U the elimination wrote, and the next stage's writes cannot
// overtake this stage's reads.
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

// Lane src's value of v in every lane (src per lane, in range).
__device__ __forceinline__ double bperm(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double rdl(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int CTRL>
__device__ __forceinline__ double dppd(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the 8 lanes of a row (xor 1, xor 2 in quads, then the half-row
// mirror): every lane of the row ends with the same value.
__device__ __forceinline__ double row_sum(double v)
{
    v = v + dppd<0xB1>(v);
    v = v + dppd<0x4E>(v);
    v = v + dppd<0x141>(v);
    return v;
}

// Component-wise select (a select of whole structs can turn into a select of
// their addresses, which moves the arrays they come from to scratch memory).
__device__ __forceinline__ cx<double> pick(bool s, cx<double> a, cx<double> b)
{
    return {s ? a.re : b.re, s ? a.im : b.im};
}

// The coefficients lane (i, j) needs, read once per path from the instance's
// kernel table (row i: constant, L_i, then c_ab for a <= b with c_aa doubled):
// the constant of row i, L_ij and c_(jb) for every b.
template <int N>
struct WaveCoef {
    cx<double> c0, L, q[N];
};

template <int N>
__device__ __forceinline__ void load_coef(const double *tab, WaveCoef<N> &w)
{
    constexpr int T = dense_terms(N);
    const int lane = threadIdx.x & 63;
    const int i = lane >> 3, j = lane & 7;
    const int ii = i < N ? i : 0, jj = j < N ? j : 0;
    const double *c = tab + (size_t)ii * T * 2;
    w.c0 = {c[0], c[1]};
    w.L = {c[2 * (1 + jj)], c[2 * (1 + jj) + 1]};
#pragma unroll
    for (int b = 0; b < N; b++) {
        const int q = jj <= b ? quad_slot(N, jj, b) : quad_slot(N, b, jj);
        w.q[b] = {c[2 * q], c[2 * q + 1]};
    }
}

// One stage: dx solves H_x dx = -H_t (pred) or -H at (x, t) for the total-degree
// homotopy H = (1 - t) gamma G + t F.  Returns true on an exactly zero pivot.
// dx and nd2 = |dx|^2 are uniform.
template <int N>
__device__ __forceinline__ bool wave_stage(const WaveCoef<N> &w, cx<double> gam, unsigned deg2,
                                           const cx<double> (&x)[N], double t, bool pred, WaveLds<N> &L,
                                           cx<double> (&dx)[N], double &nd2)
{
    const int lane = threadIdx.x & 63;
    const int i = lane >> 3, j = lane & 7;
    const bool ent = i < N && j < N;
    const int ii = i < N ? i : 0, jj = j < N ? j : 0;
    // F_x[i][j] = L_ij + sum_b c_(jb) x_b, the table holding 2 c_jj
    const cx<double> Lij = w.L;
    cx<double> J = Lij;
#pragma unroll
    for (int b = 0; b < N; b++) J = cfma(w.q[b], x[b], J);
    // F_i = c_i + (L_i . x + F_x[i] . x) / 2 (Euler's identity for the quadratic part)
    cx<double> xj = x[0];
#pragma unroll
    for (int b = 1; b < N; b++) xj = pick(jj == b, x[b], xj);
    cx<double> e = pick(ent, cmul(cx<double>{Lij.re + J.re, Lij.im + J.im}, xj), cx<double>{0.0, 0.0});
    e = {row_sum(e.re), row_sum(e.im)};
    const cx<double> F = {w.c0.re + 0.5 * e.re, w.c0.im + 0.5 * e.im};
    // G_i = x_i^d_i - 1 and its derivative
    cx<double> xi = x[0];
#pragma unroll
    for (int b = 1; b < N; b++) xi = pick(ii == b, x[b], xi);
    const bool d2 = (deg2 >> ii) & 1u;
    cx<double> G = pick(d2, cmul(xi, xi), xi);
    G.re -= 1.0;
    const cx<double> dG = pick(d2, cx<double>{2.0 * xi.re, 2.0 * xi.im}, cx<double>{1.0, 0.0});
    const double omt = 1.0 - t;
    const cx<double> gG = cmul(gam, G), gdG = cmul(gam, dG);
    cx<double> a = pick(ent, cscale(t, J), cx<double>{(i == j) ? 1.0 : 0.0, 0.0});
    if (ent && i == j) a = {a.re + omt * gdG.re, a.im + omt * gdG.im};
    cx<double> rhs;
    if (pred)
        rhs = {gG.re - F.re, gG.im - F.im};                                      // -(F - gamma G)
    else
        rhs = {-fma(t, F.re, omt * gG.re), -fma(t, F.im, omt * gG.im)};          // -H
    if (i >= N) rhs = {0.0, 0.0};

    // LU with partial pivoting, no row moves: piv holds the pivotal rows
    unsigned piv = 0;
    bool sing = false;
    cx<double> inv[N];  // reciprocals of the pivots (uniform), reused by the back substitution
#pragma unroll
    for (int k = 0; k < N; k++) {
        // pivot: the largest |Re| + |Im| in column k among the rows not yet pivotal
        const unsigned key = (j == k && i < N && !((piv >> i) & 1u))
                                 ? ((__float_as_uint((float)abs1(a)) & ~7u) | (unsigned)(7 - i))
                                 : 0u;
        unsigned best = 0;
#pragma unroll
        for (int r = 0; r < N; r++) best = max(best, (unsigned)__builtin_amdgcn_readlane((int)key, r * 8 + k));
        const int p = 7 - (int)(best & 7u);
        sing |= (best & ~7u) == 0u;
        piv |= 1u << p;
        // the pivot row is row k of U (in pivot order) for the back
        // substitution, which reads it after the elimination: stored now, no
        // wait here
        if (i == p && j >= k && j < N) L.u[k][j] = a;
        if (i == p && j == 0) L.u[k][N] = rhs;
        // the pivot row's entries and column k reach every lane across the
        // wavefront's lanes (ds_bpermute, and readlane for the uniform pivot
        // and right-hand side) rather than through an LDS round trip
        const cx<double> pk = {rdl(a.re, p * 8 + k), rdl(a.im, p * 8 + k)};
        const cx<double> pb = {rdl(rhs.re, p * 8), rdl(rhs.im, p * 8)};
        const cx<double> pr = {bperm(a.re, p * 8 + jj), bperm(a.im, p * 8 + jj)};
        const cx<double> aik = {bperm(a.re, ii * 8 + k), bperm(a.im, ii * 8 + k)};
        inv[k] = crecip(pk);
        const cx<double> l = cmul(aik, inv[k]);
        if (!((piv >> i) & 1u) && i < N) {
            if (j > k && j < N) a = cfms(l, pr, a);
            rhs = cfms(l, pb, rhs);
        }
        lds_order();
    }
    // back substitution with U (uniform: every lane reads the rows from LDS)
    nd2 = 0.0;
#pragma unroll
    for (int k = N - 1; k >= 0; k--) {
        cx<double> s = L.u[k][N];
#pragma unroll
        for (int q = k + 1; q < N; q++) s = cfms(L.u[k][q], dx[q], s);
        dx[k] = cmul(s, inv[k]);
        nd2 += abs2(dx[k]);
    }
    lds_order();
    return sing;
}

}  // namespace

// The paths still RUNNING below t_final, compacted into list[0 .. *count) (in no
// particular order: each path's result does not depend on which wavefront runs
// it).
__global__ __launch_bounds__(256) void k_list_running(const TrackArgs a, int *list, unsigned *count)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < a.total && a.s.status[g] == kRunning && a.s.t[g] < a.t_final) list[atomicAdd(count, 1u)] = (int)g;
}

// Wavefront w tracks the listed paths w, w + W, ... (W = the grid's wavefronts)
// to t_final, one path per wavefront as long as there are no more than W.
template <int N>
__global__ __launch_bounds__(64) void k_track_wave(const TrackArgs a, const int *list, const unsigned *count)
{
    __shared__ WaveLds<N> L;
    constexpr int T = dense_terms(N);
    const TrackState S = a.s;
    const long long total = a.total;
    const long long m = (long long)*count;
    for (long long idx = blockIdx.x; idx < m; idx += gridDim.x) {
      {
        const long long g = list[idx];
        const int inst = (int)(g / a.n_start);
        WaveCoef<N> wc;
        load_coef<N>(static_cast<const double *>(a.coef) + (size_t)inst * N * T * 2, wc);
        cx<double> gam = {1.0, 0.0};
        if (a.gamma) gam = {a.gamma[2 * inst], a.gamma[2 * inst + 1]};
        cx<double> x[N], xe[N], acc[N];
#pragma unroll
        for (int q = 0; q < N; q++) x[q] = {S.xr[q * total + g], S.xi[q * total + g]};
        double t = S.t[g], h = S.h[g], te = t, hu = 0.0, tn = t;
        int succ = S.succ[g], steps = S.steps[g], rejects = S.rejects[g], nits = S.nits[g], escal = S.escal[g];
        int phase = 0, nit = 0, lsteps = 0, st = kRunning;
        unsigned long long stages = 0;
        bool go = true;
        bool begin = true;  // start a step (clip it to t_final) before the next stage
        if (steps_used(steps, rejects, escal) >= a.max_steps) {
            st = HC_T_MAX_STEPS;
            go = false;
        }
        while (go) {
            if (begin) {
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
                for (int q = 0; q < N; q++) xe[q] = x[q];
                te = t;
                begin = false;
            }
            const bool pred = phase < 4;
            cx<double> d[N];
            double nd2;
            const bool sing = wave_stage<N>(wc, gam, a.deg2, xe, te, pred, L, d, nd2);
            stages++;
            int ev = 0;  // 1 accept, 2 reject, 3 failed (st)
            if (phase < 4) {
                if (sing) {
                    ev = 2;
                } else if (phase == 0 && !isfinite(nd2)) {
                    ev = 3;
                    st = HC_T_NONFINITE;
                } else {
                    const double w = (phase == 0 || phase == 3) ? 1.0 : 2.0;
                    const double cc = phase < 2 ? 0.5 * hu : hu;
#pragma unroll
                    for (int q = 0; q < N; q++) {
                        acc[q].re = phase == 0 ? d[q].re : fma(w, d[q].re, acc[q].re);
                        acc[q].im = phase == 0 ? d[q].im : fma(w, d[q].im, acc[q].im);
                        xe[q].re = phase == 3 ? fma(hu / 6.0, acc[q].re, x[q].re) : fma(cc, d[q].re, x[q].re);
                        xe[q].im = phase == 3 ? fma(hu / 6.0, acc[q].im, x[q].im) : fma(cc, d[q].im, x[q].im);
                    }
                    te = phase == 0 || phase == 1 ? t + 0.5 * hu : tn;
                    nit = 0;
                    phase++;
                    if (phase == 4 && a.max_newton <= 0) ev = 2;
                }
            } else if (sing) {
                ev = 2;
            } else {
                double nx2 = 0.0;
#pragma unroll
                for (int q = 0; q < N; q++) {
                    xe[q] = {xe[q].re + d[q].re, xe[q].im + d[q].im};
                    nx2 += abs2(xe[q]);
                }
                const double nx = sqrt(nx2), nd = sqrt(nd2);
                nit++;
                nits++;
                if (nit == 1 && !(nd <= a.pred_tol * (1.0 + nx)))
                    ev = 2;
                else if (nd <= a.tau64 * (1.0 + nx))
                    ev = 1;
                else if (nit >= a.max_newton)
                    ev = 2;
            }
            bool next_step = false;
            if (ev == 1) {
                double big = 0.0;
                bool nan_ = false;
#pragma unroll
                for (int q = 0; q < N; q++) {
                    x[q] = xe[q];
                    const double m2 = abs2(x[q]);
                    big = fmax(big, m2);
                    nan_ = nan_ || isnan(m2);
                }
                t = tn;
                steps++;
                lsteps++;
                if (++succ >= a.n_inc) {
                    h = fmin(h * a.beta_inc, a.h_max);
                    succ = 0;
                }
                if (nan_ || !(big <= a.inf2)) {
                    ev = 3;
                    st = nan_ ? HC_T_NONFINITE : HC_T_AT_INFINITY;
                } else if (t >= a.t_final) {
                    st = a.t_final >= 1.0 ? kReached : kRunning;
                    go = false;
                } else {
                    next_step = true;
                }
            } else if (ev == 2) {
                rejects++;
                lsteps++;
                succ = 0;
                h *= a.beta_dec;
                if (h < a.h_min) {
                    ev = 3;
                    st = HC_T_MIN_STEP;
                } else {
                    next_step = true;
                }
            }
            if (next_step) {
                if (a.launch_steps > 0 && lsteps >= a.launch_steps) {
                    if ((threadIdx.x & 63) == 0) atomicAdd(a.n_suspended, 1u);
                    st = kRunning;
                    go = false;
                } else if (steps_used(steps, rejects, escal) >= a.max_steps) {
                    st = HC_T_MAX_STEPS;
                    go = false;
                } else {
                    begin = true;
                }
            }
            if (ev == 3) go = false;
        }
        const int lane = threadIdx.x & 63;
        if (lane < N) {
            cx<double> v = x[0];
#pragma unroll
            for (int q = 1; q < N; q++) v = pick(lane == q, x[q], v);
            S.xr[lane * total + g] = v.re;
            S.xi[lane * total + g] = v.im;
        }
        if (lane == 0) {
            S.t[g] = t;
            S.h[g] = h;
            S.succ[g] = succ;
            S.steps[g] = steps;
            S.rejects[g] = rejects;
            S.nits[g] = nits;
            S.escal[g] = escal;
            S.status[g] = st;
            if (a.stage_count) atomicAdd(a.stage_count + 1, stages);
        }
      }
    }
}

template <int N>
static hipError_t launch_wave_n(const TrackArgs &a, const int *list, const unsigned *count, int waves,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_track_wave<N>, dim3((unsigned)waves), dim3(64), 0, st, a, list, count);
    return hipGetLastError();
}

hipError_t launch_track_wave(int n, const TrackArgs &a, int *list, unsigned *count, int waves, hipStream_t st)
{
    if (a.total == 0) return hipSuccess;
    if (waves < 1) waves = 1;
    hipError_t e = launch_fill_u32(count, 0u, 1, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_list_running, dim3((unsigned)((a.total + 255) / 256)), dim3(256), 0, st, a, list, count);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    switch (n) {
    case 2: return launch_wave_n<2>(a, list, count, waves, st);
    case 3: return launch_wave_n<3>(a, list, count, waves, st);
    case 4: return launch_wave_n<4>(a, list, count, waves, st);
    case 5: return launch_wave_n<5>(a, list, count, waves, st);
    case 6: return launch_wave_n<6>(a, list, count, waves, st);
    case 7: return launch_wave_n<7>(a, list, count, waves, st);
    case 8: return launch_wave_n<8>(a, list, count, waves, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hcx

// hc_track_group.hip -- path tracker with G lanes per path, one row per lane.
//
// Mapping: a wavefront holds 64/G paths; lane r of a group (G = 4 or 8, G >= n)
// owns equation r.  All groups of a wavefront work on the same instance, whose
// coefficient table sits in the wavefront's slice of LDS laid out
// coefficient-major ([term][equation]), so the lanes reading "their" equation's
// term hit distinct banks.  Each stage a lane builds row r of the augmented
// matrix [H_x | rhs].  The LU with partial pivoting then runs across the group
// (section 6: one row per thread):
//   * pivot search: a DPP max-reduction over the group of (|Re|+|Im|, row) keys;
//   * no rows move: the pivot row's remaining entries are broadcast to the group
//     with ds_bpermute and every not-yet-pivotal row eliminates against them;
//     each lane remembers the position at which its row became pivotal;
//   * back substitution walks the positions downwards, the pivot lane of each
//     position producing one unknown and broadcasting it, so every lane ends
//     with the whole solution vector.
// Path state is spread over the group: lane r holds component r of the point,
// of the stage point and of the RK4 accumulator (FP64); t, h and the counters are
// replicated and the group's lanes take identical decisions.  Per-stage latency
// is about G times shorter than with one path per lane, so the long paths of a
// batch no longer hold a wavefront for G times longer.
//
// Mixed precision (R = float): the Jacobian, the tangent right-hand sides and
// every LU run in FP32; the point is accumulated in FP64 and, with the ir
// option, a Newton stage's right-hand side H(x, t) is evaluated in FP64 --
// iterative refinement with an FP32 solver -- so the corrector reaches
// FP64-level residuals wherever the FP32 solve still contracts (condition
// number well below 2^24).
#include <type_traits>
#include <utility>

#include "hc_device.h"

namespace hcx {

namespace {

__device__ __forceinline__ unsigned umax(unsigned a, unsigned b) { return a > b ? a : b; }

template <int G>
__device__ __forceinline__ unsigned group_max(unsigned v)
{
    // xor 1 and xor 2 inside quads (quad_perm), then mirror across the half row
    // (lane i <-> 7-i) and the row (lane i <-> 15-i): every lane ends with the max
    v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    if (G >= 8) v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    if (G >= 16) v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    return v;
}

__device__ __forceinline__ float bcast(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

__device__ __forceinline__ double bcast(double v, int src)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename R>
__device__ __forceinline__ cx<R> bcast(cx<R> v, int src)
{
    return {bcast(v.re, src), bcast(v.im, src)};
}

template <typename R>
__device__ __forceinline__ cx<R> csel(bool s, cx<R> a, cx<R> b)
{
    return {s ? a.re : b.re, s ? a.im : b.im};
}

constexpr int nquad(int n) { return n * (n + 1) / 2; }

// LDS slice of one wavefront: the instance's kernel table, coefficient-major.
template <typename R>
using lds_tab = __attribute__((address_space(3))) cx<R> *;

template <typename R>
__device__ __forceinline__ cx<R> ldl(lds_tab<R> p, int i)
{
    return {p[i].re, p[i].im};
}

// Row r of [H_x | rhs] at (x, t) for H = (1-t) gamma G + t F (see build_td in
// hc_kernels.hip for the formulas): the lane's own equation, its terms read from
// the LDS table (term q of equation r at cl[q * N + r]).
template <int N, typename R>
__device__ __forceinline__ void build_row(lds_tab<R> cl, int r, bool d2, cx<R> gam, const cx<R> (&x)[N], R t,
                                          bool pred, cx<R> (&row)[N + 1])
{
    const int rr = r < N ? r : N - 1;  // padding lanes read a real row and are ignored
    cx<R> Lx = {R(0), R(0)};
#pragma unroll
    for (int j = 0; j < N; j++) {
        const cx<R> L = ldl(cl, (1 + j) * N + rr);
        row[j] = L;
        Lx = cfma(L, x[j], Lx);
    }
    int q = 1 + N;
#pragma unroll
    for (int a = 0; a < N; a++) {
#pragma unroll
        for (int b = a; b < N; b++) {
            const cx<R> cq = ldl(cl, (q++) * N + rr);
            if (a == b) {
                row[a] = cfma(cq, x[a], row[a]);
            } else {
                row[a] = cfma(cq, x[b], row[a]);
                row[b] = cfma(cq, x[a], row[b]);
            }
        }
    }
    cx<R> s = Lx;
#pragma unroll
    for (int j = 0; j < N; j++) s = cfma(x[j], row[j], s);
    const cx<R> c0 = ldl(cl, rr);
    const cx<R> F = {fma(R(0.5), s.re, c0.re), fma(R(0.5), s.im, c0.im)};
    cx<R> xr = x[0];
#pragma unroll
    for (int j = 1; j < N; j++) xr = csel(r == j, x[j], xr);
    cx<R> Gv, dG;
    if (d2) {
        Gv = cmul(xr, xr);
        Gv.re -= R(1);
        dG = {R(2) * xr.re, R(2) * xr.im};
    } else {
        Gv = {xr.re - R(1), xr.im};
        dG = {R(1), R(0)};
    }
    const R omt = R(1) - t;
    const cx<R> gG = cmul(gam, Gv);
    const cx<R> gdG = cmul(gam, dG);
    const cx<R> dterm = {omt * gdG.re, omt * gdG.im};
#pragma unroll
    for (int j = 0; j < N; j++) {
        row[j] = cscale(t, row[j]);
        row[j].re += (j == r) ? dterm.re : R(0);
        row[j].im += (j == r) ? dterm.im : R(0);
    }
    const cx<R> Ht = {F.re - gG.re, F.im - gG.im};
    const cx<R> H = {fma(t, F.re, omt * gG.re), fma(t, F.im, omt * gG.im)};
    row[N] = csel(pred, cx<R>{-Ht.re, -Ht.im}, cx<R>{-H.re, -H.im});
}

// H_r(x, t) in FP64 for the total-degree homotopy, with the (FP32) table terms
// widened to FP64: the residual of the iterative-refinement corrector.  F_r is
// summed row by row, F = c + sum_a x_a (L_a + sum_{b >= a} c_ab x_b), which keeps
// one running sum live instead of every monomial.
template <int N, typename R>
__device__ __forceinline__ cx<double> resid_td64(lds_tab<R> cl, int r, bool d2, cx<double> gam,
                                                 const cx<double> (&x)[N], double t)
{
    const int rr = r < N ? r : N - 1;
    const cx<R> c0r = ldl(cl, rr);
    cx<double> F = {(double)c0r.re, (double)c0r.im};
    int q = 1 + N;
#pragma unroll
    for (int a = 0; a < N; a++) {
        const cx<R> L = ldl(cl, (1 + a) * N + rr);
        cx<double> y = {(double)L.re, (double)L.im};
#pragma unroll
        for (int b = a; b < N; b++) {
            const cx<R> cq = ldl(cl, (q++) * N + rr);
            const double w = a == b ? 0.5 : 1.0;  // the table holds 2 c_aa
            y = cfma(cx<double>{w * (double)cq.re, w * (double)cq.im}, x[b], y);
        }
        F = cfma(x[a], y, F);
    }
    cx<double> xr = x[0];
#pragma unroll
    for (int j = 1; j < N; j++) xr = csel(r == j, x[j], xr);
    cx<double> Gv = d2 ? cmul(xr, xr) : xr;
    Gv.re -= 1.0;
    const cx<double> gG = cmul(gam, Gv);
    return {fma(t, F.re, (1.0 - t) * gG.re), fma(t, F.im, (1.0 - t) * gG.im)};
}

// Blended coefficient ct = (1-t) c0 + t c1 of term q, and the coefficient cr of
// the right-hand side: c1 - c0 for a predictor stage (H_t), ct otherwise (H).
template <typename R>
__device__ __forceinline__ void blend_coef(const R *e0, const R *e1, int q, R t, R omt, bool pred, cx<R> &ct,
                                           cx<R> &cr)
{
    const cx<R> a = {e0[2 * q], e0[2 * q + 1]};
    const cx<R> b = {e1[2 * q], e1[2 * q + 1]};
    ct = {fma(t, b.re, omt * a.re), fma(t, b.im, omt * a.im)};
    const cx<R> d = {b.re - a.re, b.im - a.im};
    cr = csel(pred, d, ct);
}

template <int N, typename R>
__device__ __forceinline__ void build_row_param(const R *e0, const R *e1, const cx<R> (&x)[N], R t, bool pred,
                                                cx<R> (&row)[N + 1])
{
    const R omt = R(1) - t;
    auto coefs = [&](int q, cx<R> &ct, cx<R> &cr) { blend_coef<R>(e0, e1, q, t, omt, pred, ct, cr); };
    cx<R> ct, cr;
    coefs(0, ct, cr);
    cx<R> F = cr;
#pragma unroll
    for (int j = 0; j < N; j++) {
        coefs(1 + j, ct, cr);
        row[j] = ct;
        F = cfma(cr, x[j], F);
    }
    int q = 1 + N;
#pragma unroll
    for (int a = 0; a < N; a++) {
#pragma unroll
        for (int b = a; b < N; b++) {
            coefs(q++, ct, cr);
            const cx<R> m = cmul(x[a], x[b]);
            if (a == b) {
                row[a] = cfma(ct, x[a], row[a]);
                F = cfma(cscale(R(0.5), cr), m, F);  // the table holds 2 c_aa
            } else {
                row[a] = cfma(ct, x[b], row[a]);
                row[b] = cfma(ct, x[a], row[b]);
                F = cfma(cr, m, F);
            }
        }
    }
    row[N] = {-F.re, -F.im};
}

// H_r(x, t) = F_r(x; (1-t) c0 + t c1) in FP64 from the lane's two table rows,
// summed row by row as in resid_td64.
template <int N, typename R>
__device__ __forceinline__ cx<double> resid_param64(const R *e0, const R *e1, const cx<double> (&x)[N], double t)
{
    const double omt = 1.0 - t;
    auto coef = [&](int q) {
        return cx<double>{fma(t, (double)e1[2 * q], omt * (double)e0[2 * q]),
                          fma(t, (double)e1[2 * q + 1], omt * (double)e0[2 * q + 1])};
    };
    cx<double> F = coef(0);
    int q = 1 + N;
#pragma unroll
    for (int a = 0; a < N; a++) {
        cx<double> y = coef(1 + a);
#pragma unroll
        for (int b = a; b < N; b++) {
            cx<double> c = coef(q++);
            if (a == b) c = {0.5 * c.re, 0.5 * c.im};
            y = cfma(c, x[b], y);
        }
        F = cfma(x[a], y, F);
    }
    return F;
}

// Lane J of each group of G lanes, read by every lane of the group: ds_swizzle in
// bit mode, whose and-mask keeps the group's base inside the 32-lane half and
// whose or-mask adds J (groups never straddle a half).
template <int G, int J>
__device__ __forceinline__ int gbc(int v)
{
    return __builtin_amdgcn_ds_swizzle(v, (0x1F & ~(G - 1)) | (J << 5));
}

template <int G, int J>
__device__ __forceinline__ float gbc(float v)
{
    return __int_as_float(gbc<G, J>(__float_as_int(v)));
}

template <int G, int J>
__device__ __forceinline__ double gbc(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = gbc<G, J>((int)(b & 0xffffffffll));
    const int hi = gbc<G, J>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int G, typename T, int N, int... J>
__device__ __forceinline__ void gather_impl(const cx<T> v, cx<T> (&out)[N], std::integer_sequence<int, J...>)
{
    ((out[J] = cx<T>{gbc<G, J>(v.re), gbc<G, J>(v.im)}), ...);
}

// out[j] = v of lane j of this lane's group, j < N.
template <int G, int N, typename T>
__device__ __forceinline__ void gather(const cx<T> v, cx<T> (&out)[N])
{
    gather_impl<G>(v, out, std::make_integer_sequence<int, N>{});
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the G lanes of a group by butterflies (xor 1, xor 2, then the half-row
// and row mirrors).  Each step adds the same two operands on both sides of a
// pair, so every lane of the group ends with the identical sum.  The whole group
// must be active.
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
    v = v + dpp<0xB1>(v);
    v = v + dpp<0x4E>(v);
    if (G >= 8) v = v + dpp<0x141>(v);
    if (G >= 16) v = v + dpp<0x140>(v);
    return v;
}

// True in every lane of the group if p holds in any of its lanes.
template <int G>
__device__ __forceinline__ bool group_any(bool p, int base)
{
    return ((ballot(p) >> base) & ((1ull << G) - 1ull)) != 0ull;
}

// Solves the group's n x n system [A | b] (row r in this lane) by elimination
// with partial pivoting across the group.  Lane r receives component r of the
// solution in dxr (0 in padding lanes) and every lane the squared 2-norm of the
// whole solution in nd (summed in the same order everywhere, so identical in the
// group).  Must run with the whole wavefront active.  Returns true if a pivot is
// (numerically) zero.
template <int N, int G, typename R>
__device__ __forceinline__ bool group_solve(cx<R> (&row)[N + 1], int r, int base, cx<R> &dxr, R &nd)
{
    constexpr unsigned GM = G - 1;
    int pos = r < N ? -1 : 4 * G;  // position at which this row became pivotal
    int pl[N];                     // group-relative lane of the pivot of each position
    cx<R> inv_own = {R(0), R(0)};
    bool sing = false;
#pragma unroll
    for (int k = 0; k < N; k++) {
        const float v = (float)abs1(row[k]);
        const unsigned key = pos < 0 ? (0x80000000u | (__float_as_uint(v) & ~GM) | (GM - (unsigned)r)) : 0u;
        const unsigned kmax = group_max<G>(key);
        const int p = (int)(GM - (kmax & GM));
        sing |= ((kmax & 0x7fffffffu & ~GM) == 0u);
        pl[k] = p;
        cx<R> P[N + 1];
#pragma unroll
        for (int c = k; c <= N; c++) P[c] = bcast(row[c], base + p);
        const cx<R> inv = crecip(P[k]);
        const bool piv = (r == p);
        pos = piv ? k : pos;
        inv_own = csel(piv, inv, inv_own);
        cx<R> l = cmul(row[k], inv);
        l = csel(pos < 0, l, cx<R>{R(0), R(0)});
#pragma unroll
        for (int c = k + 1; c <= N; c++) row[c] = cfms(l, P[c], row[c]);
    }
    cx<R> b = row[N];
    dxr = {R(0), R(0)};
    nd = R(0);
#pragma unroll
    for (int k = N - 1; k >= 0; k--) {
        const cx<R> xk = bcast(cmul(b, inv_own), base + pl[k]);
        dxr = csel(r == k, xk, dxr);
        nd = fma(xk.re, xk.re, fma(xk.im, xk.im, nd));
        const bool above = pos < k;
        b = csel(above, cfms(row[k], xk, b), b);
    }
    return sing;
}

}  // namespace

// Tracks the paths tb .. tend-1 of instance `inst` with the wavefront's lane
// groups until every one of them has ended or been suspended.  Called with the
// whole wavefront active and wavefront-uniform arguments.  `lds` is this
// wavefront's table slice (room for 8 x 45 complex values of R).
//
// Path state is distributed over the group: lane r < n holds component r of the
// accepted point x, of the stage point xe and of the RK4 accumulator, all in
// FP64; t, h and the counters are replicated and every lane of a group takes the
// same decisions (the group's sums and tests are computed identically in all of
// its lanes).  Each stage gathers the whole stage point into every lane of the
// group (ds_swizzle), builds the lane's row, solves, and each lane updates its
// own component.
template <int N, int G, typename R, bool PARAM>
__device__ __forceinline__ void run_item(const TrackArgs &a, const int inst, const int tb, const int tend,
                                         cx<R> *lds)
{
    static_assert(G == 4 || G == 8 || G == 16, "group size");
    static_assert(N <= G, "one row per lane");
    constexpr bool R64 = sizeof(R) == 8;
    constexpr int T = dense_terms(N);
    const int lane = threadIdx.x & 63;
    const int r = lane & (G - 1);
    const int base = lane - r;
    const bool own = r < N;  // lane holds a component of the path state
    // mixed precision: FP64 corrector right-hand side around the FP32 solves
    const bool ir = !R64 && a.ir;
    cx<R> gam = {R(1), R(0)};
    if (a.gamma) gam = {R(a.gamma[2 * inst]), R(a.gamma[2 * inst + 1])};
    const cx<double> gam64 = {a.gamma ? a.gamma[2 * inst] : 1.0, a.gamma ? a.gamma[2 * inst + 1] : 0.0};
    const long long gbase = (long long)inst * a.n_start;
    const long long total = a.total;
    const TrackState S = a.s;
    const double tau = a.tau, pred_tol = a.pred_tol;
    const bool d2 = own && ((a.deg2 >> r) & 1u);

    // total degree: stage the instance's table in LDS, coefficient-major
    if (!PARAM) {
        const R *ce = static_cast<const R *>(a.coef) + (size_t)inst * N * T * 2;
        for (int e = lane; e < N * T; e += 64) {
            const int eq = e / T, q = e - eq * T;
            lds[q * N + eq] = {ce[2 * e], ce[2 * e + 1]};
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    const lds_tab<R> cl0 = (lds_tab<R>)lds;
    // parameter homotopy: the lane's start and target rows (padding lanes read row 0)
    const R *row0 = static_cast<const R *>(a.coef0) + (size_t)(own ? r : 0) * T * 2;
    const R *row1 = static_cast<const R *>(a.coef) + ((size_t)inst * N + (own ? r : 0)) * T * 2;

    int trk = -1;
    long long g = 0;
    cx<double> x = {0.0, 0.0}, xe = {0.0, 0.0}, acc = {0.0, 0.0};  // component r
    double t = 0.0, h = 0.0, te = 0.0, hu = 0.0, tn = 0.0;
    int phase = 0, nit = 0, succ = 0, steps = 0, rejects = 0, nits = 0, lsteps = 0, escal = 0;
    unsigned lstages = 0;
    int next = tb;

    auto save = [&](int st) {
        if (own) {
            S.xr[r * total + g] = x.re;
            S.xi[r * total + g] = x.im;
        }
        if (r == 0) {
            S.t[g] = t;
            S.h[g] = h;
            S.succ[g] = succ;
            S.steps[g] = steps;
            S.rejects[g] = rejects;
            S.nits[g] = nits;
            S.escal[g] = escal;
            S.status[g] = st;
            if (a.stage_count) atomicAdd(a.stage_count, (unsigned long long)lstages);
        }
        lstages = 0;
        trk = -1;
    };
    auto begin_step = [&]() {
        const double rem = a.t_final - t;
        if (h >= rem) {
            hu = rem;
            tn = a.t_final;
        } else {
            hu = h;
            tn = t + h;
        }
        phase = 0;
        xe = x;
        te = t;
    };
    // failures the FP32 pass cannot resolve go back to RUNNING for the FP64 pass
    auto fail = [&](int st) {
        if (a.escalate && st != HC_T_AT_INFINITY) {
            escal = 1;
            h = a.h0;
            succ = 0;
            st = kRunning;
        }
        save(st);
    };
    auto refill = [&]() {
        for (;;) {
            const unsigned long long need = ballot(trk < 0 && r == 0);
            if (need == 0ull || next >= tend) break;
            const int cand = next + __popcll(need & ((1ull << base) - 1ull));
            next += __popcll(need);
            if (trk < 0 && cand < tend) {
                const long long gg = gbase + cand;
                // still going, not yet at this pass's end time, and (in the FP32
                // pass) not already handed over to FP64
                if (S.status[gg] == kRunning && S.t[gg] < a.t_final && !(a.escalate && S.escal[gg])) {
                    trk = cand;
                    g = gg;
                    x = own ? cx<double>{S.xr[r * total + g], S.xi[r * total + g]} : cx<double>{0.0, 0.0};
                    t = S.t[g];
                    h = S.h[g];
                    succ = S.succ[g];
                    steps = S.steps[g];
                    rejects = S.rejects[g];
                    nits = S.nits[g];
                    escal = S.escal[g];
                    lsteps = 0;
                    if (steps + rejects >= a.max_steps)
                        fail(HC_T_MAX_STEPS);
                    else
                        begin_step();
                }
            }
        }
    };

    refill();
    while (ballot(trk >= 0) != 0ull) {
        const bool act = trk >= 0;
        const bool pred = phase < 4;
        // the whole stage point in every lane of the group
        cx<R> xs[N];
        cx<double> xa[N];
        const bool wide = R64 || ir;
        if (wide) {
            gather<G, N>(xe, xa);
#pragma unroll
            for (int j = 0; j < N; j++) xs[j] = {R(xa[j].re), R(xa[j].im)};
        } else {
            gather<G, N>(cx<R>{R(xe.re), R(xe.im)}, xs);
        }
        cx<R> row[N + 1];
        if constexpr (PARAM) {
            // re-derived each stage so the loop-invariant table reads are not all
            // hoisted out of the loop into registers
            const R *p0 = row0, *p1 = row1;
            asm volatile("" : "+v"(p0), "+v"(p1));
            build_row_param<N, R>(p0, p1, xs, R(te), pred, row);
            if (ir && !pred) {
                const cx<double> H = resid_param64<N, R>(p0, p1, xa, te);
                row[N] = {R(-H.re), R(-H.im)};
            }
        } else {
            lds_tab<R> cl = cl0;
            asm volatile("" : "+v"(cl));
            build_row<N, R>(cl, r, d2, gam, xs, R(te), pred, row);
            if (ir && !pred) {
                const cx<double> H = resid_td64<N, R>(cl, r, d2, gam64, xa, te);
                row[N] = {R(-H.re), R(-H.im)};
            }
        }
        cx<R> dxr;
        R nd2;
        const bool sing = group_solve<N, G, R>(row, r, base, dxr, nd2);
        const cx<double> d = {(double)dxr.re, (double)dxr.im};

        if (act) {
            lstages++;
            // 0: stage done, 1: accept the step, 2: reject it, 3: path failed (fst)
            int ev = 0, fst = 0;
            if (phase < 4) {
                if (sing) {
                    ev = 2;
                } else if (phase == 0 && !isfinite(nd2)) {
                    ev = 3;
                    fst = HC_T_NONFINITE;
                } else {
                    const double w = (phase == 0 || phase == 3) ? 1.0 : 2.0;
                    acc.re = phase == 0 ? d.re : fma(w, d.re, acc.re);
                    acc.im = phase == 0 ? d.im : fma(w, d.im, acc.im);
                    const double c = phase < 2 ? 0.5 * hu : hu;
                    xe.re = phase == 3 ? fma(hu / 6.0, acc.re, x.re) : fma(c, d.re, x.re);
                    xe.im = phase == 3 ? fma(hu / 6.0, acc.im, x.im) : fma(c, d.im, x.im);
                    te = phase == 0 || phase == 1 ? t + 0.5 * hu : tn;
                    nit = 0;
                    phase++;
                    if (phase == 4 && a.max_newton <= 0) ev = 2;
                }
            } else if (sing) {
                ev = 2;
            } else {
                xe = {xe.re + d.re, xe.im + d.im};
                const double nx = sqrt(group_sum<G>(abs2(xe)));
                const double nd = sqrt((double)nd2);
                nit++;
                nits++;
                if (nit == 1 && !(nd <= pred_tol * (1.0 + nx)))
                    ev = 2;
                else if (nd <= tau * (1.0 + nx))
                    ev = 1;
                else if (nit >= a.max_newton)
                    ev = 2;
            }
            bool next_step = false;
            if (ev == 1) {
                x = xe;
                t = tn;
                steps++;
                lsteps++;
                if (++succ >= a.n_inc) {
                    h = fmin(h * a.beta_inc, a.h_max);
                    succ = 0;
                }
                const double m2 = abs2(x);
                if (group_any<G>(!(m2 <= a.inf2), base)) {
                    ev = 3;
                    fst = group_any<G>(isnan(m2), base) ? HC_T_NONFINITE : HC_T_AT_INFINITY;
                } else if (t >= a.t_final) {
                    save(a.t_final >= 1.0 ? kReached : kRunning);
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
                    fst = HC_T_MIN_STEP;
                } else {
                    next_step = true;
                }
            }
            if (next_step) {
                if (a.launch_steps > 0 && lsteps >= a.launch_steps) {
                    if (r == 0) atomicAdd(a.n_suspended, 1u);
                    save(kRunning);
                } else if (steps + rejects >= a.max_steps) {
                    ev = 3;
                    fst = HC_T_MAX_STEPS;
                } else {
                    begin_step();
                }
            }
            if (ev == 3) fail(fst);
        }
        refill();
    }
}

// LDS for the tables of the 4 wavefronts of a block: 8 x 45 complex FP64 each.
constexpr int kTabLds = 4 * 8 * 45 * 16;

// One work item per wavefront, items in block order (XCD-aware).
template <int N, int G, typename R, bool PARAM>
__global__ __launch_bounds__(256, PARAM ? 1 : 2) void k_track_grp(const TrackArgs a)
{
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int item = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * wpb + wib);
    if (item >= a.n_items) return;
    const int inst = item / a.items_per_inst;
    const int tb = (item - inst * a.items_per_inst) * a.tracks_per_item;
    const int tend = min(tb + a.tracks_per_item, a.n_start);
    __shared__ __align__(16) unsigned char tab[kTabLds];
    run_item<N, G, R, PARAM>(a, inst, tb, tend, reinterpret_cast<cx<R> *>(tab) + wib * 8 * 45);
}

// Persistent tracker over a device work queue: each wavefront pops work items
// (job, instance, path range) with one atomic until the queue is empty and runs
// them with the code for the item's n.  Jobs may differ in n, kind-matching
// PARAM, path count and instance count.  Every wavefront leaves once the queue
// head passes n_items, so the grid always drains.
template <typename R, bool PARAM>
__global__ __launch_bounds__(256, PARAM ? 1 : 2) void k_track_queue(const TrackArgs *__restrict__ jobs,
                                                     const QueueItem *__restrict__ items, int n_items,
                                                     unsigned *head)
{
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ __align__(16) unsigned char tab[kTabLds];
    cx<R> *lds = reinterpret_cast<cx<R> *>(tab) + wib * 8 * 45;
    for (;;) {
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(head, 1u);
        const int idx = (int)__builtin_amdgcn_readfirstlane(got);
        if (idx >= n_items) break;
        const QueueItem it = items[idx];
        const TrackArgs a = jobs[it.job];
        switch (a.n) {
        case 2: run_item<2, 4, R, PARAM>(a, it.inst, it.tb, it.tend, lds); break;
        case 3: run_item<3, 4, R, PARAM>(a, it.inst, it.tb, it.tend, lds); break;
        case 4: run_item<4, 4, R, PARAM>(a, it.inst, it.tb, it.tend, lds); break;
        case 5: run_item<5, 8, R, PARAM>(a, it.inst, it.tb, it.tend, lds); break;
        case 6: run_item<6, 8, R, PARAM>(a, it.inst, it.tb, it.tend, lds); break;
        case 7: run_item<7, 8, R, PARAM>(a, it.inst, it.tb, it.tend, lds); break;
        case 8: run_item<8, 8, R, PARAM>(a, it.inst, it.tb, it.tend, lds); break;
        default: break;
        }
    }
}

hipError_t launch_track_queue(bool fp32, bool param, const TrackArgs *jobs, const QueueItem *items, int n_items,
                              unsigned *head, int n_waves, hipStream_t st)
{
    if (n_items == 0) return hipSuccess;
    const dim3 grid((n_waves + 3) / 4), block(256);
    if (param) {
        if (fp32) hipLaunchKernelGGL((k_track_queue<float, true>), grid, block, 0, st, jobs, items, n_items, head);
        else hipLaunchKernelGGL((k_track_queue<double, true>), grid, block, 0, st, jobs, items, n_items, head);
    } else {
        if (fp32) hipLaunchKernelGGL((k_track_queue<float, false>), grid, block, 0, st, jobs, items, n_items, head);
        else hipLaunchKernelGGL((k_track_queue<double, false>), grid, block, 0, st, jobs, items, n_items, head);
    }
    return hipGetLastError();
}

// Resident wavefronts of the persistent tracker on this device (all CUs).
int queue_waves(bool fp32, bool param)
{
    int dev = 0, cus = 0, blocks = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    if (param)
        e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_track_queue<float, true>, 256, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_track_queue<double, true>, 256, 0);
    else
        e = fp32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_track_queue<float, false>, 256, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_track_queue<double, false>, 256, 0);
    if (e != hipSuccess || blocks < 1) blocks = 1;
    return cus * blocks * 4;
}

template <int N, int G>
static hipError_t launch_grp(bool fp32, const TrackArgs &a, int wpb, hipStream_t st)
{
    const int blocks = (a.n_items + wpb - 1) / wpb;
    const dim3 grid(blocks), block(64 * wpb);
    if (a.coef0) {
        if (fp32) hipLaunchKernelGGL((k_track_grp<N, G, float, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_track_grp<N, G, double, true>), grid, block, 0, st, a);
    } else {
        if (fp32) hipLaunchKernelGGL((k_track_grp<N, G, float, false>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_track_grp<N, G, double, false>), grid, block, 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_track_group(int n, bool fp32, const TrackArgs &a, int wpb, hipStream_t st)
{
    if (a.n_items == 0) return hipSuccess;
    switch (n) {
    case 2: return launch_grp<2, 4>(fp32, a, wpb, st);
    case 3: return launch_grp<3, 4>(fp32, a, wpb, st);
    case 4: return launch_grp<4, 4>(fp32, a, wpb, st);
    case 5: return launch_grp<5, 8>(fp32, a, wpb, st);
    case 6: return launch_grp<6, 8>(fp32, a, wpb, st);
    case 7: return launch_grp<7, 8>(fp32, a, wpb, st);
    case 8: return launch_grp<8, 8>(fp32, a, wpb, st);
    default: return hipErrorInvalidValue;
    }
}

int group_lanes(int n) { return n <= 4 ? 4 : 8; }

}  // namespace hcx

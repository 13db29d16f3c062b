// hc_group.h -- device code of the path trackers with G lanes per path, one row per lane.
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
#pragma once

#include <algorithm>
#include <atomic>
#include <type_traits>
#include <utility>

#include "hc_device.h"

namespace hcx {

namespace {

__device__ __forceinline__ unsigned umax(unsigned a, unsigned b) { return a > b ? a : b; }

// ds_swizzle bit-mode pattern that exchanges lanes i and i ^ 16 inside each
// 32-lane half (and-mask 0x1F, or-mask 0, xor-mask 0x10): the step of the group
// reductions that crosses the two rows of a 32-lane group.
constexpr int kSwzXor16 = 0x1F | (0x10 << 10);

template <int G>
__device__ __forceinline__ unsigned group_max(unsigned v)
{
    // xor 1 and xor 2 inside quads (quad_perm), then mirror across the half row
    // (lane i <-> 7-i) and the row (lane i <-> 15-i): every lane ends with the max
    v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    if (G >= 8) v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    if (G >= 16) v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    if (G >= 32) v = umax(v, (unsigned)__builtin_amdgcn_ds_swizzle((int)v, kSwzXor16));
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

template <typename R>
__device__ __forceinline__ void stl(lds_tab<R> p, int i, cx<R> v)
{
    p[i].re = v.re;
    p[i].im = v.im;
}

// Coefficient q of the lane's equation, from an LDS slot (coefficient-major,
// stride n; p already offset by the equation) ...
template <int N, typename R>
struct LdsRow {
    lds_tab<R> p;
    __device__ __forceinline__ cx<R> operator()(int q) const { return ldl(p, q * N); }
};

// ... or from the equation's row of a table in global memory ([eq][term][2]).
template <typename R>
struct GlobalRow {
    const R *p;
    __device__ __forceinline__ cx<R> operator()(int q) const { return {p[2 * q], p[2 * q + 1]}; }
};

// Row r of [H_x | rhs] at (x, t) for H = (1-t) gamma G + t F (see build_td in
// hc_kernels.hip for the formulas): the lane's own equation, its terms read
// through `cf` (term q of equation r is cf(q); padding lanes read a real row and
// their results are ignored).
template <int N, typename R, typename Tab>
__device__ __forceinline__ void build_row(const Tab &cf, int r, bool d2, cx<R> gam, const cx<R> (&x)[N], R t,
                                          bool pred, cx<R> (&row)[N + 1])
{
    cx<R> Lx = {R(0), R(0)};
#pragma unroll
    for (int j = 0; j < N; j++) {
        const cx<R> L = cf(1 + j);
        row[j] = L;
        Lx = cfma(L, x[j], Lx);
    }
    int q = 1 + N;
#pragma unroll
    for (int a = 0; a < N; a++) {
#pragma unroll
        for (int b = a; b < N; b++) {
            const cx<R> cq = cf(q++);
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
    const cx<R> c0 = cf(0);
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
template <int N, typename R, typename Tab>
__device__ __forceinline__ cx<double> resid_td64(const Tab &cf, int r, bool d2, cx<double> gam,
                                                 const cx<double> (&x)[N], double t)
{
    const cx<R> c0r = cf(0);
    cx<double> F = {(double)c0r.re, (double)c0r.im};
    int q = 1 + N;
#pragma unroll
    for (int a = 0; a < N; a++) {
        const cx<R> L = cf(1 + a);
        cx<double> y = {(double)L.re, (double)L.im};
#pragma unroll
        for (int b = a; b < N; b++) {
            const cx<R> cq = cf(q++);
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

__device__ __forceinline__ double swz_xor16(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffffll), kSwzXor16);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), kSwzXor16);
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
    if (G >= 32) v = v + swz_xor16(v);
    return v;
}

// NaN-propagating maximum over the G lanes of a group (butterflies as in
// group_sum), identical in every lane.
__device__ __forceinline__ double dmax_pick(double v, double o) { return (o > v || isnan(o)) ? o : v; }

template <int G>
__device__ __forceinline__ double group_max_d(double v)
{
    v = dmax_pick(v, dpp<0xB1>(v));
    v = dmax_pick(v, dpp<0x4E>(v));
    if (G >= 8) v = dmax_pick(v, dpp<0x141>(v));
    if (G >= 16) v = dmax_pick(v, dpp<0x140>(v));
    if (G >= 32) v = dmax_pick(v, swz_xor16(v));
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
// group).  Must run with the whole wavefront active, in a block of 4
// wavefronts.  Returns true if a pivot is (numerically) zero.
//
// nrt <= N is the system's size, the same in every group of the wavefront:
// rows r >= nrt never become pivotal and the elimination stops after nrt
// positions.  Entries of rows r < nrt in columns nrt..N-1 must be zero, so the
// result is that of the nrt x nrt system.
//
// The pivot row's remaining entries reach the group through LDS: the pivot lane
// stores them in the group's slot and every lane of the group reads them back
// (one address per group: broadcast reads), about a quarter of the LDS
// instructions of one ds_bpermute per dword.
template <int N, int G, typename R>
__device__ __forceinline__ bool group_solve(cx<R> (&row)[N + 1], int r, int base, cx<R> &dxr, R &nd, int nrt = N)
{
    constexpr unsigned GM = G - 1;
    __shared__ cx<R> pivbuf[4 * (64 / G) * (N + 1)];
    const lds_tab<R> piv =
        (lds_tab<R>)(pivbuf + ((int)(threadIdx.x >> 6) * (64 / G) + base / G) * (N + 1));
    int pos = r < nrt ? -1 : 4 * G;  // position at which this row became pivotal
    int pl[N];                       // group-relative lane of the pivot of each position
    cx<R> inv_own = {R(0), R(0)};
    bool sing = false;
#pragma unroll
    for (int k = 0; k < N; k++) {
        pl[k] = 0;
        if (k < nrt) {
            const float v = (float)abs1(row[k]);
            const unsigned key = pos < 0 ? (0x80000000u | (__float_as_uint(v) & ~GM) | (GM - (unsigned)r)) : 0u;
            const unsigned kmax = group_max<G>(key);
            const int p = (int)(GM - (kmax & GM));
            sing |= ((kmax & 0x7fffffffu & ~GM) == 0u);
            pl[k] = p;
            if (r == p) {
#pragma unroll
                for (int c = k; c <= N; c++) stl(piv, c, row[c]);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const cx<R> inv = crecip(ldl(piv, k));
            const bool is_piv = (r == p);
            pos = is_piv ? k : pos;
            inv_own = csel(is_piv, inv, inv_own);
            cx<R> l = cmul(row[k], inv);
            l = csel(pos < 0, l, cx<R>{R(0), R(0)});
            if constexpr ((N + 1) * sizeof(cx<R>) <= 256) {
                // short rows: the whole pivot row in registers at once
                cx<R> P[N + 1];
#pragma unroll
                for (int c = k + 1; c <= N; c++) P[c] = ldl(piv, c);
#pragma unroll
                for (int c = k + 1; c <= N; c++) row[c] = cfms(l, P[c], row[c]);
            } else {
                // long rows (FP64, N >= 16): the pivot row streams through in
                // chunks of 4 entries, so it never sits in registers beside the
                // whole own row (the compiler barrier keeps the loads from all
                // being hoisted ahead)
#pragma unroll
                for (int c0 = k + 1; c0 <= N; c0 += 4) {
                    cx<R> P[4];
#pragma unroll
                    for (int c = c0; c < c0 + 4 && c <= N; c++) P[c - c0] = ldl(piv, c);
#pragma unroll
                    for (int c = c0; c < c0 + 4 && c <= N; c++) row[c] = cfms(l, P[c - c0], row[c]);
                    asm volatile("" ::: "memory");
                }
            }
        }
    }
    cx<R> b = row[N];
    dxr = {R(0), R(0)};
    nd = R(0);
#pragma unroll
    for (int k = N - 1; k >= 0; k--) {
        if (k < nrt) {
            const cx<R> xk = bcast(cmul(b, inv_own), base + pl[k]);
            dxr = csel(r == k, xk, dxr);
            nd = fma(xk.re, xk.re, fma(xk.im, xk.im, nd));
            const bool above = pos < k;
            b = csel(above, cfms(row[k], xk, b), b);
        }
    }
    return sing;
}

}  // namespace

// Number of instance tables a wavefront keeps in LDS: groups still on an older
// work item's paths keep its table while idle groups start on a newer item.
constexpr int kSlots = 3;

// Work items of one launch of k_track_grp: item i is paths
// [(i mod per_inst) tpi, +tpi) of instance i / per_inst, popped in order from a
// device counter, so wavefronts that finish early take more.
struct GridSource {
    unsigned *head;
    int n_items, per_inst, tpi, n_start;
    bool done;

    __device__ __forceinline__ bool pop(int &inst, int &tb, int &tend)
    {
        if (done) return false;
        unsigned got = 0;
        if ((threadIdx.x & 63) == 0) got = atomicAdd(head, 1u);
        const int idx = (int)__builtin_amdgcn_readfirstlane(got);
        if (idx >= n_items) {
            done = true;
            return false;
        }
        inst = idx / per_inst;
        tb = (idx - inst * per_inst) * tpi;
        tend = min(tb + tpi, n_start);
        return true;
    }
};

// Work items of the persistent batch tracker for one job: the item that started
// the run, then queue items as long as they belong to the same job.  An item of
// another job ends the run and is handed back in `pending`.
struct QueueSource {
    const QueueItem *items;
    unsigned *head;
    int n_items, job;
    bool has_first, has_pending, done;
    QueueItem first, pending;

    __device__ __forceinline__ bool pop(int &inst, int &tb, int &tend)
    {
        if (has_first) {
            has_first = false;
            inst = first.inst;
            tb = first.tb;
            tend = first.tend;
            return true;
        }
        if (has_pending || done) return false;
        unsigned got = 0;
        if ((threadIdx.x & 63) == 0) got = atomicAdd(head, 1u);
        const int idx = (int)__builtin_amdgcn_readfirstlane(got);
        if (idx >= n_items) {
            done = true;
            return false;
        }
        const QueueItem it = items[idx];
        if (it.job != job) {
            pending = it;
            has_pending = true;
            return false;
        }
        inst = it.inst;
        tb = it.tb;
        tend = it.tend;
        return true;
    }
};

// Copies instance `inst`'s kernel table into an LDS slot, coefficient-major
// (term q of equation r at dst[q * N + r]).  Whole wavefront, uniform arguments.
template <int N, typename R>
__device__ __forceinline__ void stage_table(const TrackArgs &a, int inst, cx<R> *dst)
{
    constexpr int T = dense_terms(N);
    const R *ce = static_cast<const R *>(a.coef) + (size_t)inst * N * T * 2;
    for (int e = (int)(threadIdx.x & 63); e < N * T; e += 64) {
        const int eq = e / T, q = e - eq * T;
        dst[q * N + eq] = {ce[2 * e], ce[2 * e + 1]};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// One stage (evaluate + solve) of every group of the wavefront in precision R:
// gathers the group's stage point, builds the lane's row of [H_x | rhs] (table
// row cf, or the parameter rows p0/p1) and solves.  Returns the zero-pivot
// flag; d = component r of the solution, nd = its squared norm over the group.
// Must run with the whole wavefront active.
template <int N, int G, typename R, bool PARAM, typename Tab>
__device__ __forceinline__ bool stage_solve(const Tab &cf, const R *p0, const R *p1, int r, int base, bool d2,
                                            cx<R> gam, cx<double> gam64, cx<double> xe, double te, bool pred,
                                            bool ir, cx<double> &d, double &nd)
{
    cx<R> xs[N];
    cx<double> xa[N];
    if (sizeof(R) == 8 || ir) {
        gather<G, N>(xe, xa);
#pragma unroll
        for (int j = 0; j < N; j++) xs[j] = {R(xa[j].re), R(xa[j].im)};
    } else {
        gather<G, N>(cx<R>{R(xe.re), R(xe.im)}, xs);
    }
    cx<R> row[N + 1];
    if constexpr (PARAM) {
        build_row_param<N, R>(p0, p1, xs, R(te), pred, row);
        if (ir && !pred) {
            const cx<double> H = resid_param64<N, R>(p0, p1, xa, te);
            row[N] = {R(-H.re), R(-H.im)};
        }
    } else {
        build_row<N, R>(cf, r, d2, gam, xs, R(te), pred, row);
        if (ir && !pred) {
            const cx<double> H = resid_td64<N, R>(cf, r, d2, gam64, xa, te);
            row[N] = {R(-H.re), R(-H.im)};
        }
    }
    cx<R> dxr;
    R nd2;
    const bool sing = group_solve<N, G, R>(row, r, base, dxr, nd2);
    d = {(double)dxr.re, (double)dxr.im};
    nd = (double)nd2;
    return sing;
}

// Result of one stage: component r of the solution, the group's squared norm of
// it and the zero-pivot flag.
struct StageOut {
    cx<double> d;
    double nd;
    bool sing;
};

// The FP64 stage of the mixed-precision tracker as a function of its own (not
// inlined): its registers are saved and restored around the call, which runs
// only while a group of the wavefront tracks in FP64, so the FP32 loop keeps
// its own register allocation.
template <int N, int G, bool PARAM>
__device__ __attribute__((noinline)) StageOut stage64_dense(const double *q0, const double *q1, int r, int base,
                                                             bool d2, cx<double> gam64, cx<double> xe, double te,
                                                             bool pred)
{
    StageOut o;
    o.sing = stage_solve<N, G, double, PARAM>(GlobalRow<double>{q1}, q0, q1, r, base, d2, gam64, gam64, xe, te, pred,
                                              false, o.d, o.nd);
    return o;
}

// ---------------------------------------------------------------- term lists
// Layout for sparse systems (section 6: a term table per equation).  Equation r
// has T slots; slot k holds one term c_k m_k(x).  Three kernel kinds:
//   * quadratic (kTermsQ16): degree <= 2, n <= 16; the slot's variables are
//     packed as a | b << 8 in 16 bits (0xFF: no factor, so 0xFFFF is a constant
//     and an unused slot is 0xFFFF with c_k = 0);
//   * quadratic with a 10- or 14-row solver (kTermsQ10: degree <= 2, n <= 10;
//     kTermsQ14: n <= 14), the same slots as kTermsQ16;
//   * general degree (kTermsG16: n <= 16; kTermsG18: n <= 18; kTermsG20: n <= 20; kTermsG32:
//     n <= 32, every system above 20 unknowns whatever its degree): the monomial's
//     factors, with repetition, in the bytes of a 64-bit word, lowest byte first
//     (0xFF: no factor, so at most 8 factors), plus a per-slot degree that is the
//     largest over the equations (equations keep their terms in decreasing
//     degree, so that maximum is tight), on which the kernels branch uniformly.
// Kernels run with NM rows per group of G lanes: lanes r >= n carry the
// identity row e_r with a zero right-hand side and never pivot (lanes r >= NM,
// where NM < G, a zero row).  The solver's row count NM bounds every
// elimination row's length, so a system runs on the kind with the smallest NM
// that holds it.
enum TermKind {
    kTermsQ16 = 0, kTermsG16 = 1, kTermsG20 = 2, kTermsQ14 = 3, kTermsG18 = 4, kTermsQ10 = 5, kTermsG32 = 6,
    kTermKinds = 7
};

template <int TK>
struct TermCfg {
    static constexpr int NM = TK == kTermsG32   ? 32  // rows of the group solver
                              : TK == kTermsG20 ? 20
                              : TK == kTermsG18 ? 18
                              : TK == kTermsQ14 ? 14
                              : TK == kTermsQ10 ? 10
                                                : 16;
    static constexpr int G = (TK == kTermsG20 || TK == kTermsG18 || TK == kTermsG32) ? 32 : 16;  // lanes per path
    static constexpr bool GEN = TK != kTermsQ16 && TK != kTermsQ14 && TK != kTermsQ10;  // general-degree slots
    // mixed precision: FP64 stages inside the FP32 launch, else a second launch
    static constexpr bool INLINE_ESC = term_kind_inline_esc(TK);
    // wavefronts per SIMD the tracker is compiled for: 3 where the LDS slices
    // allow it and the spills at 168 VGPRs cost less than the latency a third
    // wavefront hides -- every FP32 kernel without the inline FP64 stage; the
    // FP64 kernels of q10 and g18 (14-19% faster on the 3-view batch, 6-8% on
    // the trifocal batch); q14, q16, g16 and g20 hold more than 160 KB of FP64
    // LDS slices per CU at 3 blocks.  g32's FP64 slices take 136 KB per block
    // of 4 wavefronts, so one block per CU (its 33-entry FP64 rows get the
    // whole register file of the SIMD); its FP32 slices allow two.
    template <typename R>
    static constexpr int waves()
    {
        if (TK == kTermsG32) return sizeof(R) == 4 ? 2 : 1;
        return (sizeof(R) == 4 && !INLINE_ESC) || TK == kTermsQ10 || TK == kTermsG18 ? 3 : 2;
    }
    // the batch tracker (a device queue of jobs) escalates inline on every kind:
    // its small, latency-bound batches lose more to a second launch than they
    // gain from a third wavefront (serving mix: p50 34 -> 44 ms with two)
    static constexpr int QUEUE_WAVES = TK == kTermsG32 ? 1 : TK == kTermsQ10 || TK == kTermsG18 ? 3 : 2;
    static constexpr int MAXD = GEN ? 8 : 2;                                    // factors per slot
};

constexpr int kTermsN = 16;

// LDS of one wavefront for a term-list kind: the groups' stage points (one
// component per lane) and the owned rows' accumulators (NM rows of NM entries,
// stride NM + 1 against bank conflicts), room for FP64.
template <int NM, int G>
constexpr int terms_lds_cx() { return 64 + (64 / G) * NM * (NM + 1); }

// Row accumulator of lane r (r < NM) of the group at lane `base`.
template <int NM, int G, typename R>
__device__ __forceinline__ lds_tab<R> terms_row_acc(lds_tab<R> xs, int base, int r)
{
    return xs + 64 + ((base / G) * NM + r) * (NM + 1);
}

// Term c x_{f_0} ... x_{f_{D-1}} of a general-degree slot (factor i in byte i of
// v, in increasing order with repetition; 0xFF: none, value 1).  Adds cr m(x)
// to F and, for each factor f_i, ct dm/dx_{f_i} to the row accumulator rb: the
// derivative of the product along factor i is the product of the other
// factors, taken as prefix (factors before i) times suffix (factors after i)
// products.  The term's accumulator entries are read together and written
// together (one LDS round trip per term, not one per factor); a repeated
// variable's contributions are summed into the last factor of its run, the
// only one written.
//
// PADL (kinds with NM < G): lane NM of the group holds 1 at xg[NM] and entry
// NM of the row accumulator is padding, so a missing factor reads and writes
// index NM instead of being selected around.
template <int D, int NM, typename R, bool PADL>
__device__ __forceinline__ void term_general(unsigned long long v, cx<R> cr, cx<R> ct, lds_tab<R> xg, lds_tab<R> rb,
                                             cx<R> &F)
{
    const cx<R> one = {R(1), R(0)}, zero = {R(0), R(0)};
    int f[D];
    cx<R> xv[D], acc[D];
#pragma unroll
    for (int i = 0; i < D; i++) {
        f[i] = (int)((v >> (8 * i)) & 0xFFull);
        if constexpr (PADL) {
            f[i] = min(f[i], NM);
            xv[i] = ldl(xg, f[i]);
            acc[i] = ldl(rb, f[i]);
        } else {
            xv[i] = f[i] < NM ? ldl(xg, f[i]) : one;
            acc[i] = f[i] < NM ? ldl(rb, f[i]) : zero;
        }
    }
    cx<R> P[D];  // P[i] = x_{f_0} ... x_{f_{i-1}}
    P[0] = one;
#pragma unroll
    for (int i = 1; i < D; i++) P[i] = i == 1 ? xv[0] : cmul(P[i - 1], xv[i - 1]);
    F = cfma(cr, D == 1 ? xv[0] : cmul(P[D - 1], xv[D - 1]), F);
    cx<R> dm[D];
    cx<R> S = one;  // x_{f_{i+1}} ... x_{f_{D-1}}
#pragma unroll
    for (int i = D - 1; i >= 0; i--) {
        dm[i] = i == 0 ? S : (i == D - 1 ? P[i] : cmul(P[i], S));
        if (i > 0) S = i == D - 1 ? xv[i] : cmul(S, xv[i]);
    }
    cx<R> run = zero;  // contributions of the current run of equal factors
#pragma unroll
    for (int i = 0; i < D; i++) {
        run = cfma(ct, dm[i], run);
        const bool last = i == D - 1 || f[i + 1] != f[i];
        if ((PADL || f[i] < NM) && last) stl(rb, f[i], cx<R>{acc[i].re + run.re, acc[i].im + run.im});
        if (last) run = zero;
    }
}

// Coefficient of a slot at t (ct, for the Jacobian and H) and on the right-hand
// side (cr), from its target value c (c1) and start value s (c0): c for total
// degree; (1-t) s + t c, and c - s for H_t in a predictor stage, for a
// parameter homotopy.
template <typename R, bool PARAM>
__device__ __forceinline__ void slot_coefs(cx<R> c, cx<R> s, R t, R omt, bool pred, cx<R> &ct, cx<R> &cr)
{
    ct = c;
    cr = c;
    if constexpr (PARAM) {
        ct = {fma(t, c.re, omt * s.re), fma(t, c.im, omt * s.im)};
        cr = pred ? cx<R>{c.re - s.re, c.im - s.im} : ct;
    }
}

// Row r of [H_x | rhs] from the lane's term list (vars, c1 and, for a parameter
// homotopy, c0: the equation's T slots), at the point held in xg (component j
// at xg[j]); rb is the lane's row accumulator.  Total degree: H = (1-t) gam G +
// t F with G_r = x_r^dg - 1 (dg: the degree of equation r); parameter: H =
// F(x; (1-t) c0 + t c1), H_t = F(x; c1 - c0).  The right-hand side is -H_t for
// a predictor stage, -H else.
template <int TK, typename R, bool PARAM>
__device__ __forceinline__ void build_row_terms(const void *vars, const int *sdeg, int T, const R *c1, const R *c0,
                                                lds_tab<R> xg, lds_tab<R> rb, int r, bool own, int dg,
                                                cx<R> gam, cx<R> xr, R t, bool pred,
                                                cx<R> (&row)[TermCfg<TK>::NM + 1])
{
    constexpr int NM = TermCfg<TK>::NM;
    const cx<R> zero = {R(0), R(0)}, one = {R(1), R(0)};
    if (own) {
#pragma unroll
        for (int j = 0; j < NM; j++) stl(rb, j, zero);
    }
    const R omt = R(1) - t;
    cx<R> F = zero;
    if constexpr (!TermCfg<TK>::GEN) {
        // q10, q14 (NM < G): lane NM of the group publishes 1 at xg[NM], and
        // entry NM of every row accumulator is padding, so a missing factor
        // (0xFF) reads index NM and the slot needs no branch; q16 selects around
        // a missing factor.  A squared variable's two contributions go through
        // the second write.  FP32: the next slot's variables and coefficients
        // are loaded while this one is evaluated; FP64 loads them at the top of
        // the slot (the prefetched FP64 values cost spills at 3 wavefronts per
        // SIMD and measured ~1% slower).
        constexpr bool PADQ = NM < TermCfg<TK>::G;
        constexpr bool PREF = sizeof(R) == 4;
        using gptr = const __attribute__((address_space(1))) R *;
        const gptr g1 = (gptr)c1, g0 = (gptr)c0;
        const unsigned short *vr = static_cast<const unsigned short *>(vars);
        const int cnt = own ? T : 0;
        unsigned vn = 0xFFFFu;
        cx<R> c1n = zero, c0n = zero;
        if constexpr (PREF) {
            vn = cnt > 0 ? vr[0] : 0xFFFFu;
            c1n = cnt > 0 ? cx<R>{g1[0], g1[1]} : zero;
            if constexpr (PARAM) c0n = cnt > 0 ? cx<R>{g0[0], g0[1]} : zero;
        }
        for (int k = 0; k < cnt; k++) {
            if constexpr (!PREF) {
                vn = vr[k];
                c1n = {g1[2 * k], g1[2 * k + 1]};
                if constexpr (PARAM) c0n = {g0[2 * k], g0[2 * k + 1]};
            }
            const unsigned v = vn;
            const cx<R> c = c1n, s0 = c0n;
            if (PREF && k + 1 < cnt) {
                vn = vr[k + 1];
                c1n = {g1[2 * k + 2], g1[2 * k + 3]};
                if constexpr (PARAM) c0n = {g0[2 * k + 2], g0[2 * k + 3]};
            }
            int ia = (int)(v & 0xFFu), ib = (int)(v >> 8);
            if constexpr (PADQ) {
                ia = min(ia, NM);
                ib = min(ib, NM);
            }
            cx<R> ct, cr;
            slot_coefs<R, PARAM>(c, s0, t, omt, pred, ct, cr);
            cx<R> xa, xb, ra, rbb;
            if constexpr (PADQ) {
                xa = ldl(xg, ia);
                xb = ldl(xg, ib);
                ra = ldl(rb, ia);
                rbb = ldl(rb, ib);
            } else {
                xa = ia < NM ? ldl(xg, ia) : one;
                xb = ib < NM ? ldl(xg, ib) : one;
                ra = ia < NM ? ldl(rb, ia) : zero;
                rbb = ib < NM ? ldl(rb, ib) : zero;
            }
            F = cfma(cr, cmul(xa, xb), F);
            // x_a^2 (ia == ib): the second write carries both contributions
            const cx<R> na = cfma(ct, xb, ra);
            const cx<R> nb = cfma(ct, xa, ia == ib ? na : rbb);
            if (PADQ || ia < NM) stl(rb, ia, na);
            if (PADQ || ib < NM) stl(rb, ib, nb);
        }
    } else if (own) {
        // FP32: the next slot's variables and coefficients are loaded while this
        // one is evaluated (FP64 loads them at the top of the slot, as above)
        constexpr bool PADL = NM < TermCfg<TK>::G;
        using gptr = const __attribute__((address_space(1))) R *;
        const gptr g1 = (gptr)c1, g0 = (gptr)c0;
        const unsigned long long *vr = static_cast<const unsigned long long *>(vars);
        constexpr bool PREF = sizeof(R) == 4;
        unsigned long long vn = ~0ull;
        cx<R> c1n = zero, c0n = zero;
        if constexpr (PREF) {
            vn = T > 0 ? vr[0] : ~0ull;
            c1n = T > 0 ? cx<R>{g1[0], g1[1]} : zero;
            if constexpr (PARAM) c0n = T > 0 ? cx<R>{g0[0], g0[1]} : zero;
        }
        for (int k = 0; k < T; k++) {
            const int m = __builtin_amdgcn_readfirstlane(sdeg[k]);  // same slot in every lane
            if constexpr (!PREF) {
                vn = vr[k];
                c1n = {g1[2 * k], g1[2 * k + 1]};
                if constexpr (PARAM) c0n = {g0[2 * k], g0[2 * k + 1]};
            }
            const unsigned long long v = vn;
            const cx<R> c = c1n, s0 = c0n;
            if (PREF && k + 1 < T) {
                vn = vr[k + 1];
                c1n = {g1[2 * k + 2], g1[2 * k + 3]};
                if constexpr (PARAM) c0n = {g0[2 * k + 2], g0[2 * k + 3]};
            }
            cx<R> ct, cr;
            slot_coefs<R, PARAM>(c, s0, t, omt, pred, ct, cr);
            switch (m) {
            case 0: F = cfma(cr, one, F); break;
            case 1: term_general<1, NM, R, PADL>(v, cr, ct, xg, rb, F); break;
            case 2: term_general<2, NM, R, PADL>(v, cr, ct, xg, rb, F); break;
            case 3: term_general<3, NM, R, PADL>(v, cr, ct, xg, rb, F); break;
            case 4: term_general<4, NM, R, PADL>(v, cr, ct, xg, rb, F); break;
            case 5: term_general<5, NM, R, PADL>(v, cr, ct, xg, rb, F); break;
            case 6: term_general<6, NM, R, PADL>(v, cr, ct, xg, rb, F); break;
            case 7: term_general<7, NM, R, PADL>(v, cr, ct, xg, rb, F); break;
            default: term_general<8, NM, R, PADL>(v, cr, ct, xg, rb, F); break;
            }
        }
    }
    if (own) {
#pragma unroll
        for (int j = 0; j < NM; j++) row[j] = ldl(rb, j);
    }
    if constexpr (PARAM) {
        row[NM] = {-F.re, -F.im};
    } else {
        cx<R> p = one;  // x_r^(dg-1)
        for (int e = 1; e < dg; e++) p = cmul(p, xr);
        cx<R> Gv = cmul(p, xr);
        Gv.re -= R(1);
        const cx<R> dG = {R(dg) * p.re, R(dg) * p.im};
        const cx<R> gG = cmul(gam, Gv);
        const cx<R> gdG = cmul(gam, dG);
#pragma unroll
        for (int j = 0; j < NM; j++) {
            row[j] = cscale(t, row[j]);
            row[j].re += (j == r) ? omt * gdG.re : R(0);
            row[j].im += (j == r) ? omt * gdG.im : R(0);
        }
        const cx<R> Ht = {F.re - gG.re, F.im - gG.im};
        const cx<R> H = {fma(t, F.re, omt * gG.re), fma(t, F.im, omt * gG.im)};
        row[NM] = pred ? cx<R>{-Ht.re, -Ht.im} : cx<R>{-H.re, -H.im};
    }
    if (!own) {
#pragma unroll
        for (int j = 0; j <= NM; j++) row[j] = (j == r) ? one : zero;
    }
}

// H_r(x, t) of the lane's equation in FP64 from the FP64 tables (q1, q0) at
// the point held in xg (FP64, component j at xg[j]): the right-hand side of an
// FP32 Newton stage with the fp64_residual option (iterative refinement).
template <int TK, bool PARAM>
__device__ __forceinline__ cx<double> resid_terms64(const void *vars, int T, const double *q1, const double *q0,
                                                    lds_tab<double> xg, int dg, cx<double> gam, cx<double> xr,
                                                    double t)
{
    constexpr int NM = TermCfg<TK>::NM;
    const cx<double> one = {1.0, 0.0};
    const double omt = 1.0 - t;
    cx<double> F = {0.0, 0.0};
    for (int k = 0; k < T; k++) {
        cx<double> c = {q1[2 * k], q1[2 * k + 1]};
        if constexpr (PARAM) c = {fma(t, c.re, omt * q0[2 * k]), fma(t, c.im, omt * q0[2 * k + 1])};
        cx<double> m = one;
        if constexpr (TermCfg<TK>::GEN) {
            const unsigned long long v = static_cast<const unsigned long long *>(vars)[k];
            for (int i = 0; i < 8; i++) {
                const int f = (int)((v >> (8 * i)) & 0xFFull);
                if (f >= NM) break;
                m = cmul(m, ldl(xg, f));
            }
        } else {
            const unsigned v = static_cast<const unsigned short *>(vars)[k];
            const int ia = (int)(v & 0xFFu), ib = (int)(v >> 8);
            if (ia < NM) m = ldl(xg, ia);
            if (ib < NM) m = cmul(m, ldl(xg, ib));
        }
        F = cfma(c, m, F);
    }
    if constexpr (PARAM) return F;
    cx<double> p = one;
    for (int e = 0; e < dg; e++) p = cmul(p, xr);
    p.re -= 1.0;
    const cx<double> gG = cmul(gam, p);
    return {fma(t, F.re, omt * gG.re), fma(t, F.im, omt * gG.im)};
}

// One stage of every group in precision R on the term-list layout (see
// stage_solve): the lanes publish their components of the stage point in LDS,
// build their rows and solve the n x n system.  Whole wavefront active.  With
// ir (R = float), a Newton stage's right-hand side is -H evaluated in FP64
// from the FP64 tables q1, q0 at the FP64 stage point, which goes to the upper
// half of the wavefront's LDS slice (the FP32 stage uses the lower half).
template <int TK, typename R, bool PARAM>
__device__ __forceinline__ bool stage_solve_terms(const void *vars, const int *sdeg, int T, const R *p1, const R *p0,
                                                  void *ldsv, int lane, int r, int base, bool own, int n, int dg,
                                                  cx<R> gam, cx<double> xe, double te, bool pred, cx<double> &d,
                                                  double &nd, bool ir = false, const double *q1 = nullptr,
                                                  const double *q0 = nullptr, cx<double> gam64 = {1.0, 0.0})
{
    constexpr int NM = TermCfg<TK>::NM, G = TermCfg<TK>::G;
    const lds_tab<R> xs = (lds_tab<R>)(cx<R> *)ldsv;
    // kinds with NM < G (q10, q14, g18, g20): lane NM of the group holds 1, the
    // value of a missing factor
    const R pad = (NM < G && r == NM) ? R(1) : R(0);
    const cx<R> xo = own ? cx<R>{R(xe.re), R(xe.im)} : cx<R>{pad, R(0)};
    stl(xs, lane, xo);
    const bool use_ir = sizeof(R) == 4 && ir && !pred;
    const lds_tab<double> x64 =
        (lds_tab<double>)(cx<double> *)((char *)ldsv + (size_t)terms_lds_cx<NM, G>() * sizeof(cx<float>));
    if (use_ir) stl(x64, lane, own ? xe : cx<double>{0.0, 0.0});
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    cx<R> row[NM + 1];
    build_row_terms<TK, R, PARAM>(vars, sdeg, T, p1, p0, xs + base, terms_row_acc<NM, G>(xs, base, own ? r : 0), r,
                                  own, dg, gam, xo, R(te), pred, row);
    if (use_ir && own) {
        const cx<double> H = resid_terms64<TK, PARAM>(vars, T, q1, q0, x64 + base, dg, gam64, xe, te);
        row[NM] = {R(-H.re), R(-H.im)};
    }
    cx<R> dxr;
    R nd2;
    const bool sing = group_solve<NM, G, R>(row, r, base, dxr, nd2, n);
    d = {(double)dxr.re, (double)dxr.im};
    nd = (double)nd2;
    return sing;
}

// The term-list FP64 stage of the mixed-precision tracker, not inlined (see
// stage64_dense).
template <int TK, bool PARAM>
__device__ __attribute__((noinline)) StageOut stage64_terms(const void *vars, const int *sdeg, int T,
                                                             const double *q1, const double *q0, void *ldsv, int lane,
                                                             int r, int base, bool own, int n, int dg,
                                                             cx<double> gam64, cx<double> xe, double te, bool pred)
{
    StageOut o;
    o.sing = stage_solve_terms<TK, double, PARAM>(vars, sdeg, T, q1, q0, ldsv, lane, r, base, own, n, dg, gam64, xe,
                                                  te, pred, o.d, o.nd);
    return o;
}

// Tracks the paths of the work items that `src` hands out with the wavefront's
// lane groups until the source is empty and every path has ended or been
// suspended.  Called with the whole wavefront active.  `lds` is this
// wavefront's slice: kSlots tables of N x T complex values of R.  Each group
// takes its next path from the current item; once the item is used up the
// wavefront pops another into a table slot that no running group still reads.
//
// Path state is distributed over the group: lane r < n holds component r of the
// accepted point x, of the stage point xe and of the RK4 accumulator, all in
// FP64; t, h and the counters are replicated and every lane of a group takes the
// same decisions (the group's sums and tests are computed identically in all of
// its lanes).  Each stage gathers the whole stage point into every lane of the
// group (ds_swizzle), builds the lane's row, solves, and each lane updates its
// own component.
//
// R = float is the mixed-precision tracker: a group tracks in FP32 until its
// path fails (step size below h_min, too many steps, non-finite tangent) or
// reaches t_switch, and then goes on with the same path in FP64 (from its last
// accepted point, h reset to h0 after a failure) -- the wavefront runs the FP64
// stage, with tables read from global memory, only while one of its groups
// needs it.
template <int N, int G, typename R, bool PARAM, typename Src, int TK = -1, int ESC = -1, bool KARG = false>
__device__ __forceinline__ void run_items(const TrackArgs &a, Src &src, cx<R> *lds)
{
    // KARG: `a` is the kernel's only argument, so the loop reads the launch
    // constants and state pointers it needs per stage from the kernel-argument
    // segment where it uses them (scalar loads) instead of holding them in
    // scalar registers across the loop, which spilled them to vector lanes
    using kargp = const __attribute__((address_space(4))) TrackArgs *;
    auto kap = []() {
        kargp p = (kargp)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(p));
        return p;
    };
#define HC_ARG(f) (KARG ? kap()->f : a.f)
    constexpr bool TERMS = TK >= 0;
    constexpr int TKc = TERMS ? TK : 0;
    static_assert(G == 4 || G == 8 || G == 16 || G == 32, "group size");
    static_assert(N <= G, "one row per lane");
    static_assert(!TERMS || (N == TermCfg<TKc>::NM && G == TermCfg<TKc>::G), "term-list kind");
    // FP64 stages inside this (FP32) loop: the dense tables and the term-list
    // kinds compiled for it, or as the caller asks (ESC >= 0); else failures
    // stay RUNNING for an FP64 launch
    constexpr bool kInl = kInlineEsc && (ESC >= 0 ? ESC != 0 : (!TERMS || TermCfg<TKc>::INLINE_ESC));
    constexpr bool R64 = sizeof(R) == 8;
    // dense layout: n = N and T = C(N+2, 2) slots per equation; term lists: runtime
    const int nn = TERMS ? a.n : N;
    const int T = TERMS ? a.n_tslots : dense_terms(N);
    constexpr int kSlot = TERMS ? 1 : N * dense_terms(N);  // complex entries per LDS table slot
    const int lane = threadIdx.x & 63;
    const int r = lane & (G - 1);
    const int base = lane - r;
    const bool own = r < nn;      // lane holds a component of the path state
    const int rr = own ? r : 0;   // table row the lane reads (padding lanes: row 0)
    const void *vrow = nullptr;
    if constexpr (TERMS) {
        if constexpr (TermCfg<TKc>::GEN)
            vrow = static_cast<const unsigned long long *>(a.vars) + (size_t)rr * T;
        else
            vrow = static_cast<const unsigned short *>(a.vars) + (size_t)rr * T;
    }
    // mixed precision: FP64 corrector right-hand side around the FP32 solves
    const bool ir = !R64 && a.ir;
    const long long total = a.total;
    const double pred_tol = a.pred_tol;
    const bool d2 = own && ((a.deg2 >> r) & 1u);
    // term lists: degree of the lane's equation (total-degree start system)
    const int dg = !own ? 1 : (TERMS && TermCfg<TKc>::GEN && a.eqdeg) ? a.eqdeg[r] : (d2 ? 2 : 1);

    const lds_tab<R> cl0 = (lds_tab<R>)lds + rr;
    // parameter homotopy: the lane's start rows (FP64 ones for the FP64 stage),
    // per group when every instance has its own start system
    const R *row0 = static_cast<const R *>(a.coef0) + (size_t)rr * T * 2;
    const double *row0_64 = static_cast<const double *>(a.coef0_64) + (size_t)rr * T * 2;

    // the group's path: its instance's gamma, table slot and target rows, and
    // whether it is tracked in FP64
    cx<R> gam = {R(1), R(0)};
    cx<double> gam64 = {1.0, 0.0};
    int gslot = 0;
    const R *row1 = static_cast<const R *>(a.coef);
    const double *row1_64 = static_cast<const double *>(a.coef64);
    bool p64 = R64;
    // the wavefront's current work item
    int cur_inst = 0, cur_slot = 0, next = 0, tend = 0;

    int trk = -1;
    long long g = 0;
    cx<double> x = {0.0, 0.0}, xe = {0.0, 0.0}, acc = {0.0, 0.0};  // component r
    double t = 0.0, h = 0.0, te = 0.0, hu = 0.0, tn = 0.0;
    int phase = 0, nit = 0, succ = 0, steps = 0, rejects = 0, nits = 0, lsteps = 0, escal = 0;
    unsigned lst32 = 0, lst64 = 0;

    auto save = [&](int st) {
        if (own) {
            HC_ARG(s.xr)[r * total + g] = x.re;
            HC_ARG(s.xi)[r * total + g] = x.im;
        }
        if (r == 0) {
            HC_ARG(s.t)[g] = t;
            HC_ARG(s.h)[g] = h;
            HC_ARG(s.succ)[g] = succ;
            HC_ARG(s.steps)[g] = steps;
            HC_ARG(s.rejects)[g] = rejects;
            HC_ARG(s.nits)[g] = nits;
            HC_ARG(s.escal)[g] = escal;
            HC_ARG(s.status)[g] = st;
            if (HC_ARG(stage_count)) {
                if (lst32) atomicAdd(HC_ARG(stage_count), (unsigned long long)lst32);
                if (lst64) atomicAdd(HC_ARG(stage_count) + 1, (unsigned long long)lst64);
            }
        }
        lst32 = lst64 = 0;
        trk = -1;
    };
    auto begin_step = [&]() {
        // an FP32 step ends at t_switch at the latest
        const double tf = p64 ? HC_ARG(t_final) : HC_ARG(t_switch);
        const double rem = tf - t;
        if (h >= rem) {
            hu = rem;
            tn = tf;
        } else {
            hu = h;
            tn = t + h;
        }
        phase = 0;
        xe = x;
        te = t;
    };
    auto fail = [&](int st) {
        if (!R64 && !p64 && st != HC_T_AT_INFINITY) {
            // mixed precision: the path goes on in FP64 from its last accepted point,
            // in this launch or (escalation off) in the FP64 launch that follows
            escal = steps + rejects + 1;
            h = HC_ARG(h0);
            succ = 0;
            if (!kInl) {
                save(kRunning);
                return;
            }
            p64 = true;
            if (steps_used(steps, rejects, escal) >= HC_ARG(max_steps))
                save(HC_T_MAX_STEPS);
            else
                begin_step();
            return;
        }
        save(st);
    };
    auto refill = [&]() {
        for (;;) {
            const unsigned long long need = ballot(trk < 0 && r == 0);
            if (need == 0ull) break;
            if (next >= tend) {
                // item used up: the lowest table slot no running group reads
                int fs = -1;
#pragma unroll
                for (int sl = kSlots - 1; sl >= 0; sl--)
                    if (ballot(trk >= 0 && gslot == sl) == 0ull) fs = sl;
                if (fs < 0) break;
                int ni, nb, ne;
                if (!src.pop(ni, nb, ne)) break;
                if (!PARAM && !TERMS) stage_table<N, R>(a, ni, lds + fs * kSlot);
                cur_inst = ni;
                cur_slot = fs;
                next = nb;
                tend = ne;
                continue;
            }
            const int cand = next + __popcll(need & ((1ull << base) - 1ull));
            next += __popcll(need);
            if (trk < 0 && cand < tend) {
                const long long gg = (long long)cur_inst * a.n_start + cand;
                // still going and not yet at this launch's end time
                if (HC_ARG(s.status)[gg] == kRunning && HC_ARG(s.t)[gg] < HC_ARG(t_final) &&
                    (R64 || kInl || HC_ARG(s.escal)[gg] == 0)) {
                    trk = cand;
                    g = gg;
                    gslot = cur_slot;
                    if (a.gamma) {
                        gam64 = {a.gamma[2 * cur_inst], a.gamma[2 * cur_inst + 1]};
                        gam = {R(gam64.re), R(gam64.im)};
                    }
                    const size_t ro = ((size_t)cur_inst * nn + rr) * T * 2;
                    row1 = static_cast<const R *>(a.coef) + ro;
                    if (!R64) row1_64 = static_cast<const double *>(a.coef64) + ro;
                    if (PARAM && a.coef0_stride) {
                        const size_t ro0 = (size_t)cur_inst * a.coef0_stride + (size_t)rr * T * 2;
                        row0 = static_cast<const R *>(a.coef0) + ro0;
                        if (!R64) row0_64 = static_cast<const double *>(a.coef0_64) + ro0;
                    }
                    x = own ? cx<double>{HC_ARG(s.xr)[r * total + g], HC_ARG(s.xi)[r * total + g]} : cx<double>{0.0, 0.0};
                    t = HC_ARG(s.t)[g];
                    h = HC_ARG(s.h)[g];
                    succ = HC_ARG(s.succ)[g];
                    steps = HC_ARG(s.steps)[g];
                    rejects = HC_ARG(s.rejects)[g];
                    nits = HC_ARG(s.nits)[g];
                    escal = HC_ARG(s.escal)[g];
                    p64 = R64 || (kInl && (escal != 0 || t >= HC_ARG(t_switch)));
                    lsteps = 0;
                    if (steps_used(steps, rejects, escal) >= HC_ARG(max_steps))
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
        cx<double> d = {0.0, 0.0};
        double nd2 = 0.0;
        bool sing = false;
        // the table reads are re-derived each stage (opaque pointers) so that the
        // loop-invariant ones are not all hoisted out of the loop into registers
        if (R64 || ballot(act && !p64) != 0ull) {
            const R *p0 = row0, *p1 = row1;
            lds_tab<R> cl = cl0 + gslot * kSlot;
            if constexpr (PARAM || TERMS)
                asm volatile("" : "+v"(p0), "+v"(p1));
            else
                asm volatile("" : "+v"(cl));
            if constexpr (TERMS)
                sing = stage_solve_terms<TKc, R, PARAM>(vrow, a.sdeg, T, p1, p0, lds, lane, r, base, own, nn, dg,
                                                        gam, xe, te, pred, d, nd2, ir, row1_64, row0_64, gam64);
            else
                sing = stage_solve<N, G, R, PARAM>(LdsRow<N, R>{cl}, p0, p1, r, base, d2, gam, gam64, xe, te, pred,
                                                   ir, d, nd2);
        }
        if constexpr (!R64 && kInl) {
            if (ballot(act && p64) != 0ull) {
                const double *q0 = row0_64, *q1 = row1_64;
                asm volatile("" : "+v"(q0), "+v"(q1));
                StageOut o;
                if constexpr (TERMS)
                    o = stage64_terms<TKc, PARAM>(vrow, a.sdeg, T, q1, q0, lds, lane, r, base, own, nn, dg, gam64, xe,
                                                  te, pred);
                else
                    o = stage64_dense<N, G, PARAM>(q0, q1, r, base, d2, gam64, xe, te, pred);
                if (p64) {
                    d = o.d;
                    nd2 = o.nd;
                    sing = o.sing;
                }
            }
        }

        if (act) {
            if (p64)
                lst64++;
            else
                lst32++;
            const double tau = p64 ? HC_ARG(tau64) : HC_ARG(tau);
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
                    if (phase == 4 && HC_ARG(max_newton) <= 0) ev = 2;
                }
            } else if (sing) {
                ev = 2;
            } else {
                xe = {xe.re + d.re, xe.im + d.im};
                const double nx = sqrt(group_sum<G>(abs2(xe)));
                const double nd = sqrt(nd2);
                nit++;
                nits++;
                if (nit == 1 && !(nd <= pred_tol * (1.0 + nx)))
                    ev = 2;
                else if (nd <= tau * (1.0 + nx))
                    ev = 1;
                else if (nit >= HC_ARG(max_newton))
                    ev = 2;
            }
            bool next_step = false;
            if (ev == 1) {
                x = xe;
                t = tn;
                steps++;
                lsteps++;
                if (++succ >= HC_ARG(n_inc)) {
                    h = fmin(h * HC_ARG(beta_inc), HC_ARG(h_max));
                    succ = 0;
                }
                const double m2 = abs2(x);
                if (group_any<G>(!(m2 <= HC_ARG(inf2)), base)) {
                    ev = 3;
                    fst = group_any<G>(isnan(m2), base) ? HC_T_NONFINITE : HC_T_AT_INFINITY;
                } else if (t >= HC_ARG(t_final)) {
                    save(HC_ARG(t_final) >= 1.0 ? kReached : kRunning);
                } else {
                    if (!p64 && t >= HC_ARG(t_switch)) p64 = true;  // FP64 end zone
                    next_step = true;
                }
            } else if (ev == 2) {
                rejects++;
                lsteps++;
                succ = 0;
                h *= HC_ARG(beta_dec);
                if (h < HC_ARG(h_min)) {
                    ev = 3;
                    fst = HC_T_MIN_STEP;
                } else {
                    next_step = true;
                }
            }
            if (next_step) {
                if (HC_ARG(launch_steps) > 0 && lsteps >= HC_ARG(launch_steps)) {
                    if (r == 0) atomicAdd(HC_ARG(n_suspended), 1u);
                    save(kRunning);
                } else if (steps_used(steps, rejects, escal) >= HC_ARG(max_steps)) {
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
#undef HC_ARG

}  // namespace hcx

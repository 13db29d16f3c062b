// hc_track_group.hip -- path tracker with G lanes per path, one row per lane.
//
// Mapping: a wavefront holds 64/G paths; lane r of a group (G = 4, 8 or 16,
// G >= n) owns equation r: its coefficients stay in VGPRs for the whole work
// item (every group of the wavefront works on the same instance), and each
// stage it builds row r of the augmented matrix [H_x | rhs].  The LU with
// partial pivoting then runs across the group (section 6: one row per thread):
//   * pivot search: a DPP max-reduction over the group of (|Re|+|Im|, row) keys;
//   * no rows move: the pivot row's remaining entries are broadcast to the group
//     with ds_bpermute and every not-yet-pivotal row eliminates against them;
//     each lane remembers the position at which its row became pivotal;
//   * back substitution walks the positions downwards, the pivot lane of each
//     position producing one unknown and broadcasting it, so every lane ends
//     with the whole solution vector.
// Path state (point, RK4 accumulator, t, h, counters) is replicated in the
// group's lanes, which take identical decisions on identical data.  Per-stage
// latency is about G times shorter than with one path per lane, so the long
// paths of a batch no longer hold a wavefront for G times longer.
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

// Row r of [H_x | rhs] at (x, t) for H = (1-t) gamma G + t F (see build_td in
// hc_kernels.hip for the formulas): the lane's own equation only.
template <int N, typename R>
__device__ __forceinline__ void build_row(const cx<R> &c0, const cx<R> (&L)[N], const cx<R> (&Q)[nquad(N)], int r,
                                          bool d2, cx<R> gam, const cx<R> (&x)[N], R t, bool pred,
                                          cx<R> (&row)[N + 1])
{
    cx<R> Lx = {R(0), R(0)};
#pragma unroll
    for (int j = 0; j < N; j++) {
        row[j] = L[j];
        Lx = cfma(L[j], x[j], Lx);
    }
    int q = 0;
#pragma unroll
    for (int a = 0; a < N; a++) {
#pragma unroll
        for (int b = a; b < N; b++) {
            const cx<R> cq = Q[q++];
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

// Row r of [H_x | rhs] for the parameter homotopy H = F(x; c(t)) with the
// coefficients interpolated linearly between the start and the target instance
// (section 6): c(t) = (1-t) c0 + t c1 and H_t = F(x; c1 - c0).  The lane's two
// coefficient rows are read from the kernel tables each stage.
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

// Solves the group's n x n system [A | b] (row r in this lane) by elimination
// with partial pivoting across the group; every lane receives the whole
// solution in dx.  Must run with the whole wavefront active.  Returns true if a
// pivot is (numerically) zero.
template <int N, int G, typename R>
__device__ __forceinline__ bool group_solve(cx<R> (&row)[N + 1], int r, int base, cx<R> (&dx)[N])
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
#pragma unroll
    for (int k = N - 1; k >= 0; k--) {
        const cx<R> xk = bcast(cmul(b, inv_own), base + pl[k]);
        dx[k] = xk;
        const bool above = pos < k;
        b = csel(above, cfms(row[k], xk, b), b);
    }
    return sing;
}

}  // namespace

// Tracks the paths tb .. tend-1 of instance `inst` with the wavefront's lane
// groups until every one of them has ended or been suspended.  Called with the
// whole wavefront active and wavefront-uniform arguments.
template <int N, int G, typename R, bool PARAM>
__device__ __forceinline__ void run_item(const TrackArgs &a, const int inst, const int tb, const int tend)
{
    static_assert(G == 4 || G == 8 || G == 16, "group size");
    static_assert(N <= G, "one row per lane");
    constexpr int T = dense_terms(N);
    constexpr int NQ = nquad(N);
    const int lane = threadIdx.x & 63;
    const int r = lane & (G - 1);
    const int base = lane - r;
    cx<R> gam = {R(1), R(0)};
    if (a.gamma) gam = {R(a.gamma[2 * inst]), R(a.gamma[2 * inst + 1])};
    const long long gbase = (long long)inst * a.n_start;
    const long long total = a.total;
    const TrackState S = a.s;
    const R tau = R(a.tau), pred_tol = R(a.pred_tol);

    // this lane's equation, kept in VGPRs for the whole item (total degree)
    cx<R> c0 = {R(0), R(0)}, L[N], Q[NQ];
#pragma unroll
    for (int j = 0; j < N; j++) L[j] = {R(0), R(0)};
#pragma unroll
    for (int q = 0; q < NQ; q++) Q[q] = {R(0), R(0)};
    const bool d2 = r < N && ((a.deg2 >> r) & 1u);
    // parameter homotopy: the lane's start and target rows (padding lanes read row 0)
    const R *row0 = static_cast<const R *>(a.coef0) + (size_t)(r < N ? r : 0) * T * 2;
    const R *row1 = static_cast<const R *>(a.coef) + ((size_t)inst * N + (r < N ? r : 0)) * T * 2;
    if (!PARAM && r < N) {
        const R *ce = static_cast<const R *>(a.coef) + ((size_t)inst * N + r) * T * 2;
        c0 = {ce[0], ce[1]};
#pragma unroll
        for (int j = 0; j < N; j++) L[j] = {ce[2 * (1 + j)], ce[2 * (1 + j) + 1]};
#pragma unroll
        for (int q = 0; q < NQ; q++) Q[q] = {ce[2 * (1 + N + q)], ce[2 * (1 + N + q) + 1]};
    }

    int trk = -1;
    long long g = 0;
    cx<R> x[N], xe[N], acc[N];
#pragma unroll
    for (int j = 0; j < N; j++) x[j] = xe[j] = acc[j] = {R(1), R(0)};
    double t = 0.0, h = 0.0, te = 0.0, hu = 0.0, tn = 0.0;
    int phase = 0, nit = 0, succ = 0, steps = 0, rejects = 0, nits = 0, lsteps = 0, escal = 0;
    unsigned lstages = 0;
    int next = tb;

    auto save = [&](int st) {
        if (r == 0) {
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
#pragma unroll
        for (int j = 0; j < N; j++) xe[j] = x[j];
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
        cx<R> row[N + 1];
        if constexpr (PARAM) {
            // re-derived each stage so the loop-invariant table reads are not all
            // hoisted out of the loop into registers
            const R *p0 = row0, *p1 = row1;
            asm volatile("" : "+v"(p0), "+v"(p1));
            build_row_param<N, R>(p0, p1, xe, R(te), phase < 4, row);
        } else {
            build_row<N, R>(c0, L, Q, r, d2, gam, xe, R(te), phase < 4, row);
        }
        cx<R> dx[N];
        const bool sing = group_solve<N, G, R>(row, r, base, dx);

        if (act) {
            lstages++;
            // 0: stage done, 1: accept the step, 2: reject it, 3: path failed (fst)
            int ev = 0, fst = 0;
            if (phase < 4) {
                bool ok = true;
#pragma unroll
                for (int j = 0; j < N; j++) ok = ok && finite(dx[j]);
                if (sing) {
                    ev = 2;
                } else if (phase == 0 && !ok) {
                    ev = 3;
                    fst = HC_T_NONFINITE;
                } else {
                    const R half = R(0.5 * hu), full = R(hu), sixth = R(hu / 6.0);
#pragma unroll
                    for (int j = 0; j < N; j++) {
                        const R w = (phase == 0 || phase == 3) ? R(1) : R(2);
                        acc[j].re = phase == 0 ? dx[j].re : fma(w, dx[j].re, acc[j].re);
                        acc[j].im = phase == 0 ? dx[j].im : fma(w, dx[j].im, acc[j].im);
                        const R c = phase < 2 ? half : full;
                        xe[j].re = phase == 3 ? fma(sixth, acc[j].re, x[j].re) : fma(c, dx[j].re, x[j].re);
                        xe[j].im = phase == 3 ? fma(sixth, acc[j].im, x[j].im) : fma(c, dx[j].im, x[j].im);
                    }
                    te = phase == 0 || phase == 1 ? t + 0.5 * hu : tn;
                    nit = 0;
                    phase++;
                    if (phase == 4 && a.max_newton <= 0) ev = 2;
                }
            } else if (sing) {
                ev = 2;
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
                    ev = 2;
                else if (nd <= tau * (R(1) + nx))
                    ev = 1;
                else if (nit >= a.max_newton)
                    ev = 2;
            }
            bool next_step = false;
            if (ev == 1) {
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
                if (!((double)big <= a.inf2)) {
                    ev = 3;
                    fst = isnan(big) ? HC_T_NONFINITE : HC_T_AT_INFINITY;
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

// One work item per wavefront, items in block order (XCD-aware).
template <int N, int G, typename R, bool PARAM>
__global__ __launch_bounds__(256) void k_track_grp(const TrackArgs a)
{
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = blockDim.x >> 6;
    const int item = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * wpb + wib);
    if (item >= a.n_items) return;
    const int inst = item / a.items_per_inst;
    const int tb = (item - inst * a.items_per_inst) * a.tracks_per_item;
    const int tend = min(tb + a.tracks_per_item, a.n_start);
    run_item<N, G, R, PARAM>(a, inst, tb, tend);
}

// Persistent tracker over a device work queue: each wavefront pops work items
// (job, instance, path range) with one atomic until the queue is empty and runs
// them with the code for the item's n.  Jobs may differ in n, kind-matching
// PARAM, path count and instance count.  Every wavefront leaves once the queue
// head passes n_items, so the grid always drains.
template <typename R, bool PARAM>
__global__ __launch_bounds__(256, (sizeof(R) == 4 && !PARAM) ? 2 : 1) void k_track_queue(const TrackArgs *__restrict__ jobs,
                                                     const QueueItem *__restrict__ items, int n_items,
                                                     unsigned *head)
{
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(head, 1u);
        const int idx = (int)__builtin_amdgcn_readfirstlane(got);
        if (idx >= n_items) break;
        const QueueItem it = items[idx];
        const TrackArgs a = jobs[it.job];
        switch (a.n) {
        case 2: run_item<2, 4, R, PARAM>(a, it.inst, it.tb, it.tend); break;
        case 3: run_item<3, 4, R, PARAM>(a, it.inst, it.tb, it.tend); break;
        case 4: run_item<4, 4, R, PARAM>(a, it.inst, it.tb, it.tend); break;
        case 5: run_item<5, 8, R, PARAM>(a, it.inst, it.tb, it.tend); break;
        case 6: run_item<6, 8, R, PARAM>(a, it.inst, it.tb, it.tend); break;
        case 7: run_item<7, 8, R, PARAM>(a, it.inst, it.tb, it.tend); break;
        case 8: run_item<8, 8, R, PARAM>(a, it.inst, it.tb, it.tend); break;
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

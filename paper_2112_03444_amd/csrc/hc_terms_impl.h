// hc_terms_impl.h -- kernels and launchers of the group tracker for the
// term-list layout, templated on the kernel kind (see TermKind in hc_group.h):
// G lanes per path, one row per lane, rows n..NM-1 identity.  Each kind's
// source file includes this and instantiates its launchers; the device code of
// the tracker is in hc_group.h.
#pragma once

#include "hc_group.h"

namespace hcx {

namespace {

template <int TK>
constexpr int terms_lds_bytes()
{
    return 4 * terms_lds_cx<TermCfg<TK>::NM, TermCfg<TK>::G>() * (int)sizeof(cx<double>);
}

template <int TK>
constexpr size_t terms_wave_bytes()
{
    return (size_t)terms_lds_cx<TermCfg<TK>::NM, TermCfg<TK>::G>() * sizeof(cx<double>);
}

// LDS slice of one wavefront of the tracker in precision R: FP64-sized where
// FP64 stages run in it (the FP64 tracker, an FP32 tracker with inline
// escalation), else FP32 entries plus the 64 FP64 stage-point entries of the
// fp64_residual option.
template <int TK, typename R>
constexpr size_t track_wave_bytes()
{
    return (sizeof(R) == 8 || TermCfg<TK>::INLINE_ESC)
               ? terms_wave_bytes<TK>()
               : (size_t)terms_lds_cx<TermCfg<TK>::NM, TermCfg<TK>::G>() * sizeof(cx<float>) + 64 * sizeof(cx<double>);
}

}  // namespace

// Persistent tracker for one job on the term-list layout.
template <int TK, typename R, bool PARAM>
__global__ __launch_bounds__(256, TermCfg<TK>::template waves<R>()) void k_track_terms(const TrackArgs a)
{
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ __align__(16) unsigned char buf[4 * track_wave_bytes<TK, R>()];
    GridSource src{a.head, a.n_items, a.items_per_inst, a.tracks_per_item, a.n_start, false};
    run_items<TermCfg<TK>::NM, TermCfg<TK>::G, R, PARAM, GridSource, TK, -1, true>(
        a, src, reinterpret_cast<cx<R> *>(buf + (size_t)wib * track_wave_bytes<TK, R>()));
}

// Persistent tracker over a device work queue of term-list jobs of one kind.
// Mixed precision escalates inline here on every kind (FP64-sized LDS slices).
template <int TK, typename R, bool PARAM>
__global__ __launch_bounds__(256, TermCfg<TK>::QUEUE_WAVES) void k_track_queue_terms(
    const TrackArgs *__restrict__ jobs, const QueueItem *__restrict__ items, int n_items, unsigned *head)
{
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ __align__(16) unsigned char buf[terms_lds_bytes<TK>()];
    cx<R> *lds = reinterpret_cast<cx<R> *>(buf + (size_t)wib * terms_wave_bytes<TK>());
    QueueSource src{items, head, n_items, 0, false, false, false, {}, {}};
    for (;;) {
        QueueItem it;
        if (src.has_pending) {
            it = src.pending;
            src.has_pending = false;
        } else {
            unsigned got = 0;
            if (lane == 0) got = atomicAdd(head, 1u);
            const int idx = (int)__builtin_amdgcn_readfirstlane(got);
            if (idx >= n_items) break;
            it = items[idx];
        }
        const TrackArgs a = jobs[it.job];
        src.job = it.job;
        src.first = it;
        src.has_first = true;
        src.done = false;
        run_items<TermCfg<TK>::NM, TermCfg<TK>::G, R, PARAM, QueueSource, TK, 1>(a, src, lds);
        if (src.done && !src.has_pending) break;
    }
}

// FP64 endpoint refinement and classification (as k_refine) for the term-list
// layout: Newton on F(x; c1) at t = 1 with the group solver, then the relative
// backward error eta = max_i |F_i| / sum_k |c_ik| |m_k(x)|.  One path per group
// of G lanes, 64 / G paths per wavefront.
template <int TK>
__device__ __forceinline__ void refine_terms_body(const RefineArgs &a, int block)
{
    constexpr int NM = TermCfg<TK>::NM, G = TermCfg<TK>::G, PW = 64 / G;
    constexpr bool GEN = TermCfg<TK>::GEN;
    const int lane = threadIdx.x & 63;
    const int r = lane & (G - 1);
    const int base = lane - r;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ __align__(16) unsigned char buf[terms_lds_bytes<TK>()];
    void *lds = buf + (size_t)wib * terms_wave_bytes<TK>();
    if (a.total == 0) return;
    const long long gid = ((long long)block * 4 + wib) * PW + lane / G;
    const bool valid = gid < a.total;
    const long long g = valid ? gid : 0;  // spare groups redo path 0 and write nothing
    const int n = a.n, T = a.n_tslots;
    const bool own = r < n;
    const int rr = own ? r : 0;
    const int inst = (int)(g / a.n_start);
    const double *c1 = a.coef + ((size_t)inst * n + rr) * T * 2;
    const void *vr = GEN ? (const void *)(static_cast<const unsigned long long *>(a.vars) + (size_t)rr * T)
                         : (const void *)(static_cast<const unsigned short *>(a.vars) + (size_t)rr * T);
    const TrackState S = a.s;
    const long long total = a.total;
    int st = S.status[g];
    const bool done = st == kDone;  // final from an earlier pass: nothing to write
    // a wavefront with nothing to write (the re-refinement after a crossing
    // check: all but the re-tracked paths are done) leaves at once
    if (ballot(valid && !done) == 0ull) return;
    cx<double> x = own ? cx<double>{S.xr[r * total + g], S.xi[r * total + g]} : cx<double>{0.0, 0.0};
    bool act = valid && st == kReached;
    int rits = 0;
    for (int it = 0; it < a.max_refine; it++) {
        if (ballot(act) == 0ull) break;
        const double *p1 = c1;
        asm volatile("" : "+v"(p1));
        cx<double> d;
        double nd;
        const bool sing = stage_solve_terms<TK, double, false>(vr, a.sdeg, T, p1, nullptr, lds, lane, r, base, own, n,
                                                               1, cx<double>{1.0, 0.0}, x, 1.0, false, d, nd);
        if (act) {
            if (sing) {
                st = HC_T_SINGULAR;
                act = false;
            } else {
                x = {x.re + d.re, x.im + d.im};
                const double nx = sqrt(group_sum<G>(abs2(x)));
                rits++;
                if (sqrt(nd) <= a.tau_refine * (1.0 + nx)) act = false;
            }
        }
    }
    // classification: the whole wavefront takes part in the group reductions
    const double m2 = abs2(x);
    const bool nonfin = group_any<G>(own && !finite(x), base);
    const double big = group_max_d<G>(m2);
    // residual of the lane's equation at x
    const lds_tab<double> xs = (lds_tab<double>)(cx<double> *)lds;
    stl(xs, lane, own ? x : cx<double>{0.0, 0.0});
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    cx<double> F = {0.0, 0.0};
    double den = 0.0;
    for (int k = 0; k < (own ? T : 0); k++) {
        const cx<double> c = {c1[2 * k], c1[2 * k + 1]};
        cx<double> m = {1.0, 0.0};
        double am = 1.0;  // |m_k(x)|
        if constexpr (GEN) {
            const unsigned long long v = static_cast<const unsigned long long *>(vr)[k];
            for (int i = 0; i < 8; i++) {
                const int f = (int)((v >> (8 * i)) & 0xFFull);
                if (f >= NM) break;
                const cx<double> xf = ldl(xs + base, f);
                m = cmul(m, xf);
                am *= sqrt(abs2(xf));
            }
        } else {
            const unsigned v = static_cast<const unsigned short *>(vr)[k];
            const int ia = (int)(v & 0xFFu), ib = (int)(v >> 8);
            const cx<double> xa = ia < NM ? ldl(xs + base, ia) : cx<double>{1.0, 0.0};
            const cx<double> xb = ib < NM ? ldl(xs + base, ib) : cx<double>{1.0, 0.0};
            m = cmul(xa, xb);
            am = sqrt(abs2(xa)) * sqrt(abs2(xb));
        }
        F = cfma(c, m, F);
        den += sqrt(abs2(c)) * am;
    }
    const double num = sqrt(abs2(F));
    const double e = !own ? 0.0 : den > 0.0 ? num / den : (num == 0.0 ? 0.0 : INFINITY);
    const double resid = group_max_d<G>(e);
    if (!valid || done) return;
    double res_out = NAN;
    if (st == kReached) {
        if (nonfin) {
            st = HC_T_NONFINITE;
        } else {
            res_out = resid;
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
    if (own) {
        a.endpoints[(g * n + r) * 2] = x.re;
        a.endpoints[(g * n + r) * 2 + 1] = x.im;
    }
    if (r == 0) {
        a.status[g] = st;
        if (a.info) {
            hc_track_info inf;
            inf.steps = S.steps[g];
            inf.rejects = S.rejects[g];
            inf.newton_its = S.nits[g];
            inf.refine_its = rits;
            inf.escalated = S.escal[g] != 0 ? 1 : 0;
            inf.cycle = a.eg_cycle ? S.succ[g] : 0;
            inf.residual = res_out;
            a.info[g] = inf;
        }
    }
}

template <int TK>
__global__ __launch_bounds__(256) void k_refine_terms(const RefineArgs a)
{
    refine_terms_body<TK>(a, blockIdx.x);
}

template <int TK>
__global__ __launch_bounds__(256) void k_refine_terms_many(const RefineArgs *a)
{
    refine_terms_body<TK>(a[blockIdx.y], blockIdx.x);
}

namespace {

template <typename K>
int resident_waves_terms(K kern, std::atomic<int> (&cache)[16])
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < 16) {
        const int c = cache[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int cus = 0, blocks = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kern, 256, 0) != hipSuccess || blocks < 1) blocks = 1;
    const int w = cus * blocks * 4;
    if (dev >= 0 && dev < 16) cache[dev].store(w, std::memory_order_relaxed);
    return w;
}

// Resident wavefronts of one kernel instance, cached per device.
template <int TK, bool QUEUE, typename R, bool PARAM>
int resident_waves_of()
{
    static std::atomic<int> cache[16];
    if constexpr (QUEUE)
        return resident_waves_terms(k_track_queue_terms<TK, R, PARAM>, cache);
    else
        return resident_waves_terms(k_track_terms<TK, R, PARAM>, cache);
}

}  // namespace

template <int TK>
hipError_t launch_track_terms_k(bool fp32, const TrackArgs &a, hipStream_t st)
{
    if (a.n_items == 0) return hipSuccess;
    auto go = [&](auto kern, int res) -> hipError_t {
        if (res <= 0) return hipErrorInvalidDevice;
        const int waves = std::min(a.n_items, res);
        hipLaunchKernelGGL(kern, dim3((waves + 3) / 4), dim3(256), 0, st, a);
        return hipGetLastError();
    };
    if (a.coef0)
        return fp32 ? go(k_track_terms<TK, float, true>, resident_waves_of<TK, false, float, true>())
                    : go(k_track_terms<TK, double, true>, resident_waves_of<TK, false, double, true>());
    return fp32 ? go(k_track_terms<TK, float, false>, resident_waves_of<TK, false, float, false>())
                : go(k_track_terms<TK, double, false>, resident_waves_of<TK, false, double, false>());
}

template <int TK>
hipError_t launch_track_queue_terms_k(bool fp32, bool param, const TrackArgs *jobs, const QueueItem *items,
                                      int n_items, unsigned *head, int n_waves, hipStream_t st)
{
    if (n_items == 0) return hipSuccess;
    const dim3 grid((n_waves + 3) / 4), block(256);
    if (param) {
        if (fp32)
            hipLaunchKernelGGL((k_track_queue_terms<TK, float, true>), grid, block, 0, st, jobs, items, n_items, head);
        else
            hipLaunchKernelGGL((k_track_queue_terms<TK, double, true>), grid, block, 0, st, jobs, items, n_items, head);
    } else {
        if (fp32)
            hipLaunchKernelGGL((k_track_queue_terms<TK, float, false>), grid, block, 0, st, jobs, items, n_items, head);
        else
            hipLaunchKernelGGL((k_track_queue_terms<TK, double, false>), grid, block, 0, st, jobs, items, n_items,
                               head);
    }
    return hipGetLastError();
}

template <int TK>
int queue_waves_terms_k(bool fp32, bool param)
{
    if (param) return fp32 ? resident_waves_of<TK, true, float, true>() : resident_waves_of<TK, true, double, true>();
    return fp32 ? resident_waves_of<TK, true, float, false>() : resident_waves_of<TK, true, double, false>();
}

// many: a is a device array of `count` jobs (max_total: the largest job's path
// count), else a host reference to one job (count 1).
template <int TK>
hipError_t launch_refine_terms_k(const RefineArgs *a, int count, long long max_total, bool many, hipStream_t st)
{
    if (count == 0 || max_total == 0) return hipSuccess;
    constexpr int PB = 4 * (64 / TermCfg<TK>::G);  // paths per block
    const unsigned blocks = (unsigned)((max_total + PB - 1) / PB);
    if (many)
        hipLaunchKernelGGL(k_refine_terms_many<TK>, dim3(blocks, (unsigned)count), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_refine_terms<TK>, dim3(blocks), dim3(256), 0, st, *a);
    return hipGetLastError();
}

}  // namespace hcx

// Declaration that another source file instantiates one kind's launchers.
#define HC_TERMS_EXTERN(TK)                                                                                        \
    namespace hcx {                                                                                                \
    extern template hipError_t launch_track_terms_k<TK>(bool, const TrackArgs &, hipStream_t);                    \
    extern template hipError_t launch_track_queue_terms_k<TK>(bool, bool, const TrackArgs *, const QueueItem *,   \
                                                              int, unsigned *, int, hipStream_t);                  \
    extern template int queue_waves_terms_k<TK>(bool, bool);                                                      \
    extern template hipError_t launch_refine_terms_k<TK>(const RefineArgs *, int, long long, bool, hipStream_t);  \
    }

// Explicit instantiation of one kind's launchers.
#define HC_TERMS_INSTANTIATE(TK)                                                                                   \
    namespace hcx {                                                                                                \
    template hipError_t launch_track_terms_k<TK>(bool, const TrackArgs &, hipStream_t);                           \
    template hipError_t launch_track_queue_terms_k<TK>(bool, bool, const TrackArgs *, const QueueItem *, int,     \
                                                       unsigned *, int, hipStream_t);                              \
    template int queue_waves_terms_k<TK>(bool, bool);                                                             \
    template hipError_t launch_refine_terms_k<TK>(const RefineArgs *, int, long long, bool, hipStream_t);         \
    }

// hc_track_group.hip -- kernels and launchers of the group tracker for the dense
// quadratic table layout (n <= 8); the device code is in hc_group.h.
#include "hc_group.h"

namespace hcx {

// LDS of a block of 4 wavefronts: kSlots tables of n x T complex values each.
template <typename R, int SLOT>
constexpr int tab_bytes() { return 4 * kSlots * SLOT * (int)sizeof(cx<R>); }

// Persistent tracker for one job: each wavefront pops work items from a device
// counter (GridSource) until none is left.
template <int N, int G, typename R, bool PARAM>
__global__ __launch_bounds__(256, PARAM ? 1 : 2) void k_track_grp(const TrackArgs a)
{
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr int kSlot = N * dense_terms(N);
    __shared__ __align__(16) unsigned char tab[tab_bytes<R, kSlot>()];
    GridSource src{a.head, a.n_items, a.items_per_inst, a.tracks_per_item, a.n_start, false};
    // n >= 5: launch constants read from the kernel-argument segment where they
    // are used (held in scalar registers they spill to vector lanes); the short
    // stages of n <= 4 are better off keeping them in registers
    run_items<N, G, R, PARAM, GridSource, -1, -1, (N >= 5)>(a, src,
                                                            reinterpret_cast<cx<R> *>(tab) + wib * kSlots * kSlot);
}

// Persistent tracker over a device work queue: each wavefront pops work items
// (job, instance, path range) with one atomic until the queue is empty and runs
// them with the code for the item's n, continuing with the following items of
// the same job.  Jobs may differ in n, kind-matching PARAM, path count and
// instance count.  Every wavefront leaves once the queue head passes n_items,
// so the grid always drains.
template <typename R, bool PARAM>
__global__ __launch_bounds__(256, PARAM ? 1 : 2) void k_track_queue(const TrackArgs *__restrict__ jobs,
                                                                  const QueueItem *__restrict__ items,
                                                                  int n_items, unsigned *head)
{
    constexpr int kMaxSlot = 8 * dense_terms(8);
    const int lane = threadIdx.x & 63;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ __align__(16) unsigned char tab[tab_bytes<R, kMaxSlot>()];
    cx<R> *lds = reinterpret_cast<cx<R> *>(tab) + wib * kSlots * kMaxSlot;
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
        switch (a.n) {
        case 2: run_items<2, 4, R, PARAM>(a, src, lds); break;
        case 3: run_items<3, 4, R, PARAM>(a, src, lds); break;
        case 4: run_items<4, 4, R, PARAM>(a, src, lds); break;
        case 5: run_items<5, 8, R, PARAM>(a, src, lds); break;
        case 6: run_items<6, 8, R, PARAM>(a, src, lds); break;
        case 7: run_items<7, 8, R, PARAM>(a, src, lds); break;
        case 8: run_items<8, 8, R, PARAM>(a, src, lds); break;
        default: break;
        }
        if (src.done && !src.has_pending) break;
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

// Wavefronts of kernel `K` (256-thread blocks) resident on the current device,
// cached per device.
template <typename K>
static int resident_waves(K kern)
{
    static std::atomic<int> cache[16];
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

template <typename K>
static hipError_t launch_persistent(K kern, const TrackArgs &a, hipStream_t st)
{
    const int res = resident_waves(kern);
    if (res <= 0) return hipErrorInvalidDevice;
    const int waves = std::min(a.n_items, res);
    hipLaunchKernelGGL(kern, dim3((waves + 3) / 4), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int N, int G>
static hipError_t launch_grp(bool fp32, const TrackArgs &a, hipStream_t st)
{
    if (a.coef0) {
        if (fp32) return launch_persistent(k_track_grp<N, G, float, true>, a, st);
        return launch_persistent(k_track_grp<N, G, double, true>, a, st);
    }
    if (fp32) return launch_persistent(k_track_grp<N, G, float, false>, a, st);
    return launch_persistent(k_track_grp<N, G, double, false>, a, st);
}

hipError_t launch_track_group(int n, bool fp32, const TrackArgs &a, hipStream_t st)
{
    if (a.n_items == 0) return hipSuccess;
    switch (n) {
    case 2: return launch_grp<2, 4>(fp32, a, st);
    case 3: return launch_grp<3, 4>(fp32, a, st);
    case 4: return launch_grp<4, 4>(fp32, a, st);
    case 5: return launch_grp<5, 8>(fp32, a, st);
    case 6: return launch_grp<6, 8>(fp32, a, st);
    case 7: return launch_grp<7, 8>(fp32, a, st);
    case 8: return launch_grp<8, 8>(fp32, a, st);
    default: return hipErrorInvalidValue;
    }
}

int group_lanes(int n) { return n <= 4 ? 4 : 8; }

// FP64 endpoint refinement and classification for the dense quadratic layout,
// one path per group of G lanes (64 / G per wavefront) with the trackers' row
// build and group solver: Newton on F at t = 1 (where H = F and H_x = F_x) until
// the correction is below tau_refine (1 + |x|) or max_refine iterations, then the
// relative backward error eta = max_i |F_i| / sum_k |c_ik| |m_k(x)| over the
// equations (one per lane) and the final status.  The table is the kernel table
// [inst][eq][term] in FP64, diagonal quadratic coefficients stored doubled.
template <int N, int G>
__device__ __forceinline__ void refine_grp_body(const RefineArgs &a, int block)
{
    constexpr int T = dense_terms(N), PW = 64 / G;
    const int lane = threadIdx.x & 63;
    const int r = lane & (G - 1);
    const int base = lane - r;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (a.total == 0) return;
    const long long gid = ((long long)block * 4 + wib) * PW + lane / G;
    const bool valid = gid < a.total;
    const long long g = valid ? gid : 0;  // spare groups redo path 0 and write nothing
    const bool own = r < N;
    const int rr = own ? r : 0;
    const int inst = (int)(g / a.n_start);
    const double *c1 = a.coef + ((size_t)inst * N + rr) * T * 2;
    cx<double> gam = {1.0, 0.0};
    if (a.gamma) gam = {a.gamma[2 * inst], a.gamma[2 * inst + 1]};
    const bool d2 = own && ((a.deg2 >> r) & 1u);
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
        const bool sing = stage_solve<N, G, double, false>(GlobalRow<double>{p1}, nullptr, p1, r, base, d2, gam, gam,
                                                           x, 1.0, false, false, d, nd);
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
    const bool nonfin = group_any<G>(own && !finite(x), base);
    const double big = group_max_d<G>(abs2(x));
    cx<double> xs[N];
    gather<G, N>(x, xs);
    // residual of the lane's equation: constant, linear and quadratic terms
    cx<double> F = {c1[0], c1[1]};
    double den = sqrt(abs2(F));
#pragma unroll
    for (int j = 0; j < N; j++) {
        const cx<double> L = {c1[2 * (1 + j)], c1[2 * (1 + j) + 1]};
        F = cfma(L, xs[j], F);
        den += sqrt(abs2(L)) * sqrt(abs2(xs[j]));
    }
    int q = 1 + N;
#pragma unroll
    for (int p = 0; p < N; p++) {
#pragma unroll
        for (int b = p; b < N; b++, q++) {
            cx<double> cq = {c1[2 * q], c1[2 * q + 1]};
            if (p == b) cq = {0.5 * cq.re, 0.5 * cq.im};
            const cx<double> m = cmul(xs[p], xs[b]);
            F = cfma(cq, m, F);
            den += sqrt(abs2(cq)) * sqrt(abs2(m));
        }
        asm volatile("" ::: "memory");  // one row segment of the table in registers at a time
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
        a.endpoints[(g * N + r) * 2] = x.re;
        a.endpoints[(g * N + r) * 2 + 1] = x.im;
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

template <int N, int G>
__global__ __launch_bounds__(256, 2) void k_refine_grp(const RefineArgs a) { refine_grp_body<N, G>(a, blockIdx.x); }

template <int N, int G>
__global__ __launch_bounds__(256, 2) void k_refine_grp_many(const RefineArgs *a)
{
    refine_grp_body<N, G>(a[blockIdx.y], blockIdx.x);
}

template <int N, int G>
static hipError_t launch_refine_grp(const RefineArgs *a, int count, long long max_total, bool many, hipStream_t st)
{
    constexpr int PB = 4 * (64 / G);  // paths per block
    const unsigned blocks = (unsigned)((max_total + PB - 1) / PB);
    if (many)
        hipLaunchKernelGGL((k_refine_grp_many<N, G>), dim3(blocks, (unsigned)count), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_refine_grp<N, G>), dim3(blocks), dim3(256), 0, st, *a);
    return hipGetLastError();
}

hipError_t launch_refine_group(int n, const RefineArgs *a, int count, long long max_total, bool many, hipStream_t st)
{
    if (count == 0 || max_total == 0) return hipSuccess;
    switch (n) {
    case 2: return launch_refine_grp<2, 4>(a, count, max_total, many, st);
    case 3: return launch_refine_grp<3, 4>(a, count, max_total, many, st);
    case 4: return launch_refine_grp<4, 4>(a, count, max_total, many, st);
    case 5: return launch_refine_grp<5, 8>(a, count, max_total, many, st);
    case 6: return launch_refine_grp<6, 8>(a, count, max_total, many, st);
    case 7: return launch_refine_grp<7, 8>(a, count, max_total, many, st);
    case 8: return launch_refine_grp<8, 8>(a, count, max_total, many, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hcx

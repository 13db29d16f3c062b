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
    run_items<N, G, R, PARAM>(a, src, reinterpret_cast<cx<R> *>(tab) + wib * kSlots * kSlot);
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

}  // namespace hcx

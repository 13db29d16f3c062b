// hc_terms_q16.hip -- term-list tracker kernels of kind 0 (degree <= 2, n <= 16, 16 lanes per path)
// and the dispatch over all kinds.
#include "hc_terms_impl.h"

HC_TERMS_INSTANTIATE(0)
HC_TERMS_EXTERN(1)  // hc_terms_g16.hip
HC_TERMS_EXTERN(2)  // hc_terms_g20.hip
HC_TERMS_EXTERN(3)  // hc_terms_q14.hip
HC_TERMS_EXTERN(4)  // hc_terms_g18.hip
HC_TERMS_EXTERN(5)  // hc_terms_q10.hip
HC_TERMS_EXTERN(6)  // hc_terms_g32.hip

namespace hcx {

// Dispatch on the kernel kind of a term-list system.
hipError_t launch_track_terms(int tk, bool fp32, const TrackArgs &a, hipStream_t st)
{
    switch (tk) {
    case 0: return launch_track_terms_k<0>(fp32, a, st);
    case 1: return launch_track_terms_k<1>(fp32, a, st);
    case 2: return launch_track_terms_k<2>(fp32, a, st);
    case 3: return launch_track_terms_k<3>(fp32, a, st);
    case 4: return launch_track_terms_k<4>(fp32, a, st);
    case 5: return launch_track_terms_k<5>(fp32, a, st);
    case 6: return launch_track_terms_k<6>(fp32, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_track_queue_terms(int tk, bool fp32, bool param, const TrackArgs *jobs, const QueueItem *items,
                                    int n_items, unsigned *head, int n_waves, hipStream_t st)
{
    switch (tk) {
    case 0: return launch_track_queue_terms_k<0>(fp32, param, jobs, items, n_items, head, n_waves, st);
    case 1: return launch_track_queue_terms_k<1>(fp32, param, jobs, items, n_items, head, n_waves, st);
    case 2: return launch_track_queue_terms_k<2>(fp32, param, jobs, items, n_items, head, n_waves, st);
    case 3: return launch_track_queue_terms_k<3>(fp32, param, jobs, items, n_items, head, n_waves, st);
    case 4: return launch_track_queue_terms_k<4>(fp32, param, jobs, items, n_items, head, n_waves, st);
    case 5: return launch_track_queue_terms_k<5>(fp32, param, jobs, items, n_items, head, n_waves, st);
    case 6: return launch_track_queue_terms_k<6>(fp32, param, jobs, items, n_items, head, n_waves, st);
    default: return hipErrorInvalidValue;
    }
}

int queue_waves_terms(int tk, bool fp32, bool param)
{
    switch (tk) {
    case 0: return queue_waves_terms_k<0>(fp32, param);
    case 1: return queue_waves_terms_k<1>(fp32, param);
    case 2: return queue_waves_terms_k<2>(fp32, param);
    case 3: return queue_waves_terms_k<3>(fp32, param);
    case 4: return queue_waves_terms_k<4>(fp32, param);
    case 5: return queue_waves_terms_k<5>(fp32, param);
    case 6: return queue_waves_terms_k<6>(fp32, param);
    default: return 0;
    }
}

hipError_t launch_refine_terms(int tk, const RefineArgs &a, hipStream_t st)
{
    switch (tk) {
    case 0: return launch_refine_terms_k<0>(&a, 1, a.total, false, st);
    case 1: return launch_refine_terms_k<1>(&a, 1, a.total, false, st);
    case 2: return launch_refine_terms_k<2>(&a, 1, a.total, false, st);
    case 3: return launch_refine_terms_k<3>(&a, 1, a.total, false, st);
    case 4: return launch_refine_terms_k<4>(&a, 1, a.total, false, st);
    case 5: return launch_refine_terms_k<5>(&a, 1, a.total, false, st);
    case 6: return launch_refine_terms_k<6>(&a, 1, a.total, false, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_refine_terms_many(int tk, const RefineArgs *a, int count, long long max_total, hipStream_t st)
{
    switch (tk) {
    case 0: return launch_refine_terms_k<0>(a, count, max_total, true, st);
    case 1: return launch_refine_terms_k<1>(a, count, max_total, true, st);
    case 2: return launch_refine_terms_k<2>(a, count, max_total, true, st);
    case 3: return launch_refine_terms_k<3>(a, count, max_total, true, st);
    case 4: return launch_refine_terms_k<4>(a, count, max_total, true, st);
    case 5: return launch_refine_terms_k<5>(a, count, max_total, true, st);
    case 6: return launch_refine_terms_k<6>(a, count, max_total, true, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hcx

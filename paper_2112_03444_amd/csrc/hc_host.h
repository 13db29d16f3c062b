// hc_host.h -- host-side definitions shared by the C-ABI library's sources:
// error reporting, grow-only device buffers, loaded systems and contexts.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "hc.h"
#include "hc_internal.h"

namespace hcx {

// Records the message of the last error on this thread and returns `code`.
hc_status fail(hc_status code, const char *fmt, ...);
void clear_error();

#define HIP_TRY(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return ::hcx::fail(e_ == hipErrorOutOfMemory ? HC_E_OOM : HC_E_DEVICE, "%s: %s (%s:%d)", \
                               #call, hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

// A grow-only device buffer; `moves` counts reallocations (captured graphs and
// other holders of its address must notice when it moves).
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    unsigned long long moves = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        moves++;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max<size_t>(bytes, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

}  // namespace hcx

struct hc_system {
    int device = 0;
    int n = 0, n_terms = 0, n_params = 0, kind = 0, T = 0;  // T: table slots per equation
    int layout = HC_LAYOUT_DENSE;  // HC_LAYOUT_DENSE or HC_LAYOUT_TERMS
    unsigned deg2 = 0;
    int64_t bezout = 0;
    std::vector<int> deg;
    bool has_const = false, has_map = false;
    // device copies of the tables
    int *d_slot_ptr = nullptr, *d_slot_term = nullptr, *d_slot_mult = nullptr;
    double *d_term_const = nullptr;
    int *d_map_ptr = nullptr, *d_map_col = nullptr;
    double *d_map_val = nullptr;
    void *d_vars = nullptr;   // term lists: variables of every slot (16- or 64-bit entries)
    int tk = 0;               // term lists: kernel kind (term_kind_for: 5 / 3 / 0: degree <= 2,
                              //   n <= 10 / 14 / 16; 1 / 4 / 2 / 6: any degree, n <= 16 / 18 / 20 / 32)
    int max_deg = 0;          // largest term degree
    int *d_sdeg = nullptr;    // general-degree kinds: [T] largest degree of each slot
    int *d_eqdeg = nullptr;   // general-degree kinds: [n] equation degrees
    // the description as loaded: the autotuner loads the other table layout from it
    std::vector<int> h_term_eq, h_term_exp, h_rowptr, h_col;
    std::vector<hc_c64> h_const, h_val;
    hc_system *alt = nullptr; // the same family in the other table layout (autotuner), owned here
};

// An autotuner choice: table layout, lanes per path, paths per work item and
// steps per launch (0 = to the end).
struct TuneChoice {
    int layout = 0, lanes = 0, tpi = 0, spl = 0;
};

struct hc_ctx {
    int device = 0;
    hipStream_t own_stream = nullptr;  // used by the host-buffer entry point
    std::vector<hc_system *> systems;
    hcx::DevBuf state;   // SoA path state
    hcx::DevBuf coef;    // per-instance kernel tables (FP64 then FP32)
    hcx::DevBuf io;      // device copies of host inputs/outputs for hc_track
    hcx::DevBuf counter; // suspended-path counter, then two stage counters (profiling)
    hcx::DevBuf queue;   // batch: per-pass job descriptors, work items, queue heads
    hcx::DevBuf eg;      // end-game: candidate list, samples and estimates
    hcx::DevBuf evtab;   // hc_eval_dense_device: the instances' tables (FP64 then FP32)
    std::vector<hcx::TrackArgs> h_jobs;   // host copies kept alive across the async uploads
    std::vector<hcx::QueueItem> h_items;
    std::vector<unsigned char> h_blob;   // batch: staging of the one upload per call
    // hipGraph of the last hc_track_device call with use_graph, and its arguments
    bool graph_valid = false;
    std::vector<unsigned char> graph_key;
    hipGraphExec_t graph_exec = nullptr;
    // hipGraph of the last hc_track_batch_device call with use_graph
    bool bgraph_valid = false;
    std::vector<unsigned char> bgraph_key;
    hipGraphExec_t bgraph_exec = nullptr;
    // autotuner choices by workload shape (a text key that names the device
    // architecture, the system's table layout, kind, sizes and degrees, the
    // precision and the batch sizes); persisted by hc_tune_save / hc_tune_load
    std::string arch;
    std::map<std::string, TuneChoice> tune;
    std::string tune_file;   // HC_TUNE_CACHE at creation: loaded then, rewritten by hc_autotune
    // profiling: events bracketing prep | init | FP32 pass | FP64 pass | refine
    bool profiling = false;
    bool profiled_call = false;
    hipEvent_t ev[7] = {};
    int launches_fp32 = 0, launches_fp64 = 0;
    bool had_fp32 = false;
};

// hc_scratch.hip -- the fixed device workspace of hc_track_device_noalloc.
//
// A file-scope device array: every GPU the library runs on holds its own copy
// (kScratchBytes of device memory, from module load until the process ends).
// Host code never passes the array's name to a kernel or a copy -- on the host
// that name is only a stand-in, not a device address.  Its address on each
// device is looked up once, with that device current, by scratch_init (called
// from hc_create) and kept per device; every later use goes through it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hc_internal.h"

namespace hcx {

__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return hipSuccess;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) {
        e = hipSetDevice(device);
        if (e != hipSuccess) return e;
    }
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
    return hipSuccess;
}

void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace hcx

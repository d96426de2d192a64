// scratch.hip -- the static device array behind vbw_filter_noalloc.
//
// Callers that cannot allocate device memory get every device table of a
// call (twiddles, V, work list, per-call table) from one file-scope array per
// GPU, held until the process ends.  Host code never passes the array's
// host-side name to a kernel: each device's address of it is looked up once,
// with that device current, and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "vbw.h"
#include "vbw_internal.h"

static __device__ __align__(256) unsigned char scratch[VBW_NOALLOC_SCRATCH_BYTES];

namespace vbw {
namespace {

constexpr int kMaxDevices = 64;

struct Slot {
    bool ready = false;
    unsigned char *ptr = nullptr;
};
std::mutex g_mu;
Slot g_slot[kMaxDevices];

}  // namespace

hipError_t scratch_of_device(int device, unsigned char **ptr, hipError_t (*init)(unsigned char *)) {
    *ptr = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    Slot &s = g_slot[device];
    if (!s.ready) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the lookup needs the device current
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (init && (e = init(static_cast<unsigned char *>(p))) != hipSuccess) return e;
        s.ptr = static_cast<unsigned char *>(p);
        s.ready = true;
    }
    *ptr = s.ptr;
    return hipSuccess;
}

}  // namespace vbw

// Fixed device scratch for the entry points that allocate nothing.
//
// One file-scope device array per GPU the library runs on, held until the
// process ends.  Host code never uses the array's name as an address (on the
// host it is only a stand-in symbol): the device address of each GPU's copy is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and kept in a per-device table.  Every call on a GPU shares that
// GPU's copy, which keeps the last call's contents; calls that overlap on one
// GPU race.
#include "ah_internal.h"

#include <mutex>

namespace ah {
namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t scratch_ptr(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device) {
            e = hipSetDevice(device);
            if (e != hipSuccess) return e;
        }
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return hipSuccess;
}

}  // namespace ah

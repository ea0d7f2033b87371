// Static device scratch for the entry point that allocates nothing
// (dicod_solve_device_noalloc): the whole solve workspace of one call is
// carved from this array.  Each device that the library runs on holds its own
// copy for the life of the process; its address is looked up once per device
// and cached.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>

#include "dicod_internal.h"

namespace dicod {
namespace {

constexpr size_t kScratchBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

size_t scratch_bytes() { return kScratchBytes; }

hipError_t scratch_address(int device, void** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_addr[device]) {
        // the current device must be `device`: each device has its own copy
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_addr[device] = p;
    }
    *out = g_addr[device];
    return hipSuccess;
}

}  // namespace dicod

// ram_noalloc.hip -- the device scratch of ram_shift_noalloc, the entry point
// for callers that cannot allocate device memory.
//
// A file-scope device array of kNoAllocBytes holds that call's mesh tables,
// window plan or ragged tile table.  Each GPU the library runs on has its own
// copy at its own address, held until the process ends; host code never uses
// the array's name as an address (in host code it is only a stand-in): the
// address is taken once per device, with the device current, by
// hipGetSymbolAddress, and kept here.
#include "ram_internal.h"

#include <mutex>

namespace ram {
namespace {

__device__ __attribute__((aligned(256))) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    std::once_flag once;
    void *ptr = nullptr;
    hipError_t err = hipErrorNotInitialized;
};
DeviceScratch g_scratch[kMaxDevices];

} // namespace

hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    DeviceScratch &d = g_scratch[device];
    std::call_once(d.once, [&] {
        void *p = nullptr;
        d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        d.ptr = d.err == hipSuccess ? p : nullptr;
    });
    return d.err;
}

void *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    return g_scratch[device].err == hipSuccess ? g_scratch[device].ptr : nullptr;
}

} // namespace ram

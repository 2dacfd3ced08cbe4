// Scratch memory for the entry point that allocates nothing
// (ft_consume_queries_noalloc): a fixed device array that the code object
// carries, so a caller that may not allocate device memory (work under HIP
// graph capture, serving loops, allocation-free harnesses) still has room for
// the per-element loads between the element kernel and the node assembly.
//
// Each GPU the library runs on holds its own copy of the array from the
// moment the code object is loaded there until the process ends.  On the
// host the array's name is only a stand-in for it: its device address, per
// device, comes from hipGetSymbolAddress, taken once per device (with that
// device current) on the first call there, and only that address is handed
// to kernels.  Every call on a device shares that device's array and leaves
// its contents behind; calls that overlap on one device race.
#include <mutex>

#include "common.h"

namespace ft {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;   // 64 MiB: 8M binary64 element loads
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kNoAllocMaxDevices] = {};

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

// Device address of the current device's scratch array (looked up on the
// first call on that device, then cached).
ft_status noalloc_scratch(double** out) {
    int dev = -1;
    FT_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) {
        set_error("device %d is beyond the %d devices the scratch table covers", dev, kNoAllocMaxDevices);
        return FT_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
            return FT_E_DEVICE;
        }
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return FT_OK;
}

}  // namespace ft

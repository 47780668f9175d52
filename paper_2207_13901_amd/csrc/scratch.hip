// Static device scratch for spl_spmv_noalloc: the tile bounds and carries
// of one merge- or non-zero-split SpMV live in a file-scope device array
// instead of a workspace, so that call allocates nothing.
//
// Each GPU the library runs on holds its own copy of `scratch` (kScratchBytes)
// until the process ends.  Host code never uses the array's name as an
// address: scratch_init looks up the device address of the copy on one
// device (with that device current) and keeps it per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[spl::kScratchBytes];

std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

namespace spl {

hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> hold(g_lock);
    if (g_done[device]) return g_status[device];
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
    }
    g_ptr[device] = ptr;
    g_status[device] = e;
    g_done[device] = true;
    return e;
}

void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> hold(g_lock);
    return g_done[device] && g_status[device] == hipSuccess ? g_ptr[device] : nullptr;
}

}  // namespace spl

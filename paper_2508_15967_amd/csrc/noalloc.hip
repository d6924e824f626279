// Static device scratch for rg_trace_rays_noalloc: callers that cannot
// allocate device memory (code under stream capture, tight serving loops,
// harnesses that forbid hipMalloc) get the per-call scratch of a trace from
// this fixed array instead of a workspace of their own.  Each device the
// library runs on holds its own copy of the array until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is resolved once per device with hipGetSymbolAddress (with
// that device current) and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.hpp"

static __device__ __align__(256) unsigned char scratch[RG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_addr[kMaxDevices] = {};
}  // namespace

namespace rg {

int noalloc_resolve(int device, std::string *err) {
    if (device < 0 || device >= kMaxDevices) {
        *err = "device index out of range for the static scratch table";
        return -1;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_addr[device]) return 0;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess || cur != device) {
        *err = "the device must be current when its static scratch is resolved";
        return -1;
    }
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return -1;
    }
    g_addr[device] = ptr;
    return 0;
}

void *noalloc_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_addr[device];
}

}  // namespace rg

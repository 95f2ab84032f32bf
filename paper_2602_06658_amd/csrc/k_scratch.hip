// The library's fixed scratch array for gw_solve_noalloc: every buffer of
// such a solve is carved from it, so the call allocates no device memory.
// One copy per GPU the library runs on, held until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gw_scratch.h"

// File-scope device array; host code never passes its name to a kernel or a
// copy (in host code the name is a stand-in, not a device address) but the
// per-device address from hipGetSymbolAddress.  Being referenced from host
// code, the static array is given a global symbol in the device code object,
// which the runtime needs to resolve that address.
static __device__ __align__(256) unsigned char scratch[gwr::SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};
bool g_done[MAX_DEVICES] = {};

}  // namespace

namespace gwr {

hipError_t scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_done[device]) return g_err[device];
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device) (void)hipSetDevice(cur);
    g_ptr[device] = e == hipSuccess ? p : nullptr;
    g_err[device] = e;
    g_done[device] = true;
    return e;
}

void* scratch_ptr(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_done[device] ? g_ptr[device] : nullptr;
}

}  // namespace gwr

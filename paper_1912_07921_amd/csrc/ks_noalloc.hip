// The allocation-free H.psi entry point: ks_apply_h with its projector
// scratch (coefficients, chunk partials, hull-row terms) in a static device
// array instead of a workspace, for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  Every call on a device shares that device's array:
// calls that overlap on one GPU race.
#include "../../include/ks.h"
#include "ks_internal.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device

// Device copy of the scratch; its host-side name is not a device address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, looked up once per device
// with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_looked[kMaxDevices];
hipError_t g_rc[kMaxDevices];
void *g_ptr[kMaxDevices];

int scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_looked[dev]) {
        void *p = nullptr;
        g_rc[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[dev] = g_rc[dev] == hipSuccess ? p : nullptr;
        g_looked[dev] = true;
    }
    if (g_rc[dev] != hipSuccess || !g_ptr[dev]) {
        char msg[160];
        std::snprintf(msg, sizeof msg,
                      "hipGetSymbolAddress of the static scratch on device "
                      "%d: %s", dev, hipGetErrorString(g_rc[dev]));
        return ks::set_error(KS_E_HIP, msg);
    }
    *out = g_ptr[dev];
    return KS_OK;
}

}  // namespace

extern "C" int ks_apply_h_noalloc(ks_grid *g, const void *d_psi,
                                  void *d_hpsi, int k, int s0, int ns,
                                  double t)
{
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return ks::set_error(KS_E_HIP, "hipGetDevice failed");
    }
    if (dev < 0 || dev >= kMaxDevices)
        return ks::set_error(KS_E_UNSUPPORTED, "device index beyond 63");
    void *base = nullptr;
    const int rc = scratch_address(dev, &base);
    if (rc)
        return rc;
    return ks::apply_h_scratch(g, d_psi, d_hpsi, k, s0, ns, t,
                               static_cast<char *>(base), kScratchBytes, dev);
}

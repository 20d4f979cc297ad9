// snrt_static.hip -- sn_plan_bind_static: a plan bound to a scratch area that
// the library keeps in device memory itself, for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid allocation). Everything else about the plan is unchanged: the
// same kernels run on the same layout, only the scratch base differs.
//
// The area is one file-scope device array per GPU the library is loaded on
// (each device holds its own copy until the process ends). Host code never
// passes the array's name to a kernel or a copy: on the host it names a
// stand-in, not device memory. The device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and is
// the only handle host code uses.
#include <hip/hip_runtime.h>

#include <mutex>

#include "sn_host.h"
#include "snrt.h"

static __device__ __align__(256) char scratch[SN_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};            // device address of `scratch` per device
const sn_plan* g_owner[kMaxDevices] = {};  // plan bound to it per device, or NULL

}  // namespace

// Called when a plan bound to the area of device `dev` is destroyed or bound
// to other scratch: it no longer holds the area.
void snh::release_static_scratch(const sn_plan* P, int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_owner[dev] == P) g_owner[dev] = nullptr;
}

extern "C" sn_status sn_plan_bind_static(sn_plan* P, void* psi_a, void* psi_b) {
    if (!P || !psi_a || !psi_b) return snh::fail(SN_ERR_INVALID, "NULL argument");
    if (P->scratch_bytes > (size_t)SN_STATIC_SCRATCH_BYTES)
        return snh::fail(SN_ERR_UNSUPPORTED,
                         "the plan needs %zu bytes of scratch; the library's static area holds %d "
                         "(SN_STATIC_SCRATCH_BYTES): bind caller-owned scratch with sn_plan_bind",
                         P->scratch_bytes, (int)SN_STATIC_SCRATCH_BYTES);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return snh::fail(SN_ERR_UNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_owner[dev] && g_owner[dev] != P)
        return snh::fail(SN_ERR_BUSY,
                         "the static scratch of device %d is bound to another plan; destroy that plan or "
                         "bind it to other scratch first",
                         dev);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return snh::hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return snh::fail(SN_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_ptr[dev] = p;
    }
    const int old_dev = P->static_dev;
    const sn_status st = snh::bind_buffers(P, psi_a, psi_b, g_ptr[dev]);
    if (st != SN_OK) return st;
    if (old_dev >= 0 && old_dev < kMaxDevices && old_dev != dev && g_owner[old_dev] == P) g_owner[old_dev] = nullptr;
    g_owner[dev] = P;
    P->static_dev = dev;
    return SN_OK;
}

// Allocation-free twisted-mass operator: tmh_qtm_apply with its intermediate
// even field taken from a fixed device array instead of the handle's
// scratch, for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array: every GPU the library runs on
// holds its own copy, at its own address, from the load of this code object
// until the process ends.  In host code the name is only a stand-in for the
// symbol, so the host never passes it to a kernel: the device address of the
// current GPU's copy is queried once per device with hipGetSymbolAddress
// (at tmh_lattice_create, or at the first call on a device if that query
// failed) and kept per device; kernels get that address as an argument.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/tmhop.h"
#include "api_internal.h"

static __device__ __align__(256) unsigned char scratch[TMH_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` per device, null until queried

}  // namespace

namespace tmh_api {

tmh_status noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return TMH_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[device]) return TMH_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return TMH_ERR_HIP;
    }
    g_scratch[device] = p;
    return TMH_OK;
}

}  // namespace tmh_api

namespace {

tmh_status scratch_of(int device, void** out) {
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (device >= 0 && device < kMaxDevices && g_scratch[device]) {
            *out = g_scratch[device];
            return TMH_OK;
        }
    }
    const tmh_status st = tmh_api::noalloc_setup(device);
    if (st != TMH_OK) return st;
    std::lock_guard<std::mutex> lock(g_mu);
    *out = g_scratch[device];
    return TMH_OK;
}

}  // namespace

extern "C" tmh_status tmh_qtm_apply_noalloc(tmh_lattice* l, void* out, const void* gauge, const void* in,
                                            double kappa, double mu, const double theta[4], int sign,
                                            tmh_prec prec) {
    const tmh_status chk = tmh_api::qtm_check(l, out, gauge, in, kappa, mu, theta, sign, prec);
    if (chk != TMH_OK) return chk;
    if (tmh_api::lattice_spinor_bytes(l, prec) > (size_t)TMH_NOALLOC_MAX_BYTES) return TMH_ERR_SCRATCH;
    const int dev = tmh_api::lattice_device(l);
    int old = -1;
    if (hipGetDevice(&old) != hipSuccess) return TMH_ERR_HIP;
    if (old != dev && hipSetDevice(dev) != hipSuccess) return TMH_ERR_HIP;
    void* te = nullptr;
    // The even field is written in full (every site below the half volume)
    // by the first hop before the second reads it, so what an earlier call
    // left in the array needs no clearing.
    tmh_status st = scratch_of(dev, &te);
    if (st == TMH_OK) st = tmh_api::qtm_run(l, out, gauge, in, te, kappa, mu, theta, sign, prec, false);
    if (old != dev) (void)hipSetDevice(old);
    return st;
}

// lbm_moments_device_noalloc (include/lbm2p.h): the moments read-out of
// lbm_moments_device with its staging buffer in device memory the library
// holds from load time, so that the call allocates nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbm2p.h"
#include "domain.hpp"
#include "launch.hpp"

using namespace lbm;

namespace {

// Staging planes rho, ux, uy of at most kScratchNodes nodes each (48 MiB),
// held on every GPU the library runs on until the process ends.  Host code
// never uses this name as an address: a GPU's copy is reached through the
// pointer hipGetSymbolAddress returns with that GPU current.
constexpr long long kScratchNodes = 1LL << 21;
__device__ __align__(256) double scratch[3 * kScratchNodes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device `dev` (looked up
// once per device), or null.
double* scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_scratch[dev] = static_cast<double*>(p);
    }
    return g_scratch[dev];
}

int moments_into(lbm_domain* d, double* sp, double* rho, double* ux, double* uy) {
    const size_t nn = (size_t)d->nx * d->ny;
    Ctx c = domain_ctx(d);
    c.mom_out = sp;
    // the pre-collision moments at t are pulled from f*(t - 1)
    const void* src = moments_source(d);
    if (d->storage == LBM_STORE_F64) launch_main_f64(c, src, nullptr, true);
    else launch_main_f32(c, src, nullptr, true);
    double* outs[3] = {rho, ux, uy};
    for (int k = 0; k < 3; ++k)
        if (outs[k] && hipMemcpyAsync(outs[k], sp + k * nn, nn * sizeof(double),
                                      hipMemcpyDeviceToDevice, d->stream) != hipSuccess)
            return LBM_EDEVICE;
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

}  // namespace

extern "C" int lbm_moments_device_noalloc(lbm_domain* d, double* rho, double* ux, double* uy) {
    if (!d) return LBM_EINVAL;
    if ((long long)d->nx * d->ny > kScratchNodes) return LBM_EINVAL;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return LBM_EDEVICE;
    if (prev != d->device && hipSetDevice(d->device) != hipSuccess) return LBM_EDEVICE;
    double* sp = scratch_on(d->device);
    const int rc = sp ? moments_into(d, sp, rho, ux, uy) : LBM_EDEVICE;
    if (prev != d->device) (void)hipSetDevice(prev);
    return rc;
}

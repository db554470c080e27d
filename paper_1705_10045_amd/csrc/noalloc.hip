// lbm_moments_device_noalloc (include/lbm_mi355x.h): the moments of lbm_moments_device for
// callers that cannot allocate device memory.  The scratch of the two moment kernels lives in a
// fixed file-scope device array that the code object reserves on every GPU the library runs on,
// for the life of the process, so no call allocates or frees anything.
//
// In host code the array's name is only a host-side handle of the symbol.  Its device address
// is looked up once per device, with that device current, on the entry point's first call
// there, and only that address is handed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbm_mi355x.h"
#include "kernels.hpp"
#include "sim.hpp"

namespace lbm {
namespace {

constexpr size_t kStaticScratchBytes = size_t(128) << 20;
// the moment kernels keep rho, j, E, T and Phi: 7 doubles per node
constexpr long long kNoallocMaxNodes = (long long)(kStaticScratchBytes / (7 * sizeof(double)));

static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_addr[kMaxDevices] = {};

// This device's address of `scratch` (the device must be current); null with the message set
// on failure.
double* scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) {
        set_error("device %d is beyond the %d devices the fixed scratch covers", device, kMaxDevices);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
            return nullptr;
        }
        g_addr[device] = (double*)ptr;
    }
    return g_addr[device];
}

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_moments_device_noalloc(lbm_sim* s, double* rho, double* u_star, double* E,
                                                 double* T)
{
    clear_error();
    if (!s) { set_error("simulation is NULL"); return LBM_EINVAL; }
    if (s->n > kNoallocMaxNodes) {
        set_error("lbm_moments_device_noalloc: %lld nodes exceed the fixed scratch (%zu bytes, at most "
                  "%lld nodes); use lbm_moments_device", s->n, kStaticScratchBytes, kNoallocMaxNodes);
        return LBM_EINVAL;
    }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    double* scr = scratch_address(s->device);
    if (!scr) return LBM_EDEVICE;
    // the second kernel reads only scratch elements the first one has written in this call, so
    // what an earlier call left there needs no clearing
    const hipError_t e = launch_moments(s->p.lattice, s->p.storage_bytes, s->buf[s->cur], scr, s->p.nx,
                                        s->p.ny, s->p.nz, s->geom.pitch, s->plane, s->phys, s->aux.eos_p,
                                        s->d_err, rho, u_star, E, T, s->stream);
    if (e != hipSuccess) return hip_fail(e, "moments launch");
    return LBM_OK;
}

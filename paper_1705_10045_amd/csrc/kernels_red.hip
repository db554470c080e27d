// The fused step that also forms the totals of the state it writes: the default launch of each
// lattice and storage with the RED instantiation, then the fixed-order sum of the workgroups'
// partial totals.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "step_launch.hpp"

namespace lbm {

hipError_t launch_step_totals(int Q, int storage_bytes, int variant, const void* src, void* dst,
                              const StepGeom& g, const Phys& ph, const StepAux& aux, double* out,
                              hipStream_t st)
{
    using step_launch::launch_step_t;
    hipError_t e = hipErrorNotSupported;
    if (!aux.partials || !out) return hipErrorInvalidValue;
    if (Q == 19 && storage_bytes == 4) {
        if (variant == 0) e = launch_step_t<19, float, float, 32, 16, 512, true, true, false, true>(src, dst, g, ph, aux, st);
        else if (variant == 5) e = launch_step_t<19, float, float, 32, 16, 512, true, true, true, true>(src, dst, g, ph, aux, st);
        // 64 x 8 tiles: on 512 threads (two moment slots for some) the sums fit the registers
        else if (variant == 7) e = launch_step_t<19, float, float, 64, 8, 512, false, true, true, true>(src, dst, g, ph, aux, st);
        else return hipErrorNotSupported;
    } else if (Q == 19 && storage_bytes == 8) {
        if (variant == 0) e = launch_step_t<19, double, double, 32, 8, 512, false, true, false, true>(src, dst, g, ph, aux, st);
        else return hipErrorNotSupported;
    } else if (Q == 9 && storage_bytes == 4) {
        if (variant == 0) e = launch_step_t<9, float, double, 32, 8, 256, true, false, false, true>(src, dst, g, ph, aux, st);
        else if (variant == 2) e = launch_step_t<9, float, double, 64, 8, 512, true, false, false, true>(src, dst, g, ph, aux, st);
        else return hipErrorNotSupported;
    } else if (Q == 9 && storage_bytes == 8) {
        if (variant == 0) e = launch_step_t<9, double, double, 32, 8, 256, false, false, false, true>(src, dst, g, ph, aux, st);
        else return hipErrorNotSupported;
    } else {
        return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return launch_sum_partials(aux.partials, step_workgroups(g), out, st);
}

}  // namespace lbm

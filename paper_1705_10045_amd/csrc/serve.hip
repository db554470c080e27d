// Serving pool (include/lbm_mi355x.h, lbm_pool_*).
#include <hip/hip_runtime.h>

#include "../../include/lbm_mi355x.h"
#include "sim.hpp"

using namespace lbm;

extern "C" {

lbm_status lbm_pool_create(size_t, int, int, void*, lbm_pool** out)
{
    if (out) *out = nullptr;
    set_error("serving pool not available in this build");
    return LBM_EINVAL;
}
lbm_status lbm_pool_submit(lbm_pool*, const lbm_params*, const double*, const double*, const double*,
                           long long, long long*)
{
    set_error("serving pool not available in this build");
    return LBM_EINVAL;
}
lbm_status lbm_pool_run(lbm_pool*) { set_error("serving pool not available"); return LBM_EINVAL; }
lbm_status lbm_pool_poll(lbm_pool*, long long, int*, lbm_status*) { set_error("serving pool not available"); return LBM_EINVAL; }
lbm_status lbm_pool_collect(lbm_pool*, long long, double*, double*, double*, double*) { set_error("serving pool not available"); return LBM_EINVAL; }
lbm_status lbm_pool_stats(const lbm_pool*, long long*) { set_error("serving pool not available"); return LBM_EINVAL; }
lbm_status lbm_pool_destroy(lbm_pool*) { return LBM_OK; }

}  // extern "C"

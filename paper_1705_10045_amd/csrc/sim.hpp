// Internal state of one simulation behind the opaque lbm_sim handle.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/lbm_mi355x.h"
#include "kernels.hpp"
#include "physics.hpp"

struct lbm_sim {
    lbm_params p;
    lbm::Phys phys;
    lbm::StepGeom geom;
    lbm::StepAux aux;
    long long n = 0, plane = 0;
    int device = 0;
    int cus = 256;                       // compute units of the device
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* buf[2] = {nullptr, nullptr};  // population buffers; buf[cur] holds the current state
    int cur = 0;
    long long step = 0;
    int* d_err = nullptr;
    double* d_table = nullptr;
    double* d_partials = nullptr;        // partial sums of lbm_reduce
    double* d_step_partials = nullptr;   // per-workgroup totals of lbm_step_reduce's last step
    long long step_partials_len = 0;     // doubles held by d_step_partials
    double* d_scratch = nullptr;         // moment scratch (7n doubles), allocated on first use
    double* d_eos_p = nullptr;           // tabulated EOS: reduced pressures and band per row
    double* d_eos_coex = nullptr;
    int red_blocks = 1;
    int tile_x = 0, tile_y = 0;
    int variant = 0;                     // tile shape of the fused step (see step_tile)
};

namespace lbm {
void set_error(const char* fmt, ...);
void clear_error();
lbm_status hip_fail(hipError_t e, const char* what);
// makes `device` current; LBM_EDEVICE with the message set if that fails
lbm_status use_device(int device);
bool host_band_limits(double Tr, double& rv, double& rl);
Phys make_phys(const lbm_params& p);
long long padded_plane(long long n);
long long plane_elements(const lbm_params& p);
size_t state_bytes(const lbm_params& p);
lbm_status validate_params(const lbm_params* p);
lbm_status validate_fields(const lbm_params& p, const double* rho0, const double* u0, const double* T0);
}  // namespace lbm

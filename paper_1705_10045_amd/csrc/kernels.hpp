// Launch interface between the host library and the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "physics.hpp"

namespace lbm {

// Geometry of one fused step launch.
struct StepGeom {
    int nx, ny, nz;
    long long plane;        // elements between consecutive population planes
    int ntx, nty;           // tiles along x and y
    int chunk;              // z planes per workgroup
    int nchunks;
    int resident;           // workgroups the GPU holds at once (one round), 0 if unknown
};

// Read-only tables and the error word shared by every step launch of a simulation.
struct StepAux {
    const double* __restrict__ maxwell;  // band-limit table (reduced densities)
    double tab_s0, tab_inv_ds;
    int* err;                            // device error word (atomicOr)
    const double* __restrict__ eos_p;    // tabulated EOS (Phys::eos = 1): reduced pressures
    const double* __restrict__ eos_coex; // and its coexistence band per row
};

int step_variants(int Q, int storage_bytes);
void step_tile(int Q, int storage_bytes, int variant, int& tx, int& ty, int& per_cu);
hipError_t launch_step(int Q, int storage_bytes, int variant, const void* src, void* dst,
                       const StepGeom& g, const Phys& ph, const StepAux& aux, hipStream_t st);
hipError_t launch_init(int Q, int storage_bytes, void* buf, const double* rho0, const double* u0,
                       const double* T0, int nx, int ny, int nz, long long plane, double c_v,
                       int walls, hipStream_t st);
hipError_t launch_moments(int Q, int storage_bytes, const void* buf, double* scratch, int nx, int ny,
                          int nz, long long plane, const Phys& ph, const double* eos_p, int* err,
                          double* rho, double* us, double* E, double* T, hipStream_t st);
int reduce_blocks(long long n);
hipError_t launch_reduce(int Q, int storage_bytes, const void* buf, long long n, long long plane,
                         double* partials, int nblocks, double* out, hipStream_t st);

}  // namespace lbm

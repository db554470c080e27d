// Launch interface between the host library and the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "physics.hpp"

namespace lbm {

// Geometry of one fused step launch.
struct StepGeom {
    int nx, ny, nz;
    int pitch;              // elements between consecutive x rows of a plane (>= nx)
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
    double* partials;                    // steps that also form the state's totals: 5 per
                                         // workgroup (mass, momentum x/y/z, energy)
};

int step_variants(int Q, int storage_bytes);
void step_tile(int Q, int storage_bytes, int variant, int& tx, int& ty, int& per_cu);
hipError_t launch_step(int Q, int storage_bytes, int variant, const void* src, void* dst,
                       const StepGeom& g, const Phys& ph, const StepAux& aux, hipStream_t st);
// The same step, which also sums the totals of the state it writes (as launch_reduce would sum
// them) into aux.partials, one entry of 5 per workgroup, and then into out[5].  Exists for the
// default variants (0 of every lattice and storage, 2 of D2Q9, 5 of FP32 D3Q19); the others
// return hipErrorNotSupported before launching anything.
hipError_t launch_step_totals(int Q, int storage_bytes, int variant, const void* src, void* dst,
                              const StepGeom& g, const Phys& ph, const StepAux& aux, double* out,
                              hipStream_t st);
// workgroups of one step launch (the entries of aux.partials it writes)
inline long long step_workgroups(const StepGeom& g) { return (long long)g.ntx * g.nty * g.nchunks; }
// Row pitch of the population planes: x rows padded to whole 128-byte lines, so that rows of
// every width start line-aligned (a tile row then loads and stores whole lines).
inline int row_pitch(int nx, int storage_bytes)
{
    const int per_line = 128 / storage_bytes;
    return (nx + per_line - 1) / per_line * per_line;
}
hipError_t launch_init(int Q, int storage_bytes, void* buf, const double* rho0, const double* u0,
                       const double* T0, int nx, int ny, int nz, int pitch, long long plane,
                       double c_v, int walls, hipStream_t st);
hipError_t launch_moments(int Q, int storage_bytes, const void* buf, double* scratch, int nx, int ny,
                          int nz, int pitch, long long plane, const Phys& ph, const double* eos_p,
                          int* err, double* rho, double* us, double* E, double* T, hipStream_t st);
int reduce_blocks(long long n);
// n: buffer elements of one population plane to sum (row padding is zero; a multiple of 16
// bytes' worth of elements, as the row pitch makes it)
hipError_t launch_reduce(int Q, int storage_bytes, const void* buf, long long n, long long plane,
                         double* partials, int nblocks, double* out, hipStream_t st);
// out[0..4] = the sums over nblocks entries of 5 partial totals, in a fixed order
hipError_t launch_sum_partials(const double* partials, long long nblocks, double* out, hipStream_t st);

}  // namespace lbm

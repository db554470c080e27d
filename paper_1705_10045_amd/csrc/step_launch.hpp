// Instantiation choice of the fused step (launch_one, launch_step_t), shared by the library's
// plain step launches and the launches that also form the state's totals.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "step_kernel.hpp"

namespace lbm {
namespace step_launch {

// One buffer resource per buffer needs every byte offset of the two population sets in 32 bits.
inline bool fits_buffer(const StepGeom& g, int Q, int storage_bytes)
{
    return (unsigned long long)g.plane * 2ull * Q * storage_bytes < (1ull << 32);
}


// The periodic instantiation, the one with walls and body force when the parameters ask for
// them, or the one that also carries the tabulated equation of state.
template <int Q, class S, class R, int TX, int TY, int NTH, bool PIPE, bool STASH, int ADDR,
          int NMODE, bool RED>
hipError_t launch_one(const void* src, void* dst, const StepGeom& g, const Phys& ph,
                      const StepAux& aux, hipStream_t st)
{
    const unsigned nblk = (unsigned)(g.ntx * g.nty * g.nchunks);
    const bool ext = ph.walls || ph.g[0] != 0.0 || ph.g[1] != 0.0 || ph.g[2] != 0.0;
    if (ph.eos != 0)
        hipLaunchKernelGGL((k_step<Q, S, R, TX, TY, NTH, PIPE, ADDR, NMODE, STASH, kExtTable, RED>),
                           dim3(nblk), dim3(NTH), 0, st, (const S*)src, (S*)dst, g, ph, aux);
    else if (ext)
        hipLaunchKernelGGL((k_step<Q, S, R, TX, TY, NTH, PIPE, ADDR, NMODE, STASH, kExtWalls, RED>),
                           dim3(nblk), dim3(NTH), 0, st, (const S*)src, (S*)dst, g, ph, aux);
    else
        hipLaunchKernelGGL((k_step<Q, S, R, TX, TY, NTH, PIPE, ADDR, NMODE, STASH, kExtNone, RED>),
                           dim3(nblk), dim3(NTH), 0, st, (const S*)src, (S*)dst, g, ph, aux);
    return hipGetLastError();
}

// Picks the instantiation for the run-time facts: the address form the state allows, the
// tau = 1 collision (no re-read of N_k) when 1/tau is exactly 1 with BGK, and the MRT collision
// (which re-reads N_k, with the load order of tau != 1) when asked for.
//   - FP32 states under 4 GB: one buffer resource per buffer.  Where the variant has the LDS
//     stash, the density prefetch stays on for tau = 1 only (re-reading N_k in the collision
//     leaves no registers for it).
//   - otherwise (FP64, the GLOBAL variant, states of 4 GB and more) global addressing, with the stash
//     where the variant asks for it and without the prefetch: at 512^3 the step is bound by
//     HBM traffic, and the stash saves the collision's second pull of the energy populations
//     (12.6 ms against 14.4 ms for the prefetch alone); not for FP64 with a collision that
//     re-reads N_k (it would spill).
template <int Q, class S, class R, int TX, int TY, int NTH, bool PIPE, bool STASH = false,
          bool GLOBAL = false, bool RED = false>
hipError_t launch_step_t(const void* src, void* dst, const StepGeom& g, const Phys& ph,
                         const StepAux& aux, hipStream_t st)
{
    const bool mrt = ph.collision != 0;
    const bool tau1 = ph.omega == 1.0 && !mrt;
    if constexpr (sizeof(S) == 4 && !GLOBAL) {
        if (fits_buffer(g, Q, 4)) {
            if (tau1) return launch_one<Q, S, R, TX, TY, NTH, PIPE, STASH, kAddrBuf, kTauOne, RED>(src, dst, g, ph, aux, st);
            if (mrt) return launch_one<Q, S, R, TX, TY, NTH, PIPE && !STASH, STASH, kAddrBuf, kMrt, RED>(src, dst, g, ph, aux, st);
            return launch_one<Q, S, R, TX, TY, NTH, PIPE && !STASH, STASH, kAddrBuf, kTauAny, RED>(src, dst, g, ph, aux, st);
        }
    }
    constexpr bool kStashAnyTau = STASH && sizeof(S) == 4;
    if (tau1) return launch_one<Q, S, R, TX, TY, NTH, PIPE && !STASH, STASH, kAddrGlobal, kTauOne, RED>(src, dst, g, ph, aux, st);
    if (mrt) return launch_one<Q, S, R, TX, TY, NTH, PIPE && !kStashAnyTau, kStashAnyTau, kAddrGlobal, kMrt, RED>(src, dst, g, ph, aux, st);
    return launch_one<Q, S, R, TX, TY, NTH, PIPE && !kStashAnyTau, kStashAnyTau, kAddrGlobal, kTauAny, RED>(src, dst, g, ph, aux, st);
}

}  // namespace step_launch
}  // namespace lbm

// Per-node arithmetic of the fused step (sections 2-6), shared by every launch shape of the step
// kernel so that all of them compute bit-identical results.  Each function is the update of one
// node given values the caller gathered (pulled populations, LDS neighbours).
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "physics.hpp"

namespace lbm {

// rho = sum N_k, j = sum c_k N_k, E = sum g_k (eq:hydro, section 4), summed in FP64 in direction
// order (exact for FP32 populations up to the final rounding).  The density sums come first:
// their populations may have been loaded earlier than the energy populations.
template <int Q, class S>
__device__ __forceinline__ void moment_sums(const S* pn, const S* pe, double& dr, double& djx,
                                            double& djy, double& djz, double& dE)
{
    using L = Lattice<Q>;
    dr = 0.0; djx = 0.0; djy = 0.0; djz = 0.0; dE = 0.0;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const double n = double(pn[k]);
        dr += n;
        if (L::cx[k] == 1) djx += n; else if (L::cx[k] == -1) djx -= n;
        if (L::cy[k] == 1) djy += n; else if (L::cy[k] == -1) djy -= n;
        if (L::cz[k] == 1) djz += n; else if (L::cz[k] == -1) djz -= n;
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) dE += double(pe[k]);
}

// T = E / (rho c_V), the van der Waals pressure (section 3) and Phi^2 = rho theta - p, FP64.
// `ok` is false when the node has left the domain of the EOS (Phi^2 <= 0, rho beyond the pole,
// non-finite energy).
__device__ __forceinline__ void eos_phi2(double dr, double dE, const Phys& ph, unsigned flags,
                                         double& dT, double& p, double& phi2, bool& ok)
{
    dT = dE / (dr * ph.c_v);
    const double Te = (flags & kBaro) ? ph.T0_baro : dT;
    p = vdw_pressure(dr, Te, ph);
    phi2 = dr * kTheta - p;
    ok = phi2 > 0.0 && dr * ph.inv_rho_c < 3.0 && dr > 0.0 && dE == dE && dE < 1e30;
}

// Force of section 3 in FP64 (a small difference of Phi^2 values) at index e of a plane of
// row width W:  F = (1/alpha) sum_k G_k Phi_k (A Phi_k + (1 - 2A) Phi(x)) c_k, summed over
// pairs of opposite directions.  pm, p0, pp are the Phi planes at z - 1, z, z + 1.
template <int Q, int W>
__device__ __forceinline__ void force_at(const double* pm, const double* p0, const double* pp,
                                         int e, double A, double inv_alpha, double& Fx,
                                         double& Fy, double& Fz)
{
    using L = Lattice<Q>;
    const double Bm = (1.0 - 2.0 * A) * p0[e];
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
        const int ko = opposite<Q>(k);
        if (ko < k) continue;
        const double* slp = L::cz[k] == 0 ? p0 : (L::cz[k] == 1 ? pp : pm);
        const double* slm = L::cz[k] == 0 ? p0 : (L::cz[k] == 1 ? pm : pp);
        const double a = slp[e + L::cx[k] + W * L::cy[k]];
        const double b = slm[e - L::cx[k] - W * L::cy[k]];
        double d = a * fma(A, a, Bm) - b * fma(A, b, Bm);
        if (force_coef<Q>(k) != 1.0) d *= force_coef<Q>(k);
        if (L::cx[k] == 1) fx += d; else if (L::cx[k] == -1) fx -= d;
        if (L::cy[k] == 1) fy += d; else if (L::cy[k] == -1) fy -= d;
        if (L::cz[k] == 1) fz += d; else if (L::cz[k] == -1) fz -= d;
    }
    Fx = fx * inv_alpha;
    Fy = fy * inv_alpha;
    Fz = fz * inv_alpha;
}

// Energy source dE of sections 4-6 at index e of planes of row width W: pressure work
// -p div u*, conservative conduction with face conductivity c_V chi (rho_i + rho_j)/2, and the
// latent-heat term inside the coexistence band.  r0 and t0 are the rho and T planes of the
// node; rm, tm and rp, tp the values of its neighbours at z - 1 and z + 1 (D = 3).
template <int D, class R, int W>
__device__ __forceinline__ R energy_source(R p, R div, R rho, R T, R rm, const R* r0, R rp,
                                           R tm, const R* t0, R tp, int e, R cond_half,
                                           unsigned flags, const Phys& ph, const StepAux& aux)
{
    R dE = R(0);
    if (flags & kWork) dE -= p * div;
    if (flags & kConduction) {
        const R Tc = t0[e];
        R acc = (rho + r0[e + 1]) * (t0[e + 1] - Tc) - (rho + r0[e - 1]) * (Tc - t0[e - 1]) +
                (rho + r0[e + W]) * (t0[e + W] - Tc) - (rho + r0[e - W]) * (Tc - t0[e - W]);
        if constexpr (D == 3)
            acc += (rho + rp) * (tp - Tc) - (rho + rm) * (Tc - tm);
        dE += cond_half * acc;
    }
    if (flags & kLatent) {
        const double Te = (flags & kBaro) ? ph.T0_baro : double(T);
        double r1, r2;
        if (band_limits(Te * ph.inv_T_c, aux.maxwell, aux.tab_s0, aux.tab_inv_ds, ph.rho_c, r1,
                        r2)) {
            const double rd = double(rho);
            if (rd > r1 && rd < r2) dE -= R(ph.rhoQ / (r2 - r1) * rd * double(div));
        }
    }
    return dE;
}

// Both collisions of one node as linear combinations of the equilibrium polynomials
// P_k(v) = w_k (1 + 3 c.v + 4.5 (c.v)^2 - 1.5 v^2) (eq:feq):
//   N'_k = rho P_k(v) - keepN rho P_k(u) + keepN N_k             (eq:lbe, eq:edm)
//   g'_k = gV P_k(v) + gU P_k(u) + (keepG + dE/E) g_k            (eq:gk, section 4)
// with (gV, gU) = (E, -keepG E) with pseudoforces, (0, E/tau_E) without, v = u + F/rho.
// The moving directions are produced pair by pair of opposite directions (P_k and P_-k share
// the even part of the polynomial); the rest populations close the mass and energy balances in
// FP64 over the values actually stored (the BGK, EDM and pseudoforce increments sum to zero and
// dg(1) sums to dE), so rounding of the lattice weights cannot create mass or energy.
template <int Q, class S, class R, bool WN>
struct NodeCollision {
    R ux, uy, uz, vx, vy, vz, base_u, base_v, rho, keepN, nU, gV, gU, gK;
    double sumN, sumG;

    __device__ __forceinline__ void setup(R rho_, R E, R ux_, R uy_, R uz_, R Fx, R Fy, R Fz,
                                          R inv_rho, R dE, R keepN_, R keepG, R omega_E,
                                          bool pseudo)
    {
        rho = rho_;
        ux = ux_; uy = uy_; uz = uz_;
        vx = ux + Fx * inv_rho; vy = uy + Fy * inv_rho; vz = uz + Fz * inv_rho;
        const R uu = ux * ux + uy * uy + uz * uz;
        const R vv = vx * vx + vy * vy + vz * vz;
        base_u = R(1) - R(1.5) * uu;
        base_v = R(1) - R(1.5) * vv;
        keepN = keepN_;
        nU = -keepN * rho;
        gV = pseudo ? E : R(0);
        gU = pseudo ? -keepG * E : omega_E * E;
        gK = keepG + dE / E;
        sumN = 0.0;
        sumG = 0.0;
    }

    // directions k and opposite<Q>(k) (k < opposite): out = {N'_k, g'_k, N'_-k, g'_-k}
    __device__ __forceinline__ void dir_pair(int k, const R* pk_n, const R* pk_e, S (&out)[4])
    {
        using L = Lattice<Q>;
        const int ko = opposite<Q>(k);
        const R w = R(weight<Q>(k));
        const R cu = R(L::cx[k]) * ux + R(L::cy[k]) * uy + R(L::cz[k]) * uz;
        const R cv = R(L::cx[k]) * vx + R(L::cy[k]) * vy + R(L::cz[k]) * vz;
        const R eu = fma(R(4.5) * w, cu * cu, w * base_u), ou = R(3) * w * cu;
        const R ev = fma(R(4.5) * w, cv * cv, w * base_v), ov = R(3) * w * cv;
        const R Pu[2] = {eu + ou, eu - ou}, Pv[2] = {ev + ov, ev - ov};
        const int kk[2] = {k, ko};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = kk[h];
            R nn = rho * Pv[h];
            if constexpr (WN) nn = fma(keepN, pk_n[q], fma(nU, Pu[h], nn));
            const R gn = fma(gK, pk_e[q], fma(gU, Pu[h], gV * Pv[h]));
            const S nn_s = S(nn), gn_s = S(gn);
            sumN += double(nn_s);
            sumG += double(gn_s);
            out[2 * h] = nn_s;
            out[2 * h + 1] = gn_s;
        }
    }

    // rest populations {N'_0, g'_0}, after every dir_pair
    __device__ __forceinline__ void rest(double rho_d, double E_d, R dE, S& n0, S& g0) const
    {
        n0 = S(rho_d - sumN);
        g0 = S(E_d + double(dE) - sumG);
    }
};

}  // namespace lbm

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

// T = E / (rho c_V), the pressure (section 3: the van der Waals EOS, or with TABLE the
// tabulated one) and Phi^2 = rho theta - p, FP64.  `ok` is false when the node has left the
// domain of the EOS (Phi^2 <= 0, rho beyond the pole or the table, non-finite energy).
template <bool TABLE>
__device__ __forceinline__ void eos_phi2(double dr, double dE, const Phys& ph, unsigned flags,
                                         const StepAux& aux, double& dT, double& p, double& phi2,
                                         bool& ok)
{
    dT = dE / (dr * ph.c_v);
    const double Te = (flags & kBaro) ? ph.T0_baro : dT;
    bool inside = true;
    if constexpr (TABLE)
        p = ph.p_c * table_pressure(dr * ph.inv_rho_c, Te * ph.inv_T_c, ph, aux.eos_p, inside);
    else
        p = vdw_pressure(dr, Te, ph);
    phi2 = dr * kTheta - p;
    ok = inside && phi2 > 0.0 && dr * ph.inv_rho_c < 3.0 && dr > 0.0 && dE == dE && dE < 1e30;
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
template <int D, class R, int W, bool TABLE = false>
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
        bool band;
        if constexpr (TABLE)
            band = table_band(Te * ph.inv_T_c, ph, aux.eos_coex, r1, r2);
        else
            band = band_limits(Te * ph.inv_T_c, aux.maxwell, aux.tab_s0, aux.tab_inv_ds, ph.rho_c, r1, r2);
        if (band) {
            const double rd = double(rho);
            if (rd > r1 && rd < r2) dE -= R(ph.rhoQ / (r2 - r1) * rd * double(div));
        }
    }
    return dE;
}

// Multiple-relaxation-time collision of N_k (section 2 names it beside BGK) on the orthogonal
// moment bases of Lallemand and Luo 2000 (D2Q9) and d'Humieres et al. 2002 (D3Q19), written as
// polynomials of the velocity.  The BGK form relaxes every non-conserved moment at omega, so
// only the moments outside the shear group need a term of their own, with (s_i - omega):
// D2Q9 e, eps, q_x, q_y; D3Q19 e, eps, q_x, q_y, q_z, pi_xx, pi_ww, m_x, m_y, m_z.
template <int Q>
struct MrtRows;
template <>
struct MrtRows<9> {
    static constexpr int N = 4;
    static constexpr int id[4] = {1, 2, 4, 6};
};
template <>
struct MrtRows<19> {
    static constexpr int N = 10;
    static constexpr int id[10] = {1, 2, 4, 6, 8, 10, 12, 16, 17, 18};
};

// Row i of the basis at direction k (rows of MrtRows only).
template <int Q>
__host__ __device__ constexpr double mrt_row(int i, int k)
{
    using L = Lattice<Q>;
    const double x = L::cx[k], y = L::cy[k], z = L::cz[k];
    const double c2 = x * x + y * y + z * z;
    if (Q == 9) {
        switch (i) {
        case 1: return 3.0 * c2 - 4.0;                         // e
        case 2: return 4.5 * c2 * c2 - 10.5 * c2 + 4.0;        // eps
        case 4: return (3.0 * c2 - 5.0) * x;                   // q_x
        case 6: return (3.0 * c2 - 5.0) * y;                   // q_y
        default: return 0.0;
        }
    }
    switch (i) {
    case 1: return 19.0 * c2 - 30.0;                              // e
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;     // eps
    case 4: return (5.0 * c2 - 9.0) * x;                          // q_x
    case 6: return (5.0 * c2 - 9.0) * y;                          // q_y
    case 8: return (5.0 * c2 - 9.0) * z;                          // q_z
    case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);        // pi_xx
    case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);           // pi_ww
    case 16: return (y * y - z * z) * x;                          // m_x
    case 17: return (z * z - x * x) * y;                          // m_y
    case 18: return (x * x - y * y) * z;                          // m_z
    default: return 0.0;
    }
}

// Rate group of row i: 0 e (s_e), 1 eps and pi (s_eps), 2 q (s_q), 3 m (s_m).
__host__ __device__ constexpr int mrt_group(int i)
{
    return i == 1 ? 0 : (i == 2 || i == 10 || i == 12) ? 1 : (i == 4 || i == 6 || i == 8) ? 2 : 3;
}

template <int Q>
__host__ __device__ constexpr double mrt_norm2(int i)
{
    double s = 0.0;
    for (int k = 0; k < Q; ++k) s += mrt_row<Q>(i, k) * mrt_row<Q>(i, k);
    return s;
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
// With MRT (which re-reads N_k like any tau != 1) the moving N'_k also lose
// sum_i am_i M_ik over the rows of MrtRows, am_i = (s_i - omega) m_i / |M_i|^2 with m_i the
// row's moment of N - rho P(u); those terms sum to zero over k, so the rest population still
// closes the mass balance.
template <int Q, class S, class R, bool WN, bool MRT = false>
struct NodeCollision {
    static_assert(!MRT || WN, "the MRT collision reads N_k");
    static constexpr int NG = MRT ? MrtRows<Q>::N : 1;
    R ux, uy, uz, vx, vy, vz, base_u, base_v, rho, keepN, nU, gV, gU, gK;
    R am[NG];
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

    // MRT: the rows' moments of the non-equilibrium part f_k = N_k - rho P_k(u) over the moving
    // directions; f_0 = -sum_{k>0} f_k, since both N and rho P(u) sum to rho, so each row
    // enters with M_ik - M_i0.  Call after setup.
    __device__ __forceinline__ void mrt_prepare(const R* pk_n, const Phys& ph)
    {
        if constexpr (MRT) {
            using L = Lattice<Q>;
            using G = MrtRows<Q>;
            R m[G::N];
#pragma unroll
            for (int i = 0; i < G::N; ++i) m[i] = R(0);
#pragma unroll
            for (int k = 1; k < Q; ++k) {
                const R w = R(weight<Q>(k));
                const R cu = R(L::cx[k]) * ux + R(L::cy[k]) * uy + R(L::cz[k]) * uz;
                const R P = fma(R(4.5) * w, cu * cu, w * base_u) + R(3) * w * cu;
                const R f = fma(-rho, P, pk_n[k]);
#pragma unroll
                for (int i = 0; i < G::N; ++i) {
                    const double coef = mrt_row<Q>(G::id[i], k) - mrt_row<Q>(G::id[i], 0);
                    if (coef != 0.0) m[i] = fma(R(coef), f, m[i]);
                }
            }
            const R d[4] = {R(ph.mrt_de), R(ph.mrt_deps), R(ph.mrt_dq), R(ph.mrt_dm)};
#pragma unroll
            for (int i = 0; i < G::N; ++i)
                am[i] = d[mrt_group(G::id[i])] * m[i] * R(1.0 / mrt_norm2<Q>(G::id[i]));
        }
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
            if constexpr (MRT) {
#pragma unroll
                for (int i = 0; i < NG; ++i) {
                    const double coef = mrt_row<Q>(MrtRows<Q>::id[i], q);
                    if (coef != 0.0) nn = fma(R(-coef), am[i], nn);
                }
            }
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

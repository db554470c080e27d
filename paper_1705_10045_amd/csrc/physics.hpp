// Node-local physics of the thermal multiphase LBM, shared by all kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm {

constexpr double kTheta = 1.0 / 3.0;          // (h/dt)^2 / 3 with h = dt = 1 (section 2)
constexpr double kLatentTmin = 0.4;           // reduced-temperature window of the latent band
constexpr double kLatentTmax = 0.999;
constexpr int kMaxwellPoints = 4096;          // table nodes, uniform in s = sqrt(1 - T~)

// Parameters of one simulation as the kernels see them (passed by value).
struct Phys {
    double omega, omega_E;        // 1/tau, 1/tau_E
    double A, inv_alpha;          // force mixing (section 3), 1/alpha of the lattice
    double rho_c, inv_rho_c, inv_T_c, p_c;
    double c_v, inv_c_v;
    double cond_half;             // c_v chi / 2: face conductivity per unit (rho_i + rho_j)
    double rhoQ;
    double T0_baro;
    unsigned flags;
    int walls;                    // 1: no-slip walls normal to z below z = 0 and above nz - 1
    unsigned wall_heat;           // kWallTBottom | kWallTTop: wall faces held at a temperature
    double T_bottom, T_top;
    double g[3];                  // body force per unit mass
    // collision of N_k: 0 BGK; 1 multiple relaxation times, with the shear moments at omega
    // and the other non-conserved groups at their own rates, stored as (rate - omega) for the
    // energy e, the energy square and fourth-order moments, the energy fluxes q and (D3Q19)
    // the third-order moments m
    int collision;
    double mrt_de, mrt_deps, mrt_dq, mrt_dm;
    // equation of state: 0 the reduced van der Waals EOS; 1 a table of reduced pressure on a
    // uniform grid (section 3 allows tabulated EOS of real fluids), see table_pressure
    int eos;
    int tab_nrho, tab_nT;
    double tab_rho_min, tab_rho_max, tab_drho;
    double tab_T_min, tab_T_max, tab_dT;
};

enum : unsigned { kWallTBottom = 1u, kWallTTop = 2u };

enum : unsigned { kWork = 1u, kConduction = 2u, kLatent = 4u, kPseudo = 8u, kBaro = 16u };

// w_k (1 + c.u/theta + (c.u)^2/(2 theta^2) - u^2/(2 theta)), eq:feq without the density.
template <class R>
__device__ __forceinline__ R eq_poly(R w, R cu, R uu)
{
    return w * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu);
}

// Reduced van der Waals pressure in lattice units (section 3), FP64.
__host__ __device__ inline double vdw_pressure(double rho, double T, const Phys& p)
{
    const double rr = rho * p.inv_rho_c;
    const double tr = T * p.inv_T_c;
    return p.p_c * (8.0 * rr * tr / (3.0 - rr) - 3.0 * rr * rr);
}

// Tabulated reduced pressure p~(rr, Tr) (rr = rho/rho_c, Tr = T/T_c): the table holds p~ at
// rho~_i = tab_rho_min + i tab_drho and T~_j = tab_T_min + j tab_dT as tab[j * tab_nrho + i].
// Cubic Lagrange interpolation in rho~ through the four grid densities around the point (the
// stencil shifted inward next to the grid's ends), linear in T~ between the two rows around it.
// `inside` is false (and 0 returned) outside the grid: the node has left the EOS domain.
__host__ __device__ inline double table_pressure(double rr, double Tr, const Phys& p,
                                                 const double* __restrict__ tab, bool& inside)
{
    inside = rr >= p.tab_rho_min && rr <= p.tab_rho_max && Tr >= p.tab_T_min && Tr <= p.tab_T_max;
    if (!inside) return 0.0;
    int j = (int)floor((Tr - p.tab_T_min) / p.tab_dT);
    j = j > p.tab_nT - 2 ? p.tab_nT - 2 : (j < 0 ? 0 : j);
    const double u = (Tr - (p.tab_T_min + j * p.tab_dT)) / p.tab_dT;
    int i0 = (int)floor((rr - p.tab_rho_min) / p.tab_drho) - 1;
    i0 = i0 > p.tab_nrho - 4 ? p.tab_nrho - 4 : (i0 < 0 ? 0 : i0);
    const double t = (rr - (p.tab_rho_min + i0 * p.tab_drho)) / p.tab_drho;
    // Lagrange basis on grid nodes i0 .. i0 + 3 at offset t from node i0
    const double w0 = -(t - 1.0) * (t - 2.0) * (t - 3.0) / 6.0;
    const double w1 = t * (t - 2.0) * (t - 3.0) / 2.0;
    const double w2 = -t * (t - 1.0) * (t - 3.0) / 2.0;
    const double w3 = t * (t - 1.0) * (t - 2.0) / 6.0;
    const double* a = tab + (long long)j * p.tab_nrho + i0;
    const double* b = a + p.tab_nrho;
    const double lo = w0 * a[0] + w1 * a[1] + w2 * a[2] + w3 * a[3];
    const double hi = w0 * b[0] + w1 * b[1] + w2 * b[2] + w3 * b[3];
    return (1.0 - u) * lo + u * hi;
}

// Coexistence band (rho_1, rho_2) of a tabulated EOS at reduced temperature Tr, linear in T~
// between the rows of coex (coex[2j] <= coex[2j + 1], reduced densities).  False outside the
// table's temperature range.
__host__ __device__ inline bool table_band(double Tr, const Phys& p,
                                           const double* __restrict__ coex, double& r1,
                                           double& r2)
{
    if (!(Tr >= p.tab_T_min && Tr <= p.tab_T_max)) return false;
    int j = (int)floor((Tr - p.tab_T_min) / p.tab_dT);
    j = j > p.tab_nT - 2 ? p.tab_nT - 2 : (j < 0 ? 0 : j);
    const double u = (Tr - (p.tab_T_min + j * p.tab_dT)) / p.tab_dT;
    r1 = p.rho_c * ((1.0 - u) * coex[2 * j] + u * coex[2 * j + 2]);
    r2 = p.rho_c * ((1.0 - u) * coex[2 * j + 1] + u * coex[2 * j + 3]);
    return true;
}

// Coexistence densities (rho_1, rho_2) of the band at reduced temperature Tr, cubic Lagrange
// interpolation in s = sqrt(1 - Tr) on the FP64 Maxwell table (tab[2i] vapour, tab[2i+1]
// liquid, reduced densities).  Returns false outside [kLatentTmin, kLatentTmax).
__device__ __forceinline__ bool band_limits(double Tr, const double* __restrict__ tab,
                                            double s0, double inv_ds, double rho_c,
                                            double& r1, double& r2)
{
    if (!(Tr >= kLatentTmin && Tr < kLatentTmax)) return false;
    const double pos = (sqrt(1.0 - Tr) - s0) * inv_ds;
    int j = (int)pos;
    j = j < 1 ? 1 : (j > kMaxwellPoints - 3 ? kMaxwellPoints - 3 : j);
    const double t = pos - j;
    // Lagrange basis on nodes j-1, j, j+1, j+2 at offset t from node j
    const double l0 = -t * (t - 1.0) * (t - 2.0) / 6.0;
    const double l1 = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
    const double l2 = -(t + 1.0) * t * (t - 2.0) / 2.0;
    const double l3 = (t + 1.0) * t * (t - 1.0) / 6.0;
    const double* q = tab + 2 * (j - 1);
    r1 = rho_c * (l0 * q[0] + l1 * q[2] + l2 * q[4] + l3 * q[6]);
    r2 = rho_c * (l0 * q[1] + l1 * q[3] + l2 * q[5] + l3 * q[7]);
    return true;
}

__host__ __device__ inline int wrap_index(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

}  // namespace lbm

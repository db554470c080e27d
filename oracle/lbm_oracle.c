/*
 * FP64 CPU oracle of the thermal multiphase lattice Boltzmann method
 * (Kupershtokh, Medvedev, Gribanov, arXiv:1705.10045).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product library.  It is a
 * plain, slow, whole-field implementation: one pass per physical term, in the
 * order the paper applies them, FP64 throughout, plain sums in index order,
 * push streaming on node-major (AoS) populations.
 *
 * One time step t -> t+1 (h = dt = 1, theta = 1/3):
 *   1. moments (eq:hydro, E = sum g_k, E = rho c_v T)               section 2, 4
 *   2. van der Waals pressure and Phi = sqrt(-U), U = p - rho theta   section 3
 *   3. isotropic force from Phi                                       section 3
 *   4. du = F/rho, u* = u + du/2                                      eq:edm, eq:ustar
 *   5. energy source dE = work + conduction + latent                 section 4, 5, 6.2
 *   6. BGK collision + EDM forcing of N_k                             eq:lbe, eq:edm
 *   7. BGK collision + dg(1) + pseudoforce dg(2) of g_k               eq:gk, section 4
 *   8. streaming to x + c_k, periodic                                 eq:lbe, eq:gk
 *
 * Lattices: D1Q3 (ny = nz = 1), D2Q9 (nz = 1) and D3Q19, with the force coefficients
 * G_k of section 3 (neighbours along the axes and, for D2Q9/D3Q19, the diagonals).
 *
 * Walls and body force (not in the paper; readings listed in the design notes): optional
 * no-slip walls normal to z halfway between planes (bounce-back of N and g in step 8; mirror
 * ghosts beyond them in steps 3 and 5) and F += rho g in step 3.
 *
 * Readings where the paper is not explicit (all listed in the design notes):
 *   - critical values rho_c, T_c, p_c are parameters in lattice units;
 *   - the multi-dimensional pressure work uses the central difference of
 *     section 6.2 along every axis; conduction is the conservative face-flux
 *     form with the arithmetic-mean face conductivity;
 *   - p, u*, T and rho in dE are all taken at time t (before collision);
 *   - dg(1) uses the pre-collision g_k and E = sum g_k;
 *   - g^eq and dg(2) use u from eq:hydro and the same du as the N_k;
 *   - the latent source uses rho_liq*Q as one constant (rhoQ) and is active
 *     where 0.4 <= T~ < 0.999 and rho_1(T) < rho < rho_2(T) strictly, with
 *     rho_1, rho_2 the Maxwell coexistence densities at the EOS temperature;
 *   - a tabulated EOS (section 3 allows them for real fluids) is interpolated
 *     cubically in rho~ and linearly in T~ on its uniform grid, and carries its
 *     own coexistence band for the latent source.
 *
 * Collision of N_k: BGK (eq:lbe) or, as section 2 also allows, multiple relaxation times on an
 * orthogonal moment basis (MRT), with the EDM increment added in either case.
 *
 * Every function is pinned by the CPU test suite against closed forms, exact
 * invariants, independent spectral/quadrature computations or values printed in
 * the paper; none is "parity unpinned".
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define THETA (1.0 / 3.0)          /* (h/dt)^2/3 with h = dt = 1, section 2 */
#define LATENT_TMIN 0.4            /* reduced-temperature window of the latent source */
#define LATENT_TMAX 0.999

/* Moment groups of the multiple-relaxation-time collision: which rate relaxes moment i. */
enum { MG_CONSERVED = 0, MG_SHEAR = 1, MG_BULK = 2, MG_EPS = 3, MG_Q = 4, MG_M = 5 };

typedef struct {
    int Q, D;
    int c[19][3];
    int opp[19];       /* direction with c[opp[k]] = -c[k] */
    double w[19];
    double G[19];
    double alpha;
    /* MRT moment basis (D2Q9 and D3Q19): row i of M holds moment i's polynomial evaluated at
     * every velocity; rows are orthogonal, M2[i] = sum_k M[i][k]^2; grp[i] is its group. */
    double M[19][19];
    double M2[19];
    int grp[19];
} lattice;

/* Orthogonal moment bases of the MRT collision named in section 2 (Lallemand and Luo 2000 for
 * D2Q9, d'Humieres et al. 2002 for D3Q19), written as polynomials of the velocity: density,
 * energy e, energy square eps, momentum j, energy flux q, the traceless stresses (shear),
 * and for D3Q19 the fourth-order pi and third-order m moments. */
static void mrt_basis(lattice* L)
{
    for (int k = 0; k < L->Q; ++k) {
        const double x = L->c[k][0], y = L->c[k][1], z = L->c[k][2];
        const double c2 = x * x + y * y + z * z;
        double r[19];
        if (L->Q == 9) {
            const double v[9] = {1.0, 3.0 * c2 - 4.0, 4.5 * c2 * c2 - 10.5 * c2 + 4.0,
                                 x, (3.0 * c2 - 5.0) * x, y, (3.0 * c2 - 5.0) * y,
                                 x * x - y * y, x * y};
            memcpy(r, v, sizeof(v));
        } else {
            const double v[19] = {1.0, 19.0 * c2 - 30.0, (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0,
                                  x, (5.0 * c2 - 9.0) * x, y, (5.0 * c2 - 9.0) * y,
                                  z, (5.0 * c2 - 9.0) * z,
                                  3.0 * x * x - c2, (3.0 * c2 - 5.0) * (3.0 * x * x - c2),
                                  y * y - z * z, (3.0 * c2 - 5.0) * (y * y - z * z),
                                  x * y, y * z, x * z,
                                  (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z};
            memcpy(r, v, sizeof(v));
        }
        for (int i = 0; i < L->Q; ++i) L->M[i][k] = r[i];
    }
    static const int g9[9] = {MG_CONSERVED, MG_BULK, MG_EPS, MG_CONSERVED, MG_Q, MG_CONSERVED,
                              MG_Q, MG_SHEAR, MG_SHEAR};
    static const int g19[19] = {MG_CONSERVED, MG_BULK, MG_EPS, MG_CONSERVED, MG_Q, MG_CONSERVED,
                                MG_Q, MG_CONSERVED, MG_Q, MG_SHEAR, MG_EPS, MG_SHEAR, MG_EPS,
                                MG_SHEAR, MG_SHEAR, MG_SHEAR, MG_M, MG_M, MG_M};
    for (int i = 0; i < L->Q; ++i) {
        L->grp[i] = L->Q == 9 ? g9[i] : g19[i];
        double n2 = 0.0;
        for (int k = 0; k < L->Q; ++k) n2 += L->M[i][k] * L->M[i][k];
        L->M2[i] = n2;
    }
}

/* opp[k]: the direction with the opposite velocity, found by search */
static void find_opposites(lattice* L)
{
    for (int k = 0; k < L->Q; ++k)
        for (int m = 0; m < L->Q; ++m)
            if (L->c[m][0] == -L->c[k][0] && L->c[m][1] == -L->c[k][1] && L->c[m][2] == -L->c[k][2])
                L->opp[k] = m;
}

/* Velocity sets, weights (section 2) and force coefficients G_k, alpha (section 3).
 * Index 0 is the rest particle; then the nearest neighbours, then the next-nearest. */
static int make_lattice(int Q, lattice* L)
{
    memset(L, 0, sizeof(*L));
    L->Q = Q;
    if (Q == 3) {            /* D1Q3: the paper's one-dimensional lattice */
        static const int c3[3][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}};
        L->D = 1;
        for (int k = 0; k < 3; ++k) {
            for (int a = 0; a < 3; ++a) L->c[k][a] = c3[k][a];
            L->w[k] = k == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
            L->G[k] = k == 0 ? 0.0 : 1.0;
        }
        L->alpha = 1.0;
        find_opposites(L);
        return 1;
    }
    if (Q == 9) {
        static const int c9[9][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
                                     {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
        L->D = 2;
        for (int k = 0; k < 9; ++k) {
            for (int a = 0; a < 3; ++a) L->c[k][a] = c9[k][a];
            if (k == 0) { L->w[k] = 4.0 / 9.0; L->G[k] = 0.0; }
            else if (k <= 4) { L->w[k] = 1.0 / 9.0; L->G[k] = 1.0; }
            else { L->w[k] = 1.0 / 36.0; L->G[k] = 0.25; }
        }
        L->alpha = 1.5;
        find_opposites(L);
        mrt_basis(L);
        return 2;
    }
    if (Q == 19) {
        static const int c19[19][3] = {
            {0, 0, 0},
            {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
            {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
            {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
            {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
        L->D = 3;
        for (int k = 0; k < 19; ++k) {
            for (int a = 0; a < 3; ++a) L->c[k][a] = c19[k][a];
            if (k == 0) { L->w[k] = 1.0 / 3.0; L->G[k] = 0.0; }
            else if (k <= 6) { L->w[k] = 1.0 / 18.0; L->G[k] = 1.0; }
            else { L->w[k] = 1.0 / 36.0; L->G[k] = 0.5; }
        }
        L->alpha = 3.0;
        find_opposites(L);
        mrt_basis(L);
        return 3;
    }
    return ORC_EINVAL;
}

int orc_lattice(int Q, int* c, double* w, double* G, double* alpha)
{
    lattice L;
    if (make_lattice(Q, &L) < 0) return ORC_EINVAL;
    for (int k = 0; k < Q; ++k) {
        for (int a = 0; a < 3; ++a) c[3 * k + a] = L.c[k][a];
        w[k] = L.w[k];
        G[k] = L.G[k];
    }
    *alpha = L.alpha;
    return L.D;
}

int orc_mrt_basis(int Q, double* M, double* norm2, int* group)
{
    lattice L;
    if (!(Q == 9 || Q == 19) || make_lattice(Q, &L) < 0) return ORC_EINVAL;
    for (int i = 0; i < Q; ++i) {
        for (int k = 0; k < Q; ++k) M[i * Q + k] = L.M[i][k];
        norm2[i] = L.M2[i];
        group[i] = L.grp[i];
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Van der Waals fluid in reduced variables (section 3)
 * ------------------------------------------------------------------------- */

double orc_vdw_reduced(double rr, double Tr)
{
    return 8.0 * rr * Tr / (3.0 - rr) - 3.0 * rr * rr;
}

/* ---------------------------------------------------------------------------
 * Tabulated equation of state (section 3: tabulated EOS of real fluids).
 * Cubic Lagrange interpolation in rho~ on the four grid points around the point,
 * linear interpolation in T~ between the two rows around it.
 * ------------------------------------------------------------------------- */

/* Value at offset t (in grid steps from node 0) of the cubic through f[0..3] at nodes 0..3. */
static double lagrange4(const double* f, double t)
{
    const double l0 = -(t - 1.0) * (t - 2.0) * (t - 3.0) / 6.0;
    const double l1 = t * (t - 2.0) * (t - 3.0) / 2.0;
    const double l2 = -t * (t - 1.0) * (t - 3.0) / 2.0;
    const double l3 = t * (t - 1.0) * (t - 2.0) / 6.0;
    return l0 * f[0] + l1 * f[1] + l2 * f[2] + l3 * f[3];
}

/* Grid row j and weight u of the second row for reduced temperature Tr; 0 outside. */
static int table_row(const orc_params* p, double Tr, int* j, double* u)
{
    if (!(Tr >= p->eos_T_min && Tr <= p->eos_T_max)) return 0;
    const double dT = (p->eos_T_max - p->eos_T_min) / (p->eos_nT - 1);
    int r = (int)floor((Tr - p->eos_T_min) / dT);
    if (r > p->eos_nT - 2) r = p->eos_nT - 2;
    if (r < 0) r = 0;
    *j = r;
    *u = (Tr - (p->eos_T_min + r * dT)) / dT;
    return 1;
}

double orc_table_reduced(const orc_params* p, double rr, double Tr, int* inside)
{
    int j;
    double u;
    *inside = 0;
    if (!(rr >= p->eos_rho_min && rr <= p->eos_rho_max) || !table_row(p, Tr, &j, &u)) return 0.0;
    const double dr = (p->eos_rho_max - p->eos_rho_min) / (p->eos_nrho - 1);
    /* stencil i0 .. i0+3 with the point between i0+1 and i0+2 where the grid allows */
    int i0 = (int)floor((rr - p->eos_rho_min) / dr) - 1;
    if (i0 < 0) i0 = 0;
    if (i0 > p->eos_nrho - 4) i0 = p->eos_nrho - 4;
    const double t = (rr - (p->eos_rho_min + i0 * dr)) / dr;
    const double lo = lagrange4(p->eos_p + (long)j * p->eos_nrho + i0, t);
    const double hi = lagrange4(p->eos_p + (long)(j + 1) * p->eos_nrho + i0, t);
    *inside = 1;
    return (1.0 - u) * lo + u * hi;
}

/* Coexistence band (reduced rho_1, rho_2) of the tabulated EOS at Tr; 0 outside the table. */
static int table_band(const orc_params* p, double Tr, double* r1, double* r2)
{
    int j;
    double u;
    if (!table_row(p, Tr, &j, &u)) return 0;
    *r1 = (1.0 - u) * p->eos_coex[2 * j] + u * p->eos_coex[2 * j + 2];
    *r2 = (1.0 - u) * p->eos_coex[2 * j + 1] + u * p->eos_coex[2 * j + 3];
    return 1;
}

/* Chemical potential of the reduced vdW fluid up to a T-dependent constant,
 * from d(mu) = dp/rho at fixed T. */
static double vdw_mu(double rr, double Tr)
{
    return (8.0 * Tr / 3.0) * (log(rr / (3.0 - rr)) + 3.0 / (3.0 - rr)) - 6.0 * rr;
}

/* Outer roots of p~(rho) = P at temperature Tr: the cubic
 * rho^3 - 3 rho^2 + b rho - P = 0, b = (8 Tr + P)/3, by the trigonometric
 * formula, then polished with Newton steps on the cubic. */
static void vdw_outer_roots(double Tr, double P, double* rv, double* rl)
{
    const double b = (8.0 * Tr + P) / 3.0;
    const double p = b - 3.0;            /* rho = y + 1 gives y^3 + p y + q = 0 */
    const double q = b - 2.0 - P;
    double r = sqrt(-p / 3.0);
    double arg = (3.0 * q / (2.0 * p)) * sqrt(-3.0 / p);
    if (arg > 1.0) arg = 1.0;
    if (arg < -1.0) arg = -1.0;
    double phi = acos(arg) / 3.0;
    double roots[2];
    roots[0] = 1.0 + 2.0 * r * cos(phi - 4.0 * M_PI / 3.0);  /* smallest: vapour */
    roots[1] = 1.0 + 2.0 * r * cos(phi);                      /* largest: liquid  */
    for (int i = 0; i < 2; ++i) {
        double x = roots[i];
        for (int it = 0; it < 4; ++it) {
            double f = ((x - 3.0) * x + b) * x - P;
            double df = (3.0 * x - 6.0) * x + b;
            if (df == 0.0) break;
            x -= f / df;
        }
        roots[i] = x;
    }
    *rv = roots[0];
    *rl = roots[1];
}

int orc_maxwell(double Tr, double* rv_out, double* rl_out, double* ps_out)
{
    if (!(Tr > 0.0 && Tr < 1.0)) return ORC_EINVAL;
    /* Spinodal densities: dp~/drho~ = 0  <=>  4 Tr = rho (3 - rho)^2;
     * with rho = y + 2: y^3 - 3y + 2 - 4 Tr = 0, roots 2 cos(acos(2Tr-1)/3 - 2 pi k/3). */
    double phi = acos(2.0 * Tr - 1.0) / 3.0;
    double rsp1 = 2.0 + 2.0 * cos(phi + 2.0 * M_PI / 3.0);  /* in (0,1): local maximum of p */
    double rsp2 = 2.0 + 2.0 * cos(phi - 2.0 * M_PI / 3.0);  /* in (1,3): local minimum of p */
    double Phi = orc_vdw_reduced(rsp1, Tr);
    double Plo = orc_vdw_reduced(rsp2, Tr);
    if (Plo < 1e-300) Plo = 1e-300;
    /* g(P) = mu(rho_l(P)) - mu(rho_v(P)) is decreasing in P (dg/dP = 1/rho_l - 1/rho_v);
     * safeguarded Newton inside the bracket [Plo, Phi]. */
    double lo = Plo, hi = Phi;
    double P = 0.5 * (lo + hi);
    double rv = 0.0, rl = 0.0;
    for (int it = 0; it < 200; ++it) {
        vdw_outer_roots(Tr, P, &rv, &rl);
        double g = vdw_mu(rl, Tr) - vdw_mu(rv, Tr);
        if (g > 0.0) lo = P; else hi = P;
        double dg = 1.0 / rl - 1.0 / rv;
        double Pn = P - g / dg;
        if (!(Pn > lo && Pn < hi)) Pn = 0.5 * (lo + hi);
        double step = fabs(Pn - P);
        P = Pn;
        if (step <= 1e-16 * P || hi - lo <= 1e-16 * P) break;
    }
    vdw_outer_roots(Tr, P, &rv, &rl);
    if (rv_out) *rv_out = rv;
    if (rl_out) *rl_out = rl;
    if (ps_out) *ps_out = P;
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Equilibrium (eq:feq)
 * ------------------------------------------------------------------------- */

static void equilibrium(const lattice* L, double rho, const double* u, double* feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int k = 0; k < L->Q; ++k) {
        double cu = L->c[k][0] * u[0] + L->c[k][1] * u[1] + L->c[k][2] * u[2];
        feq[k] = rho * L->w[k] *
                 (1.0 + cu / THETA + cu * cu / (2.0 * THETA * THETA) - uu / (2.0 * THETA));
    }
}

int orc_equilibrium(int Q, double rho, const double* u, double* feq)
{
    lattice L;
    if (make_lattice(Q, &L) < 0) return ORC_EINVAL;
    equilibrium(&L, rho, u, feq);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Neighbourhood operators on a periodic box
 * ------------------------------------------------------------------------- */

static long wrap(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

static long node_at(int nx, int ny, int nz, long x, long y, long z)
{
    return wrap(x, nx) + (long)nx * (wrap(y, ny) + (long)ny * wrap(z, nz));
}

/* Plane index of z on a box with walls halfway below 0 and above nz - 1: a plane beyond a
 * wall is the mirror image of the fluid plane on the other side of the wall. */
static long mirror_z(long z, int nz)
{
    if (z < 0) return -1 - z;
    if (z >= nz) return 2L * nz - 1 - z;
    return z;
}

/* F(x) = (1/alpha h) [ A sum_k G_k Phi^2(x+e_k) e_k + (1-2A) Phi(x) sum_k G_k Phi(x+e_k) e_k ],
 * sums over the moving directions k = 1..b (section 3).  With walls, Phi beyond a wall is the
 * mirror image (a wall that neither attracts nor repels the fluid more than the fluid itself). */
static void force_field(const lattice* L, int nx, int ny, int nz, double A, const double* Phi,
                        int walls, double* F)
{
    const long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long i = x + nx * (y + ny * z);
                double s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
                for (int k = 1; k < L->Q; ++k) {
                    long zz = z + L->c[k][2];
                    if (walls) zz = mirror_z(zz, nz);
                    long j = node_at(nx, ny, nz, x + L->c[k][0], y + L->c[k][1], zz);
                    double ph = Phi[j];
                    for (int a = 0; a < 3; ++a) {
                        s1[a] += L->G[k] * ph * ph * L->c[k][a];
                        s2[a] += L->G[k] * ph * L->c[k][a];
                    }
                }
                for (int a = 0; a < 3; ++a)
                    F[a * n + i] = (A * s1[a] + (1.0 - 2.0 * A) * Phi[i] * s2[a]) / L->alpha;
            }
}

int orc_force(int Q, int nx, int ny, int nz, double A, const double* Phi, double* F)
{
    lattice L;
    if (make_lattice(Q, &L) < 0) return ORC_EINVAL;
    force_field(&L, nx, ny, nz, A, Phi, 0, F);
    return ORC_OK;
}

int orc_force_walls(int nx, int ny, int nz, double A, const double* Phi, double* F)
{
    lattice L;
    make_lattice(19, &L);
    force_field(&L, nx, ny, nz, A, Phi, 1, F);
    return ORC_OK;
}

/* div u = sum_a (u_a(x + e_a) - u_a(x - e_a)) / 2h over the D spatial axes
 * (the central difference of section 6.2 on each axis).  With walls, u_z beyond a wall is the
 * mirror image with the opposite sign, so the wall face carries no flux. */
static void divergence(int D, int nx, int ny, int nz, const double* u, int walls, double* div)
{
    const long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long i = x + nx * (y + ny * z);
                double d = 0.0;
                for (int a = 0; a < D; ++a) {
                    long e[3] = {0, 0, 0};
                    e[a] = 1;
                    long ip = node_at(nx, ny, nz, x + e[0], y + e[1], z + e[2]);
                    long im = node_at(nx, ny, nz, x - e[0], y - e[1], z - e[2]);
                    double up = u[a * n + ip], um = u[a * n + im];
                    if (walls && a == 2 && z == nz - 1) up = -u[a * n + i];
                    if (walls && a == 2 && z == 0) um = -u[a * n + i];
                    d += (up - um) / 2.0;
                }
                div[i] = d;
            }
}

int orc_divergence(int D, int nx, int ny, int nz, const double* u, double* div)
{
    if (D != 2 && D != 3) return ORC_EINVAL;
    divergence(D, nx, ny, nz, u, 0, div);
    return ORC_OK;
}

int orc_divergence_walls(int nx, int ny, int nz, const double* u, double* div)
{
    divergence(3, nx, ny, nz, u, 1, div);
    return ORC_OK;
}

/* Wall description for the conduction stencil: at a wall face the node beyond the wall has
 * the mirrored density and either the mirrored temperature (adiabatic wall: no flux) or the
 * temperature 2 T_wall - T(x), which puts T_wall on the wall face half a cell away. */
typedef struct {
    int on;
    unsigned fixed;      /* ORC_WALL_T_BOTTOM | ORC_WALL_T_TOP */
    double T_bottom, T_top;
} walls_t;

/* div(lambda grad T) with lambda = rho c_v chi (section 4), conservative form:
 * sum_a [ lam(x, x+e_a) (T(x+e_a) - T(x)) - lam(x, x-e_a) (T(x) - T(x-e_a)) ],
 * lam(x, y) = c_v chi (rho(x) + rho(y)) / 2. */
static void conduction(int D, int nx, int ny, int nz, double c_v, double chi, const double* rho,
                       const double* T, const walls_t* wl, double* out)
{
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) {
                long i = x + nx * (y + ny * z);
                double s = 0.0;
                for (int a = 0; a < D; ++a) {
                    long e[3] = {0, 0, 0};
                    e[a] = 1;
                    long ip = node_at(nx, ny, nz, x + e[0], y + e[1], z + e[2]);
                    long im = node_at(nx, ny, nz, x - e[0], y - e[1], z - e[2]);
                    double rp = rho[ip], rm = rho[im], Tp = T[ip], Tm = T[im];
                    if (wl && wl->on && a == 2 && z == nz - 1) {
                        rp = rho[i];
                        Tp = (wl->fixed & ORC_WALL_T_TOP) ? 2.0 * wl->T_top - T[i] : T[i];
                    }
                    if (wl && wl->on && a == 2 && z == 0) {
                        rm = rho[i];
                        Tm = (wl->fixed & ORC_WALL_T_BOTTOM) ? 2.0 * wl->T_bottom - T[i] : T[i];
                    }
                    double lp = c_v * chi * (rho[i] + rp) / 2.0;
                    double lm = c_v * chi * (rho[i] + rm) / 2.0;
                    s += lp * (Tp - T[i]) - lm * (T[i] - Tm);
                }
                out[i] = s;
            }
}

int orc_conduction(int D, int nx, int ny, int nz, double c_v, double chi, const double* rho,
                   const double* T, double* out)
{
    if (D != 2 && D != 3) return ORC_EINVAL;
    conduction(D, nx, ny, nz, c_v, chi, rho, T, NULL, out);
    return ORC_OK;
}

int orc_conduction_walls(int nx, int ny, int nz, double c_v, double chi, const double* rho,
                         const double* T, unsigned wall_heat, double T_bottom, double T_top,
                         double* out)
{
    const walls_t wl = {1, wall_heat, T_bottom, T_top};
    conduction(3, nx, ny, nz, c_v, chi, rho, T, &wl, out);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * Simulation state and the time step
 * ------------------------------------------------------------------------- */

struct orc_sim {
    orc_params p;                   /* eos_p, eos_coex point at the copies below */
    double *eos_p, *eos_coex;
    lattice L;
    long n;
    long long step;
    double *N, *g;                  /* populations, node-major f[i*Q + k]  */
    double *Np, *gp;                /* post-collision populations          */
    double *rho, *j, *u, *E, *T;    /* moments (j, u: 3 planes)            */
    double *pr, *Phi, *F, *du, *us; /* EOS, force, velocity change, u*     */
    double *divu, *work, *cond, *latent, *dE;
};

static double* alloc0(long n)
{
    return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
}

static int valid_params(const orc_params* p)
{
    if (!(p->Q == 3 || p->Q == 9 || p->Q == 19)) return 0;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return 0;
    if (p->Q == 9 && p->nz != 1) return 0;
    if (p->Q == 3 && (p->ny != 1 || p->nz != 1)) return 0;
    if (!(p->tau > 0.5 && p->tau_E > 0.5)) return 0;
    if (!(p->rho_c > 0 && p->T_c > 0 && p->p_c > 0 && p->c_v > 0)) return 0;
    if (!(p->chi >= 0)) return 0;
    /* explicit conduction is stable for chi dt/h^2 < 0.5/d (section 6.1); d counts the axes
     * the box extends along (an axis of extent 1 contributes no conduction at all) */
    int d = (p->nx > 1) + (p->ny > 1) + (p->Q == 19 && p->nz > 1);
    if (d < 1) d = 1;
    if ((p->flags & ORC_CONDUCTION) && !(p->chi < 0.5 / d)) return 0;
    if (p->walls) {
        if (p->walls != 1 || p->Q != 19 || p->nz < 2) return 0;
        if ((p->wall_heat & ORC_WALL_T_BOTTOM) && !(p->T_bottom > 0.0)) return 0;
        if ((p->wall_heat & ORC_WALL_T_TOP) && !(p->T_top > 0.0)) return 0;
        /* a fixed-temperature wall face is half a cell away, which doubles its conductance:
         * the explicit update of a node next to it stays positive for chi < 1/(2d + 1) */
        if ((p->flags & ORC_CONDUCTION) && p->wall_heat && !(p->chi < 1.0 / (2 * d + 1))) return 0;
    }
    for (int a = 0; a < 3; ++a)
        if (!isfinite(p->gravity[a])) return 0;
    if (p->collision != ORC_BGK && p->collision != ORC_MRT) return 0;
    if (p->eos != ORC_EOS_VDW && p->eos != ORC_EOS_TABLE) return 0;
    if (p->eos == ORC_EOS_TABLE) {
        if (!p->eos_p || !p->eos_coex || p->eos_nrho < 4 || p->eos_nT < 2) return 0;
        if (!(p->eos_rho_max > p->eos_rho_min && p->eos_rho_min >= 0.0)) return 0;
        if (!(p->eos_T_max > p->eos_T_min && p->eos_T_min > 0.0)) return 0;
        for (long i = 0; i < (long)p->eos_nrho * p->eos_nT; ++i)
            if (!isfinite(p->eos_p[i])) return 0;
        for (long j = 0; j < p->eos_nT; ++j)
            if (!(p->eos_coex[2 * j] <= p->eos_coex[2 * j + 1])) return 0;
    }
    if (p->collision == ORC_MRT) {
        if (!(p->Q == 9 || p->Q == 19)) return 0;
        const double r[4] = {p->s_e, p->s_eps, p->s_q, p->s_m};
        for (int i = 0; i < 4; ++i)
            if (!(r[i] > 0.0 && r[i] < 2.0)) return 0;
    }
    return 1;
}

orc_sim* orc_create(const orc_params* p, const double* rho0, const double* u0, const double* T0,
                    int* status)
{
    if (status) *status = ORC_EINVAL;
    if (!p || !valid_params(p) || !rho0 || !u0 || !T0) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->p = *p;
    if (p->eos == ORC_EOS_TABLE) {
        const size_t np = (size_t)p->eos_nrho * p->eos_nT;
        s->eos_p = (double*)malloc(sizeof(double) * np);
        s->eos_coex = (double*)malloc(sizeof(double) * 2 * p->eos_nT);
        memcpy(s->eos_p, p->eos_p, sizeof(double) * np);
        memcpy(s->eos_coex, p->eos_coex, sizeof(double) * 2 * p->eos_nT);
        s->p.eos_p = s->eos_p;
        s->p.eos_coex = s->eos_coex;
    } else {
        s->p.eos_p = NULL;
        s->p.eos_coex = NULL;
    }
    make_lattice(p->Q, &s->L);
    const long n = (long)p->nx * p->ny * p->nz;
    const int Q = p->Q;
    s->n = n;
    s->N = alloc0(n * Q);  s->g = alloc0(n * Q);
    s->Np = alloc0(n * Q); s->gp = alloc0(n * Q);
    s->rho = alloc0(n); s->j = alloc0(3 * n); s->u = alloc0(3 * n);
    s->E = alloc0(n); s->T = alloc0(n); s->pr = alloc0(n); s->Phi = alloc0(n);
    s->F = alloc0(3 * n); s->du = alloc0(3 * n); s->us = alloc0(3 * n);
    s->divu = alloc0(n); s->work = alloc0(n); s->cond = alloc0(n); s->latent = alloc0(n);
    s->dE = alloc0(n);
    for (long i = 0; i < n; ++i) {
        if (!(rho0[i] > 0.0 && rho0[i] / p->rho_c < 3.0 && T0[i] > 0.0)) {
            orc_free(s);
            return NULL;
        }
        double u[3] = {u0[i], u0[n + i], u0[2 * n + i]};
        equilibrium(&s->L, rho0[i], u, &s->N[i * Q]);
        equilibrium(&s->L, rho0[i] * p->c_v * T0[i], u, &s->g[i * Q]);
    }
    if (status) *status = ORC_OK;
    return s;
}

void orc_free(orc_sim* s)
{
    if (!s) return;
    double* fields[] = {s->N, s->g, s->Np, s->gp, s->rho, s->j, s->u, s->E, s->T, s->pr, s->Phi,
                        s->F, s->du, s->us, s->divu, s->work, s->cond, s->latent, s->dE};
    for (size_t i = 0; i < sizeof(fields) / sizeof(fields[0]); ++i) free(fields[i]);
    free(s->eos_p);
    free(s->eos_coex);
    free(s);
}

/* Step 1: rho = sum N_k, rho u = sum c_k N_k (eq:hydro); E = sum g_k, T = E/(rho c_v). */
static void pass_moments(orc_sim* s)
{
    const long n = s->n;
    const int Q = s->p.Q;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double r = 0, jx = 0, jy = 0, jz = 0, e = 0;
        for (int k = 0; k < Q; ++k) {
            double f = s->N[i * Q + k];
            r += f;
            jx += s->L.c[k][0] * f;
            jy += s->L.c[k][1] * f;
            jz += s->L.c[k][2] * f;
            e += s->g[i * Q + k];
        }
        s->rho[i] = r;
        s->j[i] = jx; s->j[n + i] = jy; s->j[2 * n + i] = jz;
        s->u[i] = jx / r; s->u[n + i] = jy / r; s->u[2 * n + i] = jz / r;
        s->E[i] = e;
        s->T[i] = e / (r * s->p.c_v);
    }
}

/* Temperature that enters the equation of state (section 4: barotropic variant). */
static double eos_temperature(const orc_sim* s, long i)
{
    return (s->p.flags & ORC_BAROTROPIC) ? s->p.T0_baro : s->T[i];
}

/* Step 2: p = p_c p~(rho/rho_c, T/T_c); U = p - rho theta; Phi = sqrt(-U).
 * Returns 0 if some node has -U <= 0 or a non-finite moment. */
static int pass_eos(orc_sim* s)
{
    const long n = s->n;
    int ok = 1;
    for (long i = 0; i < n; ++i) {
        double rr = s->rho[i] / s->p.rho_c;
        double Tr = eos_temperature(s, i) / s->p.T_c;
        int inside = 1;
        double p = s->p.eos == ORC_EOS_TABLE ? s->p.p_c * orc_table_reduced(&s->p, rr, Tr, &inside)
                                             : s->p.p_c * orc_vdw_reduced(rr, Tr);
        double minusU = s->rho[i] * THETA - p;
        s->pr[i] = p;
        if (!inside || !(minusU > 0.0) || !(rr < 3.0) || !isfinite(s->E[i]) || !(s->rho[i] > 0.0)) {
            ok = 0;
            s->Phi[i] = 0.0;
        } else {
            s->Phi[i] = sqrt(minusU);
        }
    }
    return ok;
}

/* Step 3 (continued): uniform body force, F += rho g. */
static void pass_body_force(orc_sim* s)
{
    const long n = s->n;
    for (int a = 0; a < 3; ++a)
        if (s->p.gravity[a] != 0.0)
            for (long i = 0; i < n; ++i) s->F[a * n + i] += s->rho[i] * s->p.gravity[a];
}

/* Step 4: du = F dt / rho (eq:edm); u* = u + du/2 (eq:ustar). */
static void pass_velocity(orc_sim* s)
{
    const long n = s->n;
    for (int a = 0; a < 3; ++a)
        for (long i = 0; i < n; ++i) {
            s->du[a * n + i] = s->F[a * n + i] / s->rho[i];
            s->us[a * n + i] = (s->j[a * n + i] + s->F[a * n + i] / 2.0) / s->rho[i];
        }
}

/* Step 5: energy source per node and time step.
 *   work:   -p div u*                                  (section 4, 6.2)
 *   cond:   div(lambda grad T), lambda = rho c_v chi   (section 4)
 *   latent: -rho_liq Q / (rho_2 - rho_1) rho div u*    (section 5) */
static void pass_energy_source(orc_sim* s)
{
    const orc_params* p = &s->p;
    const long n = s->n;
    divergence(s->L.D, p->nx, p->ny, p->nz, s->us, p->walls, s->divu);
    const walls_t wl = {p->walls, p->wall_heat, p->T_bottom, p->T_top};
    if (p->flags & ORC_CONDUCTION)
        conduction(s->L.D, p->nx, p->ny, p->nz, p->c_v, p->chi, s->rho, s->T, &wl, s->cond);
    else
        memset(s->cond, 0, sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < n; ++i) {
        s->work[i] = (p->flags & ORC_WORK) ? -s->pr[i] * s->divu[i] : 0.0;
        s->latent[i] = 0.0;
        if (p->flags & ORC_LATENT) {
            double Tr = eos_temperature(s, i) / p->T_c;
            double rv, rl;
            int band = 0;
            if (p->eos == ORC_EOS_TABLE)
                band = table_band(p, Tr, &rv, &rl);
            else if (Tr >= LATENT_TMIN && Tr < LATENT_TMAX)
                band = orc_maxwell(Tr, &rv, &rl, NULL) == ORC_OK;
            if (band) {
                double r1 = rv * p->rho_c, r2 = rl * p->rho_c;
                if (s->rho[i] > r1 && s->rho[i] < r2)
                    s->latent[i] = -p->rhoQ / (r2 - r1) * s->rho[i] * s->divu[i];
            }
        }
        s->dE[i] = s->work[i] + s->cond[i] + s->latent[i];
    }
}

/* Steps 6-7: collisions.
 *   N'_k = N_k + (Neq(rho,u) - N_k)/tau + [Neq(rho,u+du) - Neq(rho,u)]             (eq:lbe, eq:edm)
 *   g'_k = g_k + (geq(E,u) - g_k)/tau_E + g_k dE/E + [geq(E,u+du) - geq(E,u)]      (eq:gk, section 4) */
static void pass_collide(orc_sim* s)
{
    const orc_params* p = &s->p;
    const long n = s->n;
    const int Q = p->Q;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double u[3] = {s->u[i], s->u[n + i], s->u[2 * n + i]};
        double v[3] = {u[0] + s->du[i], u[1] + s->du[n + i], u[2] + s->du[2 * n + i]};
        double Neq_u[19], Neq_v[19], geq_u[19], geq_v[19];
        equilibrium(&s->L, s->rho[i], u, Neq_u);
        equilibrium(&s->L, s->rho[i], v, Neq_v);
        equilibrium(&s->L, s->E[i], u, geq_u);
        equilibrium(&s->L, s->E[i], v, geq_v);
        if (p->collision == ORC_MRT) {
            /* multiple relaxation times: the non-equilibrium part N - Neq(rho, u) relaxes moment
             * by moment, m_i -> m_i (1 - s_i), with the shear rate 1/tau; the EDM increment is
             * added as for BGK.  With every rate equal to 1/tau this is the BGK update. */
            const double rate[6] = {0.0, 1.0 / p->tau, p->s_e, p->s_eps, p->s_q, p->s_m};
            double fneq[19], m[19];
            for (int k = 0; k < Q; ++k) fneq[k] = s->N[i * Q + k] - Neq_u[k];
            for (int a = 0; a < Q; ++a) {
                m[a] = 0.0;
                for (int k = 0; k < Q; ++k) m[a] += s->L.M[a][k] * fneq[k];
            }
            for (int k = 0; k < Q; ++k) {
                double relax = 0.0;
                for (int a = 0; a < Q; ++a)
                    relax += rate[s->L.grp[a]] * m[a] / s->L.M2[a] * s->L.M[a][k];
                s->Np[i * Q + k] = Neq_v[k] + fneq[k] - relax;
            }
        }
        for (int k = 0; k < Q; ++k) {
            double N = s->N[i * Q + k];
            if (p->collision != ORC_MRT)
                s->Np[i * Q + k] = N + (Neq_u[k] - N) / p->tau + (Neq_v[k] - Neq_u[k]);
            double g = s->g[i * Q + k];
            double gnew = g + (geq_u[k] - g) / p->tau_E + g * s->dE[i] / s->E[i];
            if (p->flags & ORC_PSEUDOFORCE) gnew += geq_v[k] - geq_u[k];
            s->gp[i * Q + k] = gnew;
        }
    }
}

/* Step 8: N_k(x + c_k, t + 1) = N'_k(x, t), same for g_k; periodic.  With walls, a population
 * whose target lies beyond a wall returns to its own node in the opposite direction:
 * N_{-k}(x, t + 1) = N'_k(x, t) (bounce-back, the wall halfway between the planes). */
static void pass_stream(orc_sim* s)
{
    const orc_params* p = &s->p;
    const int Q = p->Q;
#pragma omp parallel for schedule(static)
    for (long z = 0; z < p->nz; ++z)
        for (long y = 0; y < p->ny; ++y)
            for (long x = 0; x < p->nx; ++x) {
                long i = x + p->nx * (y + p->ny * z);
                for (int k = 0; k < Q; ++k) {
                    const long zt = z + s->L.c[k][2];
                    if (p->walls && (zt < 0 || zt >= p->nz)) {
                        const int kb = s->L.opp[k];
                        s->N[i * Q + kb] = s->Np[i * Q + k];
                        s->g[i * Q + kb] = s->gp[i * Q + k];
                        continue;
                    }
                    long j = node_at(p->nx, p->ny, p->nz, x + s->L.c[k][0], y + s->L.c[k][1], zt);
                    s->N[j * Q + k] = s->Np[i * Q + k];
                    s->g[j * Q + k] = s->gp[i * Q + k];
                }
            }
}

int orc_step(orc_sim* s, int nsteps)
{
    if (!s || nsteps < 0) return ORC_EINVAL;
    for (int t = 0; t < nsteps; ++t) {
        pass_moments(s);
        if (!pass_eos(s)) return ORC_EUNSTABLE;
        force_field(&s->L, s->p.nx, s->p.ny, s->p.nz, s->p.A, s->Phi, s->p.walls, s->F);
        pass_body_force(s);
        pass_velocity(s);
        pass_energy_source(s);
        pass_collide(s);
        pass_stream(s);
        s->step += 1;
    }
    return ORC_OK;
}

int orc_moments(orc_sim* s, double* rho, double* ustar, double* E, double* T)
{
    const long n = s->n;
    pass_moments(s);
    int ok = pass_eos(s);
    force_field(&s->L, s->p.nx, s->p.ny, s->p.nz, s->p.A, s->Phi, s->p.walls, s->F);
    pass_body_force(s);
    pass_velocity(s);
    if (rho) memcpy(rho, s->rho, sizeof(double) * (size_t)n);
    if (ustar) memcpy(ustar, s->us, sizeof(double) * (size_t)(3 * n));
    if (E) memcpy(E, s->E, sizeof(double) * (size_t)n);
    if (T) memcpy(T, s->T, sizeof(double) * (size_t)n);
    return ok ? ORC_OK : ORC_EUNSTABLE;
}

void orc_totals(orc_sim* s, double* out5)
{
    const long n = s->n;
    const int Q = s->p.Q;
    double m = 0, px = 0, py = 0, pz = 0, e = 0;
    for (long i = 0; i < n; ++i)
        for (int k = 0; k < Q; ++k) {
            double f = s->N[i * Q + k];
            m += f;
            px += s->L.c[k][0] * f;
            py += s->L.c[k][1] * f;
            pz += s->L.c[k][2] * f;
            e += s->g[i * Q + k];
        }
    out5[0] = m; out5[1] = px; out5[2] = py; out5[3] = pz; out5[4] = e;
}

void orc_last_sources(orc_sim* s, double* work, double* cond, double* latent)
{
    const size_t bytes = sizeof(double) * (size_t)s->n;
    if (work) memcpy(work, s->work, bytes);
    if (cond) memcpy(cond, s->cond, bytes);
    if (latent) memcpy(latent, s->latent, bytes);
}

void orc_get_pops(orc_sim* s, double* N, double* g)
{
    const long n = s->n;
    const int Q = s->p.Q;
    for (int k = 0; k < Q; ++k)
        for (long i = 0; i < n; ++i) {
            if (N) N[k * n + i] = s->N[i * Q + k];
            if (g) g[k * n + i] = s->g[i * Q + k];
        }
}

void orc_set_pops(orc_sim* s, const double* N, const double* g)
{
    const long n = s->n;
    const int Q = s->p.Q;
    for (int k = 0; k < Q; ++k)
        for (long i = 0; i < n; ++i) {
            if (N) s->N[i * Q + k] = N[k * n + i];
            if (g) s->g[i * Q + k] = g[k * n + i];
        }
}

long long orc_step_count(orc_sim* s) { return s->step; }

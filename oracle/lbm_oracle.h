/*
 * FP64 CPU oracle of the thermal multiphase lattice Boltzmann method of
 * Kupershtokh, Medvedev and Gribanov, "Thermal lattice Boltzmann method for
 * multiphase flows" (arXiv:1705.10045).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product (the HIP
 * library under paper_1705_10045_amd/) shares no code, header, table or
 * constant with it.
 *
 * Layout of every field argument: row-major over nodes, idx = x + nx*(y + ny*z);
 * vector fields are three consecutive planes [vx(n) | vy(n) | vz(n)].
 * Populations inside the oracle are node-major (AoS): f[idx*Q + k].
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Physical terms that can be switched on and off (the ablations of sections 4-6). */
#define ORC_WORK        1u   /* pressure work -p div u*                              */
#define ORC_CONDUCTION  2u   /* heat conduction div(lambda grad T)                   */
#define ORC_LATENT      4u   /* latent heat inside the transition layer (section 5)  */
#define ORC_PSEUDOFORCE 8u   /* EDM "pseudoforces" on the energy populations         */
#define ORC_BAROTROPIC 16u   /* EOS at the fixed temperature T0_baro (section 4)     */

/* Walls (walls = 1): which walls are held at a fixed temperature; the others are adiabatic. */
#define ORC_WALL_T_BOTTOM 1u /* z = -1/2 held at T_bottom                            */
#define ORC_WALL_T_TOP    2u /* z = nz - 1/2 held at T_top                           */

#define ORC_BGK 0           /* collision of N_k: one relaxation time tau (section 2)   */
#define ORC_MRT 1           /* several relaxation times on an orthogonal moment basis */

#define ORC_EOS_VDW   0     /* reduced van der Waals equation of state (section 3)     */
#define ORC_EOS_TABLE 1     /* reduced pressure interpolated in a table (section 3)    */

#define ORC_OK         0
#define ORC_EINVAL    -1
#define ORC_EUNSTABLE -3

typedef struct {
    int Q;                 /* 3 (D1Q3, ny = nz = 1), 9 (D2Q9, nz = 1), 19 (D3Q19) */
    int nx, ny, nz;        /* periodic box                                    */
    double tau, tau_E;     /* BGK relaxation times of N_k and g_k             */
    double A;              /* force mixing parameter (section 3)              */
    double rho_c, T_c, p_c;/* critical point of the van der Waals fluid       */
    double c_v, chi, rhoQ; /* specific heat, thermal diffusivity, rho_liq*Q   */
    double T0_baro;        /* EOS temperature when ORC_BAROTROPIC is set      */
    unsigned flags;
    /* Solid walls normal to z (not part of the paper, which is periodic): walls = 1 puts
     * no-slip walls halfway between lattice planes, below z = 0 and above z = nz - 1.  Streaming
     * bounces populations back at them (N and g alike); beyond a wall Phi and rho are mirrored,
     * u*_z is mirrored with the opposite sign, and T is mirrored (adiabatic wall) or set so that
     * the wall face has the wall temperature (ORC_WALL_T_* in wall_heat).  D3Q19 only. */
    int walls;
    unsigned wall_heat;
    double T_bottom, T_top;
    /* Uniform body force per unit mass: F += rho g at every node (section 2, external force
     * through the exact difference method). */
    double gravity[3];
    /* Collision of the density populations (section 2 names both forms): ORC_BGK, or ORC_MRT
     * with the shear moments relaxed at 1/tau, the energy moment e at s_e (bulk viscosity),
     * the energy-square and fourth-order moments at s_eps, the energy fluxes q at s_q and (D3Q19)
     * the third-order moments m at s_m, each rate in (0, 2).  D2Q9 and D3Q19 only.  The energy
     * populations g_k keep the single relaxation time tau_E of eq:gk. */
    int collision;
    double s_e, s_eps, s_q, s_m;
    /* Equation of state.  ORC_EOS_VDW: p = p_c p~(rho/rho_c, T/T_c) with the reduced van der
     * Waals p~ of section 3.  ORC_EOS_TABLE: section 3 allows tabulated equations of state of
     * real fluids; p~ is then interpolated in eos_p, given on the uniform grid
     * rho~_i = eos_rho_min + i (eos_rho_max - eos_rho_min)/(eos_nrho - 1),
     * T~_j = eos_T_min + j (eos_T_max - eos_T_min)/(eos_nT - 1), eos_p[j*eos_nrho + i]:
     * cubic Lagrange interpolation in rho~ through the four grid densities around the point
     * (the stencil shifted inward at the ends), linear in T~ between the two grid rows around
     * it.  A node outside the grid has left the EOS domain.  The coexistence band of the latent
     * heat (section 5) is eos_coex[2j], eos_coex[2j+1] (reduced rho_1 <= rho_2) at row j,
     * linear in T~ between rows; it acts over the table's whole temperature range.  Both arrays
     * are read at orc_create and copied. */
    int eos;
    const double* eos_p;
    const double* eos_coex;
    int eos_nrho, eos_nT;
    double eos_rho_min, eos_rho_max, eos_T_min, eos_T_max;
} orc_params;

/* Lattice tables: c[Q*3], w[Q], G[Q] (G[0] = 0), alpha.  Returns D or ORC_EINVAL. */
int orc_lattice(int Q, int* c, double* w, double* G, double* alpha);

/* MRT moment basis of D2Q9 or D3Q19: M[Q*Q] (row i = moment i at every velocity, in the
 * oracle's velocity order), norm2[Q] = squared row norms, group[Q] = 0 conserved, 1 shear,
 * 2 energy e, 3 energy square and fourth-order, 4 energy flux q, 5 third-order m. */
int orc_mrt_basis(int Q, double* M, double* norm2, int* group);

/* Reduced van der Waals pressure p~(rho~, T~) (section 3). */
double orc_vdw_reduced(double rr, double Tr);

/* Reduced pressure of the tabulated equation of state of p (ORC_EOS_TABLE) at (rr, Tr);
 * *inside = 0 (and 0 returned) outside the table's grid. */
double orc_table_reduced(const orc_params* p, double rr, double Tr, int* inside);

/* Maxwell equal-chemical-potential coexistence at reduced temperature Tr in (0,1):
 * reduced vapour density, liquid density and saturation pressure. */
int orc_maxwell(double Tr, double* rv, double* rl, double* psat);

/* Equilibrium populations (eq:feq) of a lattice at density rho and velocity u[3]. */
int orc_equilibrium(int Q, double rho, const double* u, double* feq);

/* Isotropic pseudopotential force of section 3 from a field Phi on a periodic box (no walls,
 * no body force). */
int orc_force(int Q, int nx, int ny, int nz, double A, const double* Phi, double* F);

/* Central-difference divergence of a vector field (3 planes) on a periodic box. */
int orc_divergence(int D, int nx, int ny, int nz, const double* u, double* div);

/* Conservative heat-conduction increment div(lambda grad T) per unit time,
 * lambda = rho c_v chi, face conductivity = arithmetic mean of the two nodes. */
int orc_conduction(int D, int nx, int ny, int nz, double c_v, double chi,
                   const double* rho, const double* T, double* out);

/* The same three operators on a D3Q19 box with walls normal to z (mirror ghosts as described
 * at orc_params.walls). */
int orc_force_walls(int nx, int ny, int nz, double A, const double* Phi, double* F);
int orc_divergence_walls(int nx, int ny, int nz, const double* u, double* div);
int orc_conduction_walls(int nx, int ny, int nz, double c_v, double chi, const double* rho,
                         const double* T, unsigned wall_heat, double T_bottom, double T_top,
                         double* out);

typedef struct orc_sim orc_sim;

/* Equilibrium initial state N = Neq(rho0,u0), g = geq(rho0 c_v T0, u0).
 * Returns NULL and *status = ORC_EINVAL on bad parameters or fields. */
orc_sim* orc_create(const orc_params* p, const double* rho0, const double* u0,
                    const double* T0, int* status);
/* Advance nsteps time steps; returns ORC_OK or ORC_EUNSTABLE (state is left at
 * the failing step). */
int orc_step(orc_sim* s, int nsteps);
/* rho, u* (eq:ustar, 3 planes), E, T of the current state.  Any pointer may be NULL. */
int orc_moments(orc_sim* s, double* rho, double* ustar, double* E, double* T);
/* Totals in index order: mass, momentum x,y,z, internal energy. */
void orc_totals(orc_sim* s, double* out5);
/* Energy-source fields of the last step: work, conduction, latent (each n values). */
void orc_last_sources(orc_sim* s, double* work, double* cond, double* latent);
/* Copy populations out / in, k-major planes: f[k*n + idx]. */
void orc_get_pops(orc_sim* s, double* N, double* g);
void orc_set_pops(orc_sim* s, const double* N, const double* g);
long long orc_step_count(orc_sim* s);
void orc_free(orc_sim* s);

#ifdef __cplusplus
}
#endif
#endif

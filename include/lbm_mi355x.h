/*
 * lbm_mi355x.h -- C ABI of the MI355X (gfx950) thermal multiphase lattice Boltzmann library.
 *
 * Method: Kupershtokh, Medvedev, Gribanov, "Thermal lattice Boltzmann method for multiphase
 * flows" (arXiv:1705.10045).  One time step advances two population sets on a periodic
 * D2Q9 or D3Q19 lattice (h = dt = 1, theta = 1/3):
 *   - density populations N_k: BGK collision (section 2, eq:lbe, eq:feq) with the
 *     pseudopotential force of a van der Waals fluid (section 3, eq:force2 and its isotropic
 *     lattice form) applied by the exact difference method (eq:edm);
 *   - energy populations g_k, E = sum g_k = rho c_v T: BGK collision with relaxation time
 *     tau_E (eq:gk), the finite-difference source dE spread in proportion to g_k (dg(1),
 *     section 4) and the EDM "pseudoforces" dg(2) (section 4);
 *   - dE = pressure work -p div u* (sections 4 and 6.2) + heat conduction div(lambda grad T),
 *     lambda = rho c_v chi (section 4) + latent heat released inside the transition layer
 *     (section 5).
 *
 * Conventions for every host array argument: FP64, row-major over nodes,
 * idx = x + nx*(y + ny*z); vector fields are three consecutive planes [vx(n)|vy(n)|vz(n)].
 * Host arrays are owned by the caller and only read/written during the call.  All device
 * memory is owned by the library and released by lbm_free / lbm_pool_destroy.
 * Functions never throw; they return an lbm_status and record a message retrievable with
 * lbm_last_error() on the calling thread.  Calls on one lbm_sim are not re-entrant.
 */
#ifndef LBM_MI355X_H
#define LBM_MI355X_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* bad parameter, shape or initial field                        */
    LBM_ENOMEM = -2,     /* device allocation failed                                     */
    LBM_EUNSTABLE = -3,  /* a node left the EOS domain (Phi^2 <= 0, rho~ >= 3, non-finite) */
    LBM_EDEVICE = -4,    /* HIP runtime error                                            */
    LBM_EBUSY = -5       /* serving pool: no free slot or memory budget for the request   */
} lbm_status;

/* Walls held at a fixed temperature (lbm_params.wall_heat); the others are adiabatic. */
enum {
    LBM_WALL_T_BOTTOM = 1u,  /* wall below z = 0 held at T_bottom                            */
    LBM_WALL_T_TOP = 2u      /* wall above z = nz - 1 held at T_top                          */
};

/* Collision of the density populations N_k (lbm_params.collision).  Section 2 names both the
 * single-relaxation-time (BGK) form it uses and the multiple-relaxation-time (MRT) form. */
enum {
    LBM_COLLISION_BGK = 0,  /* N_k relaxes toward Neq(rho, u) at 1/tau                       */
    LBM_COLLISION_MRT = 1   /* moments of N_k - Neq(rho, u) relax at their own rates         */
};

/* Equation of state (lbm_params.eos).  Section 3 uses the reduced van der Waals EOS and names
 * tabulated equations of state of real fluids as the alternative. */
enum {
    LBM_EOS_VDW = 0,    /* p = p_c p~(rho/rho_c, T/T_c), reduced van der Waals                */
    LBM_EOS_TABLE = 1   /* p~ interpolated in a caller's table (see lbm_params.eos_p)         */
};

/* Physical terms (the ablations of sections 4-6). */
enum {
    LBM_WORK = 1u,         /* pressure work -p div u*                                      */
    LBM_CONDUCTION = 2u,   /* heat conduction                                              */
    LBM_LATENT = 4u,       /* latent heat inside the transition layer                      */
    LBM_PSEUDOFORCE = 8u,  /* EDM pseudoforces on the energy populations                   */
    LBM_BAROTROPIC = 16u   /* EOS evaluated at the fixed temperature T0_baro (section 4)   */
};

typedef struct {
    int lattice;          /* 9 = D2Q9 (nz must be 1) or 19 = D3Q19                           */
    int nx, ny, nz;       /* periodic box, each >= 1                                         */
    int storage_bytes;    /* 4 = FP32 populations (D3Q19: FP32 arithmetic with FP64 EOS and
                             latent band; D2Q9: FP64 arithmetic), 8 = FP64 populations and
                             arithmetic                                                      */
    double tau, tau_E;    /* BGK relaxation times of N_k and g_k, both > 1/2                 */
    double A;             /* force mixing parameter of section 3 (the paper uses -0.152)     */
    double rho_c, T_c, p_c; /* critical point of the reduced vdW EOS, lattice units         */
    double c_v, chi;      /* specific heat at constant volume, thermal diffusivity           */
    double rhoQ;          /* rho_liq * Q, energy per volume released across the band         */
    double T0_baro;       /* EOS temperature with LBM_BAROTROPIC                             */
    unsigned flags;       /* LBM_WORK | LBM_CONDUCTION | LBM_LATENT | LBM_PSEUDOFORCE [...]  */
    /* Solid walls for pool boiling.  The paper's boxes are periodic, so this is an extension
     * with its own conventions (D3Q19 only).  walls = 1 puts no-slip walls normal to z halfway
     * between lattice planes, below z = 0 and above z = nz - 1:
     *   - streaming bounces N_k and g_k back at them (a population pulled from beyond a wall
     *     is the opposite population leaving the node itself);
     *   - beyond a wall, Phi and rho are mirrored and u*_z is mirrored with the opposite sign
     *     (no flux through the wall face);
     *   - T is mirrored (adiabatic wall) or set to 2 T_wall - T, which holds the wall face at
     *     T_wall (LBM_WALL_T_* in wall_heat).
     * walls = 0: periodic in z; wall_heat, T_bottom and T_top are then ignored. */
    int walls;
    unsigned wall_heat;
    double T_bottom, T_top;
    /* Uniform body force per unit mass (gravity): F += rho g at every node, applied by the
     * exact difference method like the interparticle force (eq:edm).  Zero for none. */
    double gravity[3];
    /* Collision of N_k.  LBM_COLLISION_MRT relaxes, on an orthogonal moment basis (Lallemand
     * and Luo 2000 for D2Q9, d'Humieres et al. 2002 for D3Q19), the traceless stresses at
     * 1/tau (so the shear viscosity is (tau - 1/2)/3 as with BGK), the energy moment e at s_e
     * (bulk viscosity), the energy-square and fourth-order moments at s_eps, the energy fluxes
     * at s_q and, for D3Q19, the third-order moments at s_m; each rate in (0, 2).  Density and
     * momentum are conserved as with BGK, and the EDM increment (eq:edm) is added unchanged.
     * The energy populations keep the single relaxation time tau_E of eq:gk.  With every rate
     * equal to 1/tau the update is the BGK one up to rounding.  The rates are ignored with
     * LBM_COLLISION_BGK. */
    int collision;
    double s_e, s_eps, s_q, s_m;
    /* Equation of state.  LBM_EOS_VDW (0, default): the reduced van der Waals EOS.
     * LBM_EOS_TABLE: the reduced pressure p~ = p/p_c is given by the caller on a uniform grid,
     * eos_p[j * eos_nrho + i] at rho~_i = eos_rho_min + i (eos_rho_max - eos_rho_min)/(eos_nrho - 1)
     * and T~_j = eos_T_min + j (eos_T_max - eos_T_min)/(eos_nT - 1) (rho~ = rho/rho_c,
     * T~ = T/T_c), and interpolated cubically in rho~ (Lagrange, the four grid densities around
     * the point, the stencil shifted inward next to the ends) and linearly in T~ between the two
     * rows around the point.  A node outside the grid has left the EOS domain (LBM_EUNSTABLE).
     * eos_coex[2j], eos_coex[2j + 1] are the reduced coexistence densities rho_1 <= rho_2 of row
     * j, the band of the latent heat (section 5), linear in T~ between rows; the latent source
     * acts over the table's whole temperature range (rho_1 = rho_2 leaves a row without band).
     * Both host arrays are read by lbm_init, which keeps its own device copy; eos_nrho >= 4,
     * eos_nT >= 2, at most 2^26 points.  lbm_pool_submit likewise keeps a device copy with
     * the request. */
    int eos;
    const double* eos_p;
    const double* eos_coex;
    int eos_nrho, eos_nT;
    double eos_rho_min, eos_rho_max, eos_T_min, eos_T_max;
} lbm_params;

typedef struct lbm_sim lbm_sim;

/* Create a simulation in the equilibrium state N_k = Neq_k(rho0, u0),
 * g_k = geq_k(rho0 c_v T0, u0) (eq:feq with E in place of rho, section 4).
 * rho0[n], u0[3n], T0[n]: host FP64 fields.  stream: a hipStream_t on the current device on
 * which every later call enqueues its work, or NULL for a library-created stream.
 * Rejects (LBM_EINVAL) tau or tau_E <= 1/2, lattice/shape mismatch, walls other than 0 or 1,
 * walls with D2Q9 or with nz < 2, a held wall temperature that is not positive, chi >=
 * 1/(2d + 1) with conduction and a held wall (its face is half a cell away), a non-finite
 * gravity, a collision other than LBM_COLLISION_BGK / _MRT or an MRT rate outside (0, 2), a
 * box whose population
 * plane (nx*ny*nz values, x rows padded to whole 128-byte lines) would exceed 4 GB (beyond any
 * state that fits in HBM), chi >= 0.5/d with
 * conduction on (d = number of axes with extent > 1; section 6.1), a non-positive or
 * non-finite field, rho0/rho_c >= 3, Phi^2 = rho theta - p <= 0 at any node (section 3), and
 * an initial field violating (dp/drho)_T <= (h/dt)^2 + theta (section 3). */
lbm_status lbm_init(const lbm_params* params, const double* rho0, const double* u0,
                    const double* T0, void* stream, lbm_sim** out);

/* Enqueue nsteps (>= 0) time steps on the simulation's stream, then synchronise and check the
 * device error word.  LBM_EUNSTABLE if any node left the EOS domain during these steps; the
 * state is then not meaningful (restore a checkpoint). */
lbm_status lbm_step(lbm_sim* sim, int nsteps);

/* Enqueue nsteps time steps without synchronising (for timing and overlap); errors found on
 * the device are reported by the next lbm_step, lbm_check or lbm_moments. */
lbm_status lbm_step_async(lbm_sim* sim, int nsteps);

/* Synchronise the stream and report the device error word (LBM_OK or LBM_EUNSTABLE). */
lbm_status lbm_check(lbm_sim* sim);

/* Fields of the current state: rho = sum N_k and E = sum g_k (eq:hydro, section 4),
 * u* = (sum c_k N_k + F/2)/rho (eq:ustar) with F the force of section 3 plus the body force
 * rho g, T = E/(rho c_v).  With walls, the populations pulled from beyond a wall are the
 * bounced-back ones, as in the step.  Each argument is a caller-owned host FP64 array of n
 * values (u_star: 3n), or NULL to skip it.  Synchronises. */
lbm_status lbm_moments(lbm_sim* sim, double* rho, double* u_star, double* E, double* T);

/* Same as lbm_moments but into caller-owned device FP64 arrays on the simulation's device;
 * enqueued on the simulation's stream (not synchronised).  The first call allocates a moment
 * scratch of 10 n doubles that the simulation keeps until lbm_free. */
lbm_status lbm_moments_device(lbm_sim* sim, double* rho, double* u_star, double* E, double* T);

/* lbm_moments_device for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid the allocator).  Same kernels and the
 * same results, bit for bit, but the scratch (7 n doubles) is a fixed 128 MiB device array of
 * the library, so the call allocates and frees nothing.  Limit: boxes of at most 2,396,745
 * nodes (128^3 fits); LBM_EINVAL for larger ones.  Outputs: caller-owned device FP64 arrays of
 * n values (u_star: 3n) on the simulation's device, any may be NULL; enqueued on the
 * simulation's stream, not synchronised.  The array is one per GPU, shared by every simulation
 * on it, and keeps the last call's contents: calls whose work overlaps on one GPU (from other
 * host threads, or on other streams before the previous call's work has finished) race on it
 * and give undefined fields; calls ordered on one stream are safe.  Each GPU the library runs
 * on holds the array until the process ends; the first call on a device looks up its address
 * there. */
lbm_status lbm_moments_device_noalloc(lbm_sim* sim, double* rho, double* u_star, double* E, double* T);

/* Totals of the current state accumulated in FP64 with a deterministic reduction order:
 * out[0] = sum N_k (mass), out[1..3] = sum c_k N_k (momentum), out[4] = sum g_k (internal
 * energy), over the stored post-collision populations.  Mass and momentum are conserved by the
 * step on a periodic box without gravity (eq:edm and the antisymmetric force); energy is
 * conserved when work and latent heat are off.  With walls, mass is conserved; the momentum is
 * that of the populations before they bounce back, and the walls exchange energy and
 * momentum. */
lbm_status lbm_reduce(lbm_sim* sim, double out[5]);

/* lbm_step followed by lbm_reduce, with the totals formed inside the last of the nsteps (>= 1)
 * steps: its collision sums, in FP64, the post-collision populations it stores (section 2,
 * eq:edm; the same quantities as lbm_reduce, out[0..4] as there, equal to them up to the order
 * of the FP64 sums), so the state is not read a second time.  The fields are bitwise those of
 * lbm_step.  The fused form exists for the lbm_set_launch variants 0, 5 and 7 of FP32 D3Q19,
 * 0 of FP64 D3Q19, 0 and 2 of FP32 D2Q9 and 0 of FP64 D2Q9 (every variant lbm_init starts
 * with); the others run the step and then the separate reduction.  The first call, and any
 * call after lbm_set_launch raised the workgroup count, allocates a device array of 5 doubles
 * per workgroup that the simulation keeps until lbm_free.  Synchronises; returns
 * LBM_EUNSTABLE like lbm_step (out is then not meaningful) and LBM_EINVAL for nsteps < 1 or
 * a NULL out. */
lbm_status lbm_step_reduce(lbm_sim* sim, int nsteps, double out[5]);

/* Number of time steps taken since lbm_init (or restored by lbm_restore). */
long long lbm_step_count(const lbm_sim* sim);

/* Bytes of device memory the state of a simulation with these parameters occupies
 * (population buffers; excludes transient buffers of lbm_moments). */
size_t lbm_footprint_bytes(const lbm_params* params);

/* Serialise the complete state (populations, step count) into host_buf of capacity cap;
 * *used receives the size (call with host_buf = NULL to query it).  Synchronises. */
lbm_status lbm_checkpoint(lbm_sim* sim, void* host_buf, size_t cap, size_t* used);

/* Restore a state written by lbm_checkpoint for the same parameters and shape. */
lbm_status lbm_restore(lbm_sim* sim, const void* host_buf, size_t len);

/* Release the simulation and its device memory.  NULL is accepted. */
lbm_status lbm_free(lbm_sim* sim);

/* Message of the last failing call on this thread ("" if none). */
const char* lbm_last_error(void);

/* Launch geometry of the fused step kernel: tile width/height in nodes, z-chunk length and
 * number of workgroups per step (for profiling reports). */
lbm_status lbm_launch_info(const lbm_sim* sim, int info[4]);

/* The launch lbm_init chooses for these parameters (default variant, automatic z chunk) on a
 * device with `cus` compute units (256 on MI355X), in the layout of lbm_launch_info.  Host
 * arithmetic only: touches no device and validates only the lattice, storage and shape
 * (LBM_EINVAL otherwise).  The z chunk minimises the number of rounds of resident workgroups
 * times (chunk + 4) planes, the moment stage's halo planes included. */
lbm_status lbm_launch_plan(const lbm_params* params, int cus, int info[4]);

/* Select the launch variant of the fused step kernel (0 .. n-1: tile shape, threads per
 * workgroup, prefetch or LDS stash; D3Q19 has eight with FP32 populations and four with FP64,
 * D2Q9 three: 32x8, 32x16 and 64x8 tiles) and the z-chunk length (0 = automatic).  lbm_init
 * starts with variant 0, except for FP32 D3Q19 states of 4 GB and more whose x extent tiles
 * at 64 with no more idle columns than at 32: those start with variant 7 (64x8 tiles, global
 * addressing).  Results do not depend on the choice (the per-node arithmetic is the same);
 * only speed does.  LBM_EINVAL for an unknown variant or a negative chunk. */
lbm_status lbm_set_launch(lbm_sim* sim, int variant, int chunk);

/* Velocity set used by the library (section 2) and the force coefficients of section 3:
 * c[3Q] (integer components), w[Q], G[Q], *alpha.  Returns the dimension D, or LBM_EINVAL
 * for an unsupported Q.  Host only; touches no device. */
int lbm_lattice_info(int Q, int* c, double* w, double* G, double* alpha);

/* Reduced van der Waals coexistence densities (rho~_vapour, rho~_liquid) at reduced
 * temperature Tr, from the library's FP64 Maxwell table (section 5 uses them as the band
 * limits rho_1, rho_2).  LBM_EINVAL outside the table range [0.4, 0.999]. */
lbm_status lbm_coexistence(double Tr, double* rho_v, double* rho_l);

/* ---------------------------------------------------------------------------------------
 * Serving: many independent D3Q19 simulations resident on one device.
 *
 * A pool owns device memory up to hbm_budget_bytes and up to max_slots slots.  Requests are
 * admitted into free slots while their footprint fits the remaining budget; one call to
 * lbm_pool_run advances every active slot by steps_per_run time steps with one batched
 * launch per step (captured once into a HIP graph and replayed), so requests of different
 * lattice sizes overlap on the device.  A slot whose remaining step count reaches zero stops
 * being advanced; its result stays resident until collected, after which the slot and its
 * memory are free for new requests.  Each request's result does not depend on which other
 * requests share the pool.
 * --------------------------------------------------------------------------------------- */
typedef struct lbm_pool lbm_pool;

/* Create a pool on the current device.  params of submitted requests must use lattice 19,
 * storage 4 and edges up to max_edge; walls, gravity, a tabulated EOS and the MRT collision are
 * accepted (each kind of request runs in its own launch of the batched step). */
lbm_status lbm_pool_create(size_t hbm_budget_bytes, int max_slots, int steps_per_run,
                           void* stream, lbm_pool** out);

/* Admit a request (fields as for lbm_init).  *ticket identifies it.  Its footprint is its two
 * population buffers plus, with a tabulated EOS, its own copy of the table (the caller's arrays
 * are read during the call only).  LBM_EBUSY if no slot is free or its footprint exceeds the
 * remaining budget (nothing is allocated then). */
lbm_status lbm_pool_submit(lbm_pool* pool, const lbm_params* params, const double* rho0,
                           const double* u0, const double* T0, long long nsteps,
                           long long* ticket);

/* Advance every active request by up to steps_per_run steps; synchronises and refreshes the
 * completion state. */
lbm_status lbm_pool_run(lbm_pool* pool);

/* The same replay without waiting for it: waits for the replay a previous call left in flight
 * (if any), refreshes the completion state from it, then enqueues the next replay of every
 * active request and returns.  Submissions and collections made while a replay is in flight
 * run on a second stream and overlap it (a request admitted then joins the next replay);
 * lbm_pool_poll reports the state as of the last replay waited for.  A call with no active
 * request only waits and refreshes.  lbm_pool_run waits for the replay it starts. */
lbm_status lbm_pool_run_async(lbm_pool* pool);

/* Completion of a ticket: *done = 1 when all its steps have run; *result = LBM_OK or
 * LBM_EUNSTABLE for a request that left the EOS domain (retired early, others unaffected). */
lbm_status lbm_pool_poll(lbm_pool* pool, long long ticket, int* done, lbm_status* result);

/* Copy the final fields of a finished request (as lbm_moments) and release its slot. */
lbm_status lbm_pool_collect(lbm_pool* pool, long long ticket, double* rho, double* u_star,
                            double* E, double* T);

/* Totals of a finished request that has not been collected yet, as lbm_reduce gives them
 * (mass, momentum x/y/z, internal energy; FP64, fixed order): initial[] of the state right
 * after admission, final_[] of its last state.  Either may be NULL.  LBM_EBUSY if the ticket
 * has not finished, LBM_EINVAL for an unknown ticket.  Synchronises the pool's second stream
 * only (a replay in flight continues). */
lbm_status lbm_pool_totals(lbm_pool* pool, long long ticket, double initial[5], double final_[5]);

/* Counters: out[0] active slots, out[1] bytes in use, out[2] budget, out[3] free slots. */
lbm_status lbm_pool_stats(const lbm_pool* pool, long long out[4]);

lbm_status lbm_pool_destroy(lbm_pool* pool);

#ifdef __cplusplus
}
#endif
#endif /* LBM_MI355X_H */

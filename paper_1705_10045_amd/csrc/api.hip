// Host side of the C ABI (include/lbm_mi355x.h): parameter validation, the FP64 Maxwell
// table, device memory, stepping, moments, reductions and checkpoints.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/lbm_mi355x.h"
#include "kernels.hpp"
#include "lattice.hpp"
#include "physics.hpp"
#include "sim.hpp"

namespace lbm {

static thread_local char g_last_error[512] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

void clear_error() { g_last_error[0] = '\0'; }

lbm_status hip_fail(hipError_t e, const char* what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE;
}

lbm_status use_device(int device)
{
    const hipError_t e = hipSetDevice(device);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "hipSetDevice");
}

// ------------------------------------------------------------------------------------------
// Maxwell coexistence table (section 5 band limits), reduced van der Waals fluid.
//
// Equal-area rule in specific volume v = 1/rho: p(v_l) = p(v_g) and
// integral_{v_l}^{v_g} p dv = p (v_g - v_l), with p(v) = 8T/(3v - 1) - 3/v^2 and the
// antiderivative (8T/3) ln(3v - 1) + 3/v.  Solved by Newton's method in (v_l, v_g),
// continued from the critical point (rho = 1 -/+ 2 sqrt(1 - T)) down the temperature grid.
// ------------------------------------------------------------------------------------------
namespace {

double p_of_v(double v, double T) { return 8.0 * T / (3.0 * v - 1.0) - 3.0 / (v * v); }
double dp_of_v(double v, double T)
{
    const double a = 3.0 * v - 1.0;
    return -24.0 * T / (a * a) + 6.0 / (v * v * v);
}
double int_p(double v, double T) { return (8.0 * T / 3.0) * std::log(3.0 * v - 1.0) + 3.0 / v; }

bool solve_coexistence(double T, double& vl, double& vg)
{
    for (int it = 0; it < 100; ++it) {
        const double pl = p_of_v(vl, T), pg = p_of_v(vg, T);
        const double f1 = pl - pg;
        const double f2 = int_p(vg, T) - int_p(vl, T) - pl * (vg - vl);
        const double a11 = dp_of_v(vl, T), a12 = -dp_of_v(vg, T);
        const double a21 = -dp_of_v(vl, T) * (vg - vl), a22 = pg - pl;
        const double det = a11 * a22 - a12 * a21;
        if (det == 0.0 || !std::isfinite(det)) return false;
        const double dl = (f1 * a22 - a12 * f2) / det;
        const double dg = (a11 * f2 - a21 * f1) / det;
        vl -= dl;
        vg -= dg;
        if (!(vl > 1.0 / 3.0) || !(vg > vl)) return false;
        if (std::fabs(dl) < 1e-15 * vl && std::fabs(dg) < 1e-15 * vg) return true;
    }
    return true;
}

struct MaxwellTable {
    std::vector<double> rho;  // interleaved (vapour, liquid) reduced densities
    double s0 = 0.0, ds = 0.0;
    bool ok = false;
};

const MaxwellTable& maxwell_table()
{
    static MaxwellTable tab;
    static std::once_flag once;
    std::call_once(once, [] {
        const int n = kMaxwellPoints;
        tab.rho.assign(2 * n, 0.0);
        tab.s0 = std::sqrt(1.0 - kLatentTmax);
        tab.ds = (std::sqrt(1.0 - kLatentTmin) - tab.s0) / (n - 1);
        double vl = 0, vg = 0, pl1 = 0, pg1 = 0, pl2 = 0, pg2 = 0;  // last two solutions
        bool good = true;
        for (int i = 0; i < n && good; ++i) {
            const double s = tab.s0 + i * tab.ds;
            const double T = 1.0 - s * s;
            if (i == 0) {          // critical-point asymptotics rho = 1 -/+ 2 sqrt(1 - T)
                vl = 1.0 / (1.0 + 2.0 * s);
                vg = 1.0 / (1.0 - 2.0 * s);
            } else if (i == 1) {   // previous solution
                vl = pl1;
                vg = pg1;
            } else {               // linear extrapolation along the branch
                vl = 2.0 * pl1 - pl2;
                vg = 2.0 * pg1 - pg2;
            }
            good = solve_coexistence(T, vl, vg);
            pl2 = pl1; pg2 = pg1;
            pl1 = vl; pg1 = vg;
            tab.rho[2 * i] = 1.0 / vg;
            tab.rho[2 * i + 1] = 1.0 / vl;
        }
        tab.ok = good;
    });
    return tab;
}

// dp/drho at fixed T for the reduced EOS in lattice units.
double dp_drho(double rho, double T, const Phys& ph)
{
    const double rr = rho * ph.inv_rho_c, tr = T * ph.inv_T_c;
    const double a = 3.0 - rr;
    return ph.p_c * ph.inv_rho_c * (24.0 * tr / (a * a) - 6.0 * rr);
}

// Pressure in lattice units of the simulation's EOS (the tabulated one from its host table);
// `inside` false outside a table's grid.
double host_pressure(double rho, double T, const Phys& ph, const double* table, bool& inside)
{
    inside = true;
    if (ph.eos == 0) return vdw_pressure(rho, T, ph);
    return ph.p_c * table_pressure(rho * ph.inv_rho_c, T * ph.inv_T_c, ph, table, inside);
}

// dp/drho at fixed T of the simulation's EOS: analytic for van der Waals, a central
// difference of the interpolant for a table (one-sided next to the grid's ends).
double host_dp_drho(double rho, double T, const Phys& ph, const double* table)
{
    if (ph.eos == 0) return dp_drho(rho, T, ph);
    const double h = 1e-6 * ph.rho_c;
    bool in_lo, in_hi;
    double lo_r = rho - h, hi_r = rho + h;
    double plo = host_pressure(lo_r, T, ph, table, in_lo);
    double phi = host_pressure(hi_r, T, ph, table, in_hi);
    if (!in_lo) { lo_r = rho; plo = host_pressure(rho, T, ph, table, in_lo); }
    if (!in_hi) { hi_r = rho; phi = host_pressure(rho, T, ph, table, in_hi); }
    return (phi - plo) / (hi_r - lo_r);
}

}  // namespace

bool host_band_limits(double Tr, double& rv, double& rl)
{
    const MaxwellTable& t = maxwell_table();
    if (!t.ok || !(Tr >= kLatentTmin && Tr <= kLatentTmax)) return false;
    const double pos = (std::sqrt(1.0 - Tr) - t.s0) / t.ds;
    int j = (int)pos;
    j = j < 1 ? 1 : (j > kMaxwellPoints - 3 ? kMaxwellPoints - 3 : j);
    const double x = pos - j;
    const double l0 = -x * (x - 1.0) * (x - 2.0) / 6.0, l1 = (x + 1.0) * (x - 1.0) * (x - 2.0) / 2.0;
    const double l2 = -(x + 1.0) * x * (x - 2.0) / 2.0, l3 = (x + 1.0) * x * (x - 1.0) / 6.0;
    const double* q = t.rho.data() + 2 * (j - 1);
    rv = l0 * q[0] + l1 * q[2] + l2 * q[4] + l3 * q[6];
    rl = l0 * q[1] + l1 * q[3] + l2 * q[5] + l3 * q[7];
    return true;
}

Phys make_phys(const lbm_params& p)
{
    Phys ph;
    ph.omega = 1.0 / p.tau;
    ph.omega_E = 1.0 / p.tau_E;
    ph.A = p.A;
    ph.inv_alpha = p.lattice == 9 ? 1.0 / Lattice<9>::alpha : 1.0 / Lattice<19>::alpha;
    ph.rho_c = p.rho_c;
    ph.inv_rho_c = 1.0 / p.rho_c;
    ph.inv_T_c = 1.0 / p.T_c;
    ph.p_c = p.p_c;
    ph.c_v = p.c_v;
    ph.inv_c_v = 1.0 / p.c_v;
    ph.cond_half = 0.5 * p.c_v * p.chi;
    ph.rhoQ = p.rhoQ;
    ph.T0_baro = p.T0_baro;
    ph.flags = p.flags;
    ph.walls = p.walls;
    ph.wall_heat = p.walls ? p.wall_heat : 0u;
    ph.T_bottom = p.T_bottom;
    ph.T_top = p.T_top;
    for (int a = 0; a < 3; ++a) ph.g[a] = p.gravity[a];
    ph.collision = p.collision;
    const bool mrt = p.collision == LBM_COLLISION_MRT;
    ph.mrt_de = mrt ? p.s_e - ph.omega : 0.0;
    ph.mrt_deps = mrt ? p.s_eps - ph.omega : 0.0;
    ph.mrt_dq = mrt ? p.s_q - ph.omega : 0.0;
    ph.mrt_dm = mrt ? p.s_m - ph.omega : 0.0;
    ph.eos = p.eos == LBM_EOS_TABLE ? 1 : 0;
    ph.tab_nrho = ph.eos ? p.eos_nrho : 0;
    ph.tab_nT = ph.eos ? p.eos_nT : 0;
    ph.tab_rho_min = p.eos_rho_min;
    ph.tab_rho_max = p.eos_rho_max;
    ph.tab_T_min = p.eos_T_min;
    ph.tab_T_max = p.eos_T_max;
    ph.tab_drho = ph.eos ? (p.eos_rho_max - p.eos_rho_min) / (p.eos_nrho - 1) : 0.0;
    ph.tab_dT = ph.eos ? (p.eos_T_max - p.eos_T_min) / (p.eos_nT - 1) : 0.0;
    return ph;
}

// Elements between consecutive population planes: the node count rounded up to 64 (256 B in
// FP32), plus 64 more, so that the same node of consecutive planes does not sit at the same
// power-of-two alignment (for the power-of-two boxes of the workloads every plane would
// otherwise start at a multiple of 8 MB-512 MB).  Measured 1-2.5% faster at 512^3, neutral at
// 128^3 and 256^3.
long long padded_plane(long long n) { return (n + 63) / 64 * 64 + 64; }

// Elements of one population plane's rows (x rows padded to the row pitch).
long long plane_elements(const lbm_params& p)
{
    return (long long)row_pitch(p.nx, p.storage_bytes) * p.ny * p.nz;
}

size_t state_bytes(const lbm_params& p)
{
    return (size_t)2 * p.lattice * padded_plane(plane_elements(p)) * p.storage_bytes;
}

lbm_status validate_params(const lbm_params* p)
{
    if (!p) { set_error("params is NULL"); return LBM_EINVAL; }
    if (p->lattice != 9 && p->lattice != 19) {
        set_error("lattice must be 9 (D2Q9) or 19 (D3Q19), got %d", p->lattice);
        return LBM_EINVAL;
    }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { set_error("box extents must be >= 1"); return LBM_EINVAL; }
    if (p->lattice == 9 && p->nz != 1) { set_error("D2Q9 needs nz == 1"); return LBM_EINVAL; }
    if ((long long)p->nx * p->ny * p->nz >= (1LL << 31)) { set_error("box exceeds 2^31 nodes"); return LBM_EINVAL; }
    if (p->storage_bytes != 4 && p->storage_bytes != 8) { set_error("storage_bytes must be 4 or 8"); return LBM_EINVAL; }
    if (!(p->tau > 0.5) || !(p->tau_E > 0.5)) { set_error("BGK needs tau > 1/2 and tau_E > 1/2"); return LBM_EINVAL; }
    if (!(p->rho_c > 0) || !(p->T_c > 0) || !(p->p_c > 0) || !(p->c_v > 0)) {
        set_error("rho_c, T_c, p_c and c_v must be positive");
        return LBM_EINVAL;
    }
    if (!(p->chi >= 0) || !(p->rhoQ >= 0) || !std::isfinite(p->A)) { set_error("chi, rhoQ must be >= 0 and A finite"); return LBM_EINVAL; }
    const int d = (p->nx > 1) + (p->ny > 1) + (p->lattice == 19 && p->nz > 1);
    if ((p->flags & LBM_CONDUCTION) && !(p->chi < 0.5 / (d < 1 ? 1 : d))) {
        set_error("explicit conduction needs chi < 0.5/d = %g (section 6.1)", 0.5 / (d < 1 ? 1 : d));
        return LBM_EINVAL;
    }
    if ((p->flags & LBM_BAROTROPIC) && !(p->T0_baro > 0)) { set_error("barotropic EOS needs T0_baro > 0"); return LBM_EINVAL; }
    if (p->walls != 0 && p->walls != 1) { set_error("walls must be 0 (periodic) or 1, got %d", p->walls); return LBM_EINVAL; }
    if (p->walls) {
        if (p->lattice != 19 || p->nz < 2) { set_error("walls need D3Q19 and nz >= 2"); return LBM_EINVAL; }
        if (((p->wall_heat & LBM_WALL_T_BOTTOM) && !(p->T_bottom > 0 && std::isfinite(p->T_bottom))) ||
            ((p->wall_heat & LBM_WALL_T_TOP) && !(p->T_top > 0 && std::isfinite(p->T_top)))) {
            set_error("a held wall temperature must be positive and finite");
            return LBM_EINVAL;
        }
        // a held wall face is half a cell from the node next to it, which doubles its conductance
        const double lim = 1.0 / (2 * (d < 1 ? 1 : d) + 1);
        if ((p->flags & LBM_CONDUCTION) && (p->wall_heat & (LBM_WALL_T_BOTTOM | LBM_WALL_T_TOP)) &&
            !(p->chi < lim)) {
            set_error("conduction next to a held wall needs chi < 1/(2d + 1) = %g", lim);
            return LBM_EINVAL;
        }
    }
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->gravity[a])) { set_error("gravity must be finite"); return LBM_EINVAL; }
    if (p->collision != LBM_COLLISION_BGK && p->collision != LBM_COLLISION_MRT) {
        set_error("collision must be LBM_COLLISION_BGK (0) or LBM_COLLISION_MRT (1), got %d", p->collision);
        return LBM_EINVAL;
    }
    if (p->collision == LBM_COLLISION_MRT) {
        const double r[4] = {p->s_e, p->s_eps, p->s_q, p->s_m};
        for (int i = 0; i < 4; ++i)
            if (!(r[i] > 0.0 && r[i] < 2.0)) { set_error("MRT rates must lie in (0, 2)"); return LBM_EINVAL; }
    }
    if (p->eos != LBM_EOS_VDW && p->eos != LBM_EOS_TABLE) {
        set_error("eos must be LBM_EOS_VDW (0) or LBM_EOS_TABLE (1), got %d", p->eos);
        return LBM_EINVAL;
    }
    if (p->eos == LBM_EOS_TABLE) {
        if (!p->eos_p || !p->eos_coex || p->eos_nrho < 4 || p->eos_nT < 2 ||
            (long long)p->eos_nrho * p->eos_nT > (1LL << 26)) {
            set_error("a tabulated EOS needs eos_p and eos_coex, eos_nrho >= 4, eos_nT >= 2 and at most 2^26 points");
            return LBM_EINVAL;
        }
        if (!(p->eos_rho_max > p->eos_rho_min && p->eos_rho_min >= 0.0 && std::isfinite(p->eos_rho_max)) ||
            !(p->eos_T_max > p->eos_T_min && p->eos_T_min > 0.0 && std::isfinite(p->eos_T_max))) {
            set_error("a tabulated EOS needs 0 <= eos_rho_min < eos_rho_max and 0 < eos_T_min < eos_T_max");
            return LBM_EINVAL;
        }
        for (long long i = 0; i < (long long)p->eos_nrho * p->eos_nT; ++i)
            if (!std::isfinite(p->eos_p[i])) { set_error("EOS table value %lld is not finite", i); return LBM_EINVAL; }
        for (int j = 0; j < p->eos_nT; ++j)
            if (!(p->eos_coex[2 * j] <= p->eos_coex[2 * j + 1]) || !std::isfinite(p->eos_coex[2 * j + 1])) {
                set_error("EOS coexistence row %d needs finite rho_1 <= rho_2", j);
                return LBM_EINVAL;
            }
    }
    // the step addresses nodes within one population plane with 32-bit byte offsets
    const long long n = plane_elements(*p);
    if ((unsigned long long)padded_plane(n) * (unsigned long long)p->storage_bytes >= (1ull << 32)) {
        set_error("one population plane of %lld elements exceeds 4 GB", n);
        return LBM_EINVAL;
    }
    if ((p->flags & LBM_LATENT) && !maxwell_table().ok) { set_error("Maxwell table construction failed"); return LBM_EDEVICE; }
    return LBM_OK;
}

lbm_status validate_fields(const lbm_params& p, const double* rho0, const double* u0, const double* T0)
{
    if (!rho0 || !u0 || !T0) { set_error("initial fields must not be NULL"); return LBM_EINVAL; }
    const long long n = (long long)p.nx * p.ny * p.nz;
    const Phys ph = make_phys(p);
    const double bound = 1.0 + kTheta;  // (h/dt)^2 + theta, section 3
    for (long long i = 0; i < n; ++i) {
        const double r = rho0[i], T = T0[i];
        if (!(r > 0) || !(r * ph.inv_rho_c < 3.0) || !(T > 0) || !std::isfinite(T)) {
            set_error("node %lld: need 0 < rho0 < 3 rho_c and T0 > 0 (rho0 = %g, T0 = %g)", i, r, T);
            return LBM_EINVAL;
        }
        if (!std::isfinite(u0[i]) || !std::isfinite(u0[n + i]) || !std::isfinite(u0[2 * n + i])) {
            set_error("node %lld: non-finite velocity", i);
            return LBM_EINVAL;
        }
        const double Te = (p.flags & LBM_BAROTROPIC) ? p.T0_baro : T;
        bool inside;
        const double pr = host_pressure(r, Te, ph, p.eos_p, inside);
        if (!inside) {
            set_error("node %lld: (rho, T) = (%g, %g) outside the EOS table", i, r, Te);
            return LBM_EINVAL;
        }
        if (!(r * kTheta - pr > 0)) {
            set_error("node %lld: Phi^2 = rho theta - p <= 0 (section 3)", i);
            return LBM_EINVAL;
        }
        const double dpdr = host_dp_drho(r, Te, ph, p.eos_p);
        if (dpdr > bound) {
            set_error("node %lld: (dp/drho)_T = %g exceeds the stability bound %g (section 3)", i, dpdr,
                      bound);
            return LBM_EINVAL;
        }
    }
    return LBM_OK;
}

// Launch geometry: tiles of the selected variant and z chunks sized so that one round of
// workgroups fills the GPU, unless a chunk length is given.
// The launch of the fused step for these parameters, launch variant and z-chunk request
// (0 = automatic) on a device with `cus` compute units; host arithmetic only.
StepGeom plan_geometry(const lbm_params& p, int variant, int chunk_request, int cus, int& tx, int& ty)
{
    int per_cu;
    step_tile(p.lattice, p.storage_bytes, variant, tx, ty, per_cu);
    StepGeom g{};
    g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
    g.pitch = row_pitch(p.nx, p.storage_bytes);
    g.plane = padded_plane(plane_elements(p));
    g.ntx = (p.nx + tx - 1) / tx;
    g.nty = (p.ny + ty - 1) / ty;
    int chunk = p.nz;
    // workgroups the device holds at once: the launch runs in rounds of this many, and the
    // kernel gives each round a contiguous band of tiles
    g.resident = cus * per_cu;
    if (p.lattice == 19) {
        // z chunks.  Each chunk runs the moment stage on 4 planes outside it (2 on each side),
        // and the launch runs in rounds of `target` workgroups (later ones start as earlier
        // ones retire), so a step takes about ceil(workgroups / target) x (chunk + 4) plane
        // times of one workgroup.  The chunk count minimising that is taken (the fewest
        // chunks among equals; chunks of at least 4 planes): a box whose columns do not fill
        // whole rounds gets more, shorter chunks (288^3: 162 columns, 3 chunks, 486
        // workgroups in two nearly full rounds, instead of 324 in one full and one quarter
        // round), and powers of two keep one round of long chunks.
        const long long cols = (long long)g.ntx * g.nty;
        const long long target = (long long)cus * per_cu;
        const long long maxc = p.nz / 4 > 0 ? p.nz / 4 : 1;
        long long best_cost = -1;
        for (long long nc = 1; nc <= maxc; ++nc) {
            const long long c = (p.nz + nc - 1) / nc;
            const long long chunks = (p.nz + c - 1) / c;
            const long long rounds = (cols * chunks + target - 1) / target;
            const long long cost = rounds * (c + 4);
            if (best_cost < 0 || cost < best_cost) {
                best_cost = cost;
                chunk = (int)c;
            }
        }
        if (chunk_request > 0) chunk = chunk_request < p.nz ? chunk_request : p.nz;
    }
    g.chunk = chunk;
    g.nchunks = (p.nz + chunk - 1) / chunk;
    return g;
}

// Variant lbm_init starts with: 7 (64 x 8 tiles, global addressing) for FP32 D3Q19 states
// beyond one buffer resource's 4 GB where 64-wide tiles leave no more x columns idle than
// 32-wide ones, else 0.
int default_variant(const lbm_params& p)
{
    if (p.lattice != 19 || p.storage_bytes != 4) return 0;
    if (state_bytes(p) < (1ull << 32)) return 0;
    const long long w64 = (p.nx + 63LL) / 64 * 64, w32 = (p.nx + 31LL) / 32 * 32;
    return w64 <= w32 ? 7 : 0;
}

void choose_geometry(lbm_sim* s, int chunk_request)
{
    int tx, ty;
    s->geom = plan_geometry(s->p, s->variant, chunk_request, s->cus, tx, ty);
    s->geom.plane = s->plane;
    s->tile_x = tx;
    s->tile_y = ty;
}

lbm_status upload_table(lbm_sim* s)
{
    const MaxwellTable& t = maxwell_table();
    hipError_t e = hipMalloc(&s->d_table, sizeof(double) * t.rho.size());
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(Maxwell table)");
    e = hipMemcpyAsync(s->d_table, t.rho.data(), sizeof(double) * t.rho.size(), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "upload Maxwell table");
    s->aux.maxwell = s->d_table;
    s->aux.tab_s0 = t.s0;
    s->aux.tab_inv_ds = 1.0 / t.ds;
    return LBM_OK;
}

lbm_status enqueue_steps(lbm_sim* s, int nsteps)
{
    if (!s->aux.err || !s->aux.maxwell || !s->buf[0] || !s->buf[1]) {
        set_error("simulation is not fully initialised (null device pointer)");
        return LBM_EDEVICE;
    }
    for (int i = 0; i < nsteps; ++i) {
        hipError_t e = launch_step(s->p.lattice, s->p.storage_bytes, s->variant, s->buf[s->cur],
                                   s->buf[1 - s->cur], s->geom, s->phys, s->aux, s->stream);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        s->cur ^= 1;
        s->step += 1;
    }
    return LBM_OK;
}

lbm_status read_error_word(lbm_sim* s)
{
    int h = 0;
    hipError_t e = hipMemcpyAsync(&h, s->d_err, sizeof(int), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "reading the device error word");
    if (h) {
        set_error("a node left the EOS domain (Phi^2 <= 0, rho >= 3 rho_c or non-finite) by step %lld", s->step);
        return LBM_EUNSTABLE;
    }
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" {

const char* lbm_last_error(void) { return g_last_error; }

size_t lbm_footprint_bytes(const lbm_params* p)
{
    if (!p) return 0;
    size_t tables = sizeof(double) * 2 * kMaxwellPoints + 64;
    if (p->eos == LBM_EOS_TABLE && p->eos_nrho > 0 && p->eos_nT > 0)
        tables += sizeof(double) * ((size_t)p->eos_nrho * p->eos_nT + 2 * (size_t)p->eos_nT);
    return 2 * state_bytes(*p) + tables;
}

int lbm_lattice_info(int Q, int* c, double* w, double* G, double* alpha)
{
    if (Q == 9) {
        for (int k = 0; k < 9; ++k) {
            c[3 * k] = Lattice<9>::cx[k]; c[3 * k + 1] = Lattice<9>::cy[k]; c[3 * k + 2] = Lattice<9>::cz[k];
            w[k] = weight<9>(k); G[k] = force_coef<9>(k);
        }
        *alpha = Lattice<9>::alpha;
        return 2;
    }
    if (Q == 19) {
        for (int k = 0; k < 19; ++k) {
            c[3 * k] = Lattice<19>::cx[k]; c[3 * k + 1] = Lattice<19>::cy[k]; c[3 * k + 2] = Lattice<19>::cz[k];
            w[k] = weight<19>(k); G[k] = force_coef<19>(k);
        }
        *alpha = Lattice<19>::alpha;
        return 3;
    }
    return LBM_EINVAL;
}

lbm_status lbm_coexistence(double Tr, double* rho_v, double* rho_l)
{
    double rv, rl;
    if (!host_band_limits(Tr, rv, rl)) {
        set_error("reduced temperature %g outside the Maxwell table [%g, %g]", Tr, kLatentTmin, kLatentTmax);
        return LBM_EINVAL;
    }
    if (rho_v) *rho_v = rv;
    if (rho_l) *rho_l = rl;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_params* params, const double* rho0, const double* u0, const double* T0,
                    void* stream, lbm_sim** out)
{
    clear_error();
    if (!out) { set_error("out is NULL"); return LBM_EINVAL; }
    *out = nullptr;
    lbm_status st = validate_params(params);
    if (st != LBM_OK) return st;
    st = validate_fields(*params, rho0, u0, T0);
    if (st != LBM_OK) return st;

    lbm_sim* s = new lbm_sim();
    s->p = *params;
    s->phys = make_phys(*params);
    s->n = (long long)params->nx * params->ny * params->nz;
    s->plane = padded_plane(plane_elements(s->p));
    if (hipError_t e = hipGetDevice(&s->device); e != hipSuccess) {
        delete s;
        return hip_fail(e, "hipGetDevice");
    }
    if (hipError_t e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device);
        e != hipSuccess || s->cus < 1) {
        delete s;
        return hip_fail(e == hipSuccess ? hipErrorInvalidDevice : e, "compute unit count");
    }
    if (stream) {
        s->stream = (hipStream_t)stream;
        s->own_stream = false;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { delete s; return hip_fail(e, "hipStreamCreate"); }
        s->own_stream = true;
    }
    s->variant = default_variant(s->p);
    choose_geometry(s, 0);
    const size_t bytes = state_bytes(s->p);
    hipError_t e = hipMalloc(&s->buf[0], bytes);
    if (e == hipSuccess) e = hipMalloc(&s->buf[1], bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_err, sizeof(int) * 16);
    s->red_blocks = reduce_blocks(s->n);
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_partials, sizeof(double) * (5 * s->red_blocks + 8));
    if (e != hipSuccess) { lbm_status r = hip_fail(e, "hipMalloc(state)"); lbm_free(s); return r; }
    s->aux.err = s->d_err;
    e = hipMemsetAsync(s->d_err, 0, sizeof(int) * 16, s->stream);
    // zero padding so checkpoints are deterministic
    if (e == hipSuccess) e = hipMemsetAsync(s->buf[0], 0, bytes, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->buf[1], 0, bytes, s->stream);
    if (e != hipSuccess) { lbm_status r = hip_fail(e, "clear state"); lbm_free(s); return r; }
    st = upload_table(s);
    if (st != LBM_OK) { lbm_free(s); return st; }
    if (s->phys.eos) {
        // the simulation keeps its own device copy of the caller's tables
        const size_t np = (size_t)params->eos_nrho * params->eos_nT, nc = 2 * (size_t)params->eos_nT;
        e = hipMalloc((void**)&s->d_eos_p, sizeof(double) * np);
        if (e == hipSuccess) e = hipMalloc((void**)&s->d_eos_coex, sizeof(double) * nc);
        if (e == hipSuccess) e = hipMemcpy(s->d_eos_p, params->eos_p, sizeof(double) * np, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(s->d_eos_coex, params->eos_coex, sizeof(double) * nc, hipMemcpyHostToDevice);
        if (e != hipSuccess) { lbm_status r = hip_fail(e, "EOS table upload"); lbm_free(s); return r; }
    }
    s->aux.eos_p = s->d_eos_p;
    s->aux.eos_coex = s->d_eos_coex;
    s->aux.partials = nullptr;   // set by the steps that form the totals
    // the caller's table pointers are not kept
    s->p.eos_p = nullptr;
    s->p.eos_coex = nullptr;

    double* d_fields = nullptr;
    e = hipMalloc((void**)&d_fields, sizeof(double) * 5 * s->n);
    if (e != hipSuccess) { lbm_status r = hip_fail(e, "hipMalloc(initial fields)"); lbm_free(s); return r; }
    e = hipMemcpyAsync(d_fields, rho0, sizeof(double) * s->n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_fields + s->n, u0, sizeof(double) * 3 * s->n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_fields + 4 * s->n, T0, sizeof(double) * s->n, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = launch_init(s->p.lattice, s->p.storage_bytes, s->buf[0], d_fields, d_fields + s->n, d_fields + 4 * s->n,
                        s->p.nx, s->p.ny, s->p.nz, s->geom.pitch, s->plane, s->p.c_v, s->p.walls, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d_fields);
    if (e != hipSuccess) { lbm_status r = hip_fail(e, "initial state"); lbm_free(s); return r; }
    s->cur = 0;
    s->step = 0;
    *out = s;
    return LBM_OK;
}

lbm_status lbm_step_async(lbm_sim* s, int nsteps)
{
    clear_error();
    if (!s || nsteps < 0) { set_error("bad simulation handle or step count"); return LBM_EINVAL; }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    return enqueue_steps(s, nsteps);
}

lbm_status lbm_check(lbm_sim* s)
{
    clear_error();
    if (!s) { set_error("simulation is NULL"); return LBM_EINVAL; }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    return read_error_word(s);
}

lbm_status lbm_step(lbm_sim* s, int nsteps)
{
    lbm_status st = lbm_step_async(s, nsteps);
    if (st != LBM_OK) return st;
    return read_error_word(s);
}

long long lbm_step_count(const lbm_sim* s) { return s ? s->step : -1; }

lbm_status lbm_set_launch(lbm_sim* s, int variant, int chunk)
{
    clear_error();
    if (!s) { set_error("simulation is NULL"); return LBM_EINVAL; }
    if (variant < 0 || variant >= step_variants(s->p.lattice, s->p.storage_bytes) || chunk < 0) {
        set_error("launch variant %d / chunk %d not available for this lattice and storage", variant, chunk);
        return LBM_EINVAL;
    }
    s->variant = variant;
    choose_geometry(s, chunk);
    return LBM_OK;
}

lbm_status lbm_launch_plan(const lbm_params* p, int cus, int info[4])
{
    clear_error();
    if (!p || !info || cus < 1) { set_error("NULL argument or compute-unit count below 1"); return LBM_EINVAL; }
    if (!((p->lattice == 9 && p->nz == 1) || p->lattice == 19) ||
        (p->storage_bytes != 4 && p->storage_bytes != 8) || p->nx < 1 || p->ny < 1 || p->nz < 1) {
        set_error("lattice, storage or shape not supported");
        return LBM_EINVAL;
    }
    int tx, ty;
    const StepGeom g = plan_geometry(*p, default_variant(*p), 0, cus, tx, ty);
    info[0] = tx;
    info[1] = ty;
    info[2] = g.chunk;
    info[3] = g.ntx * g.nty * g.nchunks;
    return LBM_OK;
}

lbm_status lbm_launch_info(const lbm_sim* s, int info[4])
{
    if (!s || !info) { set_error("NULL argument"); return LBM_EINVAL; }
    info[0] = s->tile_x;
    info[1] = s->tile_y;
    info[2] = s->geom.chunk;
    info[3] = s->geom.ntx * s->geom.nty * s->geom.nchunks;
    return LBM_OK;
}

static lbm_status ensure_scratch(lbm_sim* s)
{
    if (s->d_scratch) return LBM_OK;
    hipError_t e = hipMalloc((void**)&s->d_scratch, sizeof(double) * 10 * s->n);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(moment scratch)");
    return LBM_OK;
}

lbm_status lbm_moments_device(lbm_sim* s, double* rho, double* u_star, double* E, double* T)
{
    clear_error();
    if (!s) { set_error("simulation is NULL"); return LBM_EINVAL; }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    lbm_status st = ensure_scratch(s);
    if (st != LBM_OK) return st;
    hipError_t e = launch_moments(s->p.lattice, s->p.storage_bytes, s->buf[s->cur], s->d_scratch, s->p.nx,
                                  s->p.ny, s->p.nz, s->geom.pitch, s->plane, s->phys, s->aux.eos_p, s->d_err, rho,
                                  u_star, E, T, s->stream);
    if (e != hipSuccess) return hip_fail(e, "moments launch");
    return LBM_OK;
}

lbm_status lbm_moments(lbm_sim* s, double* rho, double* u_star, double* E, double* T)
{
    clear_error();
    if (!s) { set_error("simulation is NULL"); return LBM_EINVAL; }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    lbm_status st = ensure_scratch(s);
    if (st != LBM_OK) return st;
    const long long n = s->n;
    double* scr = s->d_scratch;
    double* d_us = scr + 7 * n;
    hipError_t e = launch_moments(s->p.lattice, s->p.storage_bytes, s->buf[s->cur], scr, s->p.nx, s->p.ny,
                                  s->p.nz, s->geom.pitch, s->plane, s->phys, s->aux.eos_p, s->d_err, nullptr,
                                  u_star ? d_us : nullptr, nullptr, nullptr, s->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, scr, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && u_star) e = hipMemcpyAsync(u_star, d_us, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && E) e = hipMemcpyAsync(E, scr + 4 * n, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && T) e = hipMemcpyAsync(T, scr + 5 * n, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "moments");
    return read_error_word(s);
}

lbm_status lbm_reduce(lbm_sim* s, double out[5])
{
    clear_error();
    if (!s || !out) { set_error("NULL argument"); return LBM_EINVAL; }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    double* d_out = s->d_partials + 5 * s->red_blocks;
    // the padding of the rows is zero (cleared at init, never written by the step)
    hipError_t e = launch_reduce(s->p.lattice, s->p.storage_bytes, s->buf[s->cur], plane_elements(s->p), s->plane,
                                 s->d_partials, s->red_blocks, d_out, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, sizeof(double) * 5, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "reduction");
    return LBM_OK;
}

lbm_status lbm_step_reduce(lbm_sim* s, int nsteps, double out[5])
{
    clear_error();
    if (!s || !out || nsteps < 1) {
        set_error("bad simulation handle, NULL output or step count below 1");
        return LBM_EINVAL;
    }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    lbm_status st = enqueue_steps(s, nsteps - 1);
    if (st != LBM_OK) return st;
    // the last step's partial totals (5 per workgroup) and the totals, grown on demand
    const long long wg = step_workgroups(s->geom);
    if (5 * wg + 8 > s->step_partials_len) {
        if (s->d_step_partials) {
            hipError_t e = hipFree(s->d_step_partials);
            s->d_step_partials = nullptr;
            s->step_partials_len = 0;
            if (e != hipSuccess) return hip_fail(e, "hipFree(step partials)");
        }
        hipError_t e = hipMalloc((void**)&s->d_step_partials, sizeof(double) * (5 * wg + 8));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(step partials)");
        s->step_partials_len = 5 * wg + 8;
    }
    double* d_out = s->d_step_partials + 5 * wg;
    StepAux aux = s->aux;
    aux.partials = s->d_step_partials;
    hipError_t e = launch_step_totals(s->p.lattice, s->p.storage_bytes, s->variant, s->buf[s->cur],
                                      s->buf[1 - s->cur], s->geom, s->phys, aux, d_out, s->stream);
    if (e == hipErrorNotSupported) {
        // a launch variant without the fused form: the plain step, then the separate reduction
        st = enqueue_steps(s, 1);
        if (st != LBM_OK) return st;
        e = launch_reduce(s->p.lattice, s->p.storage_bytes, s->buf[s->cur], plane_elements(s->p), s->plane,
                          s->d_partials, s->red_blocks, d_out, s->stream);
        if (e != hipSuccess) return hip_fail(e, "reduction");
    } else if (e != hipSuccess) {
        return hip_fail(e, "step launch");
    } else {
        s->cur ^= 1;
        s->step += 1;
    }
    e = hipMemcpyAsync(out, d_out, sizeof(double) * 5, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "reading the totals");
    return read_error_word(s);
}

struct CheckpointHeader {
    char magic[8];
    int lattice, nx, ny, nz, storage_bytes, pitch;   // pitch: x row pitch of the layout, in elements
    long long step;
    long long bytes;
};

lbm_status lbm_checkpoint(lbm_sim* s, void* host_buf, size_t cap, size_t* used)
{
    clear_error();
    if (!s || !used) { set_error("NULL argument"); return LBM_EINVAL; }
    const size_t bytes = state_bytes(s->p);
    *used = sizeof(CheckpointHeader) + bytes;
    if (!host_buf) return LBM_OK;
    if (cap < *used) { set_error("checkpoint buffer too small (%zu < %zu)", cap, *used); return LBM_EINVAL; }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    CheckpointHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, "LBMCKPT2", 8);
    h.lattice = s->p.lattice; h.nx = s->p.nx; h.ny = s->p.ny; h.nz = s->p.nz;
    h.storage_bytes = s->p.storage_bytes; h.pitch = s->geom.pitch; h.step = s->step; h.bytes = (long long)bytes;
    memcpy(host_buf, &h, sizeof(h));
    hipError_t e = hipMemcpyAsync((char*)host_buf + sizeof(h), s->buf[s->cur], bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
    return LBM_OK;
}

lbm_status lbm_restore(lbm_sim* s, const void* host_buf, size_t len)
{
    clear_error();
    if (!s || !host_buf) { set_error("NULL argument"); return LBM_EINVAL; }
    CheckpointHeader h;
    if (len < sizeof(h)) { set_error("checkpoint too short"); return LBM_EINVAL; }
    memcpy(&h, host_buf, sizeof(h));
    const size_t bytes = state_bytes(s->p);
    if (memcmp(h.magic, "LBMCKPT2", 8) != 0 || h.lattice != s->p.lattice || h.nx != s->p.nx || h.ny != s->p.ny ||
        h.nz != s->p.nz || h.storage_bytes != s->p.storage_bytes || h.pitch != s->geom.pitch ||
        h.bytes != (long long)bytes ||
        len < sizeof(h) + bytes) {
        set_error("checkpoint does not match this simulation's lattice, shape or storage");
        return LBM_EINVAL;
    }
    if (lbm_status sd = use_device(s->device); sd != LBM_OK) return sd;
    hipError_t e = hipMemcpyAsync(s->buf[s->cur], (const char*)host_buf + sizeof(h), bytes, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_err, 0, sizeof(int), s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "restore copy");
    s->step = h.step;
    return LBM_OK;
}

lbm_status lbm_free(lbm_sim* s)
{
    if (!s) return LBM_OK;
    // release everything even if the device reports an error: nothing here can be retried
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->buf[0]) (void)hipFree(s->buf[0]);
    if (s->buf[1]) (void)hipFree(s->buf[1]);
    if (s->d_err) (void)hipFree(s->d_err);
    if (s->d_partials) (void)hipFree(s->d_partials);
    if (s->d_step_partials) (void)hipFree(s->d_step_partials);
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->d_scratch) (void)hipFree(s->d_scratch);
    if (s->d_eos_p) (void)hipFree(s->d_eos_p);
    if (s->d_eos_coex) (void)hipFree(s->d_eos_coex);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return LBM_OK;
}

}  // extern "C"

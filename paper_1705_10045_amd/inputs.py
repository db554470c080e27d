"""Seeded synthetic inputs for the thermal multiphase LBM workloads.

This module is pure data generation: geometry masks, counter-based random
numbers and parameter sets.  It holds none of the method's arithmetic and is
the only module shared by the HIP product path and the FP64 oracle.

Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) evaluated on the counter (seed, node index),
so a field depends only on the seed and the node, never on the order of
generation.  Uniform variates take the top 53 bits; Gaussian variates use the
Box-Muller transform of the uniforms at counters 2i and 2i+1.

Physical setting (lattice units h = dt = 1): periodic boxes, the reduced van der
Waals fluid with critical values (rho_c, T_c, p_c), liquid/vapour initial
states at the coexistence densities of the table below joined by a tanh profile
of about the equilibrium interface width (a voxel-sharp step drives the first
steps far outside the equation of state's domain), temperature uniform.
"""
import numpy as np

# --------------------------------------------------------------------------
# Counter-based random numbers
# --------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, counters):
    """SplitMix64 output for state seed*golden + (counter+1)*golden (uint64 array)."""
    with np.errstate(over="ignore"):
        c = np.asarray(counters, dtype=np.uint64)
        z = np.uint64(seed) * _GOLDEN + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed, n, offset=0):
    """n variates in [0, 1) from counters offset .. offset+n-1."""
    bits = splitmix64(seed, np.arange(offset, offset + n, dtype=np.uint64))
    return (bits >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def symmetric(seed, n, offset=0):
    """n variates uniform in [-1, 1)."""
    return 2.0 * uniform(seed, n, offset) - 1.0


def gaussian(seed, n, offset=0):
    """n standard normal variates (Box-Muller on counter pairs)."""
    u = uniform(seed, 2 * n, 2 * offset).reshape(n, 2)
    u1 = 1.0 - u[:, 0]  # in (0, 1]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u[:, 1])


# --------------------------------------------------------------------------
# Coexistence densities of the reduced van der Waals fluid (data)
# --------------------------------------------------------------------------
# (T~, rho~_vapour, rho~_liquid), equal-area rule, 9 significant digits.  Used
# only to place the initial liquid and vapour densities; the test suite checks
# the table against the oracle's Maxwell solver.
COEXISTENCE = np.array([
    (0.60, 0.059778111, 2.311556529), (0.61, 0.065078624, 2.295675967),
    (0.62, 0.070688219, 2.279549167), (0.63, 0.076617053, 2.263167043),
    (0.64, 0.082875729, 2.246519932), (0.65, 0.089475357, 2.229597536),
    (0.66, 0.096427633, 2.212388856), (0.67, 0.103744915, 2.194882124),
    (0.68, 0.111440313, 2.177064718), (0.69, 0.119527796, 2.158923068),
    (0.70, 0.128022302, 2.140442549), (0.71, 0.136939867, 2.121607355),
    (0.72, 0.146297779, 2.102400360), (0.73, 0.156114746, 2.082802951),
    (0.74, 0.166411095, 2.062794834), (0.75, 0.177209006, 2.042353804),
    (0.76, 0.188532783, 2.021455484), (0.77, 0.200409175, 2.000072998),
    (0.78, 0.212867766, 1.978176600), (0.79, 0.225941437, 1.955733202),
    (0.80, 0.239666922, 1.932705829), (0.81, 0.254085506, 1.909052920),
    (0.82, 0.269243872, 1.884727490), (0.83, 0.285195167, 1.859676058),
    (0.84, 0.302000358, 1.833837303), (0.85, 0.319729965, 1.807140327),
    (0.86, 0.338466322, 1.779502398), (0.87, 0.358306586, 1.750825942),
    (0.88, 0.379366793, 1.720994492), (0.89, 0.401787477, 1.689867068),
    (0.90, 0.425741638, 1.657270212), (0.91, 0.451446397, 1.622986331),
    (0.92, 0.479180675, 1.586736027), (0.93, 0.509313189, 1.548150093),
    (0.94, 0.542349288, 1.506722684), (0.95, 0.579014927, 1.461727344),
    (0.96, 0.620421780, 1.412051891), (0.97, 0.668436809, 1.355828851),
    (0.98, 0.726691333, 1.289426391), (0.99, 0.804535449, 1.203493895),
])


def coexistence(Tr):
    """Tabulated reduced (rho_v, rho_l) at Tr; linear between table rows
    (initial-state placement only)."""
    T = COEXISTENCE[:, 0]
    if not (T[0] - 1e-12 <= Tr <= T[-1] + 1e-12):
        raise ValueError("reduced temperature %.4f outside the table [0.60, 0.99]" % Tr)
    return (float(np.interp(Tr, T, COEXISTENCE[:, 1])),
            float(np.interp(Tr, T, COEXISTENCE[:, 2])))


# --------------------------------------------------------------------------
# Parameter sets
# --------------------------------------------------------------------------
WORK, CONDUCTION, LATENT, PSEUDOFORCE, BAROTROPIC = 1, 2, 4, 8, 16
ALL_TERMS = WORK | CONDUCTION | LATENT | PSEUDOFORCE

P_C = 0.02  # critical pressure in lattice units (rho_c = T_c = 1)


def physics(**overrides):
    """Default physical parameters (lattice units) with overrides."""
    p = dict(tau=1.0, tau_E=0.53, A=-0.152, rho_c=1.0, T_c=1.0, p_c=P_C,
             c_v=4.0 * P_C, chi=0.01, rhoQ=0.02 * P_C, T0_baro=0.0, flags=ALL_TERMS)
    p.update(overrides)
    return p


# --------------------------------------------------------------------------
# Geometries
# --------------------------------------------------------------------------
def _grid(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def slab_distance(shape, width, axis=0):
    """Signed distance to the faces of a centred slab of the given width normal to
    `axis` (0 = x, 1 = y, 2 = z): negative inside, positive outside."""
    coords = _grid(shape)[axis]
    n = shape[2 - axis]
    return np.abs(coords - (n - 1) / 2.0) - width / 2.0


def sphere_distance(shape, radius, center=None):
    """Signed distance to a centred sphere (a disc if nz == 1): negative inside."""
    nz, ny, nx = shape
    x, y, z = _grid(shape)
    if center is None:
        center = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    r2 = (x - center[0]) ** 2 + (y - center[1]) ** 2
    if nz > 1:
        r2 = r2 + (z - center[2]) ** 2
    return np.sqrt(r2) - radius


def slab_mask(shape, width, axis=0):
    return slab_distance(shape, width, axis) < 0


def sphere_mask(shape, radius, center=None):
    return sphere_distance(shape, radius, center) < 0


def two_phase(mask, rho_liquid, rho_vapour):
    """Sharp liquid/vapour step on a boolean mask."""
    return np.where(mask, rho_liquid, rho_vapour).astype(np.float64)


INTERFACE_WIDTH = 3.0


def two_phase_smooth(distance, rho_liquid, rho_vapour, width=INTERFACE_WIDTH):
    """Liquid where distance < 0, vapour outside, joined by the profile
    rho_v + (rho_l - rho_v) (1 - tanh(d / width)) / 2."""
    s = 0.5 * (1.0 - np.tanh(distance / width))
    return (rho_vapour + (rho_liquid - rho_vapour) * s).astype(np.float64)


def with_uniform_noise(rho, seed, amplitude):
    """rho * (1 + amplitude * xi), xi ~ U[-1, 1) per node."""
    return rho * (1.0 + amplitude * symmetric(seed, rho.size).reshape(rho.shape))


def with_gaussian_noise(rho, seed, sigma):
    """rho * (1 + sigma * N(0,1)) per node."""
    return rho * (1.0 + sigma * gaussian(seed, rho.size).reshape(rho.shape))


def uniform_velocity(shape, u):
    out = np.zeros((3,) + tuple(shape))
    for a in range(3):
        out[a] = u[a]
    return out


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
SEED = 1705


def slab_2d(n=128, width=40, Tr=0.85, noise=0.01, seed=SEED, params=None):
    """D2Q9 liquid slab (normal along x) in vapour, uniform temperature, at rest."""
    shape = (1, n, n)
    rv, rl = coexistence(Tr)
    p = params or physics()
    rho = two_phase_smooth(slab_distance(shape, width, axis=0), rl * p["rho_c"], rv * p["rho_c"])
    rho = with_uniform_noise(rho, seed, noise)
    return dict(Q=9, params=p, rho0=rho, u0=uniform_velocity(shape, (0, 0, 0)),
                T0=np.full(shape, Tr * p["T_c"]))


def droplet_3d(n=128, radius=24.0, Tr=0.8, noise=0.005, velocity=(0.05, 0.0, 0.0), seed=SEED,
               params=None, shape=None):
    """D3Q19 liquid sphere in vapour moving with a uniform velocity."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    rv, rl = coexistence(Tr)
    p = params or physics()
    rho = two_phase_smooth(sphere_distance(shape, radius), rl * p["rho_c"], rv * p["rho_c"])
    rho = with_uniform_noise(rho, seed, noise)
    return dict(Q=19, params=p, rho0=rho, u0=uniform_velocity(shape, velocity),
                T0=np.full(shape, Tr * p["T_c"]))


def spinodal_3d(n=256, Tr=0.75, rho_mean=1.0, sigma=0.02, seed=SEED, params=None, shape=None):
    """D3Q19 uniform fluid inside the spinodal with Gaussian density noise, at rest."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    p = params or physics()
    rho = with_gaussian_noise(np.full(shape, rho_mean * p["rho_c"]), seed, sigma)
    return dict(Q=19, params=p, rho0=rho, u0=uniform_velocity(shape, (0, 0, 0)),
                T0=np.full(shape, Tr * p["T_c"]))


def layer_distance(shape, height):
    """Signed distance to the top of a layer filling the planes z < height above a wall at
    z = -1/2 (negative inside the layer)."""
    z = _grid(shape)[2]
    return z - (height - 0.5)


WALL_T_BOTTOM = 1
WALL_T_TOP = 2


def pool_boiling_3d(n=512, fill=0.6, Tr=0.8, T_bottom_r=0.9, T_top_r=0.7, gravity=1e-5,
                    noise=0.01, seed=SEED, params=None, shape=None):
    """D3Q19 pool boiling: walls normal to z (bottom held at T_bottom_r T_c, above the
    saturation temperature of the layer; top held at T_top_r T_c), gravity along -z, a liquid
    layer filling the lower `fill` of the box under its vapour at the coexistence densities of
    Tr, +-noise uniform density noise, temperature Tr T_c, at rest."""
    shape = tuple(shape) if shape is not None else (n, n, n)
    p = dict(params or physics())
    p.update(walls=1, wall_heat=WALL_T_BOTTOM | WALL_T_TOP, T_bottom=T_bottom_r * p["T_c"],
             T_top=T_top_r * p["T_c"], gravity=(0.0, 0.0, -gravity))
    rv, rl = coexistence(Tr)
    rho = two_phase_smooth(layer_distance(shape, fill * shape[0]), rl * p["rho_c"],
                           rv * p["rho_c"])
    rho = with_uniform_noise(rho, seed, noise)
    return dict(Q=19, params=p, rho0=rho, u0=uniform_velocity(shape, (0, 0, 0)),
                T0=np.full(shape, Tr * p["T_c"]))


SERVING_EDGES = (32, 48, 64, 96, 128)


def serving_requests(count=512, seed=SEED, edges=SERVING_EDGES, t_range=(0.70, 0.95),
                     steps_range=(500, 5000), noise=0.01):
    """Request descriptors of the serving stream: lattice edge, reduced temperature,
    droplet or slab, step count.  Fields are built on demand by `request_fields`."""
    u = uniform(seed + 1, 4 * count).reshape(count, 4)
    reqs = []
    for i in range(count):
        edge = int(edges[min(int(u[i, 0] * len(edges)), len(edges) - 1)])
        Tr = round(t_range[0] + (t_range[1] - t_range[0]) * u[i, 1], 6)
        kind = "droplet" if u[i, 2] < 0.5 else "slab"
        lo, hi = steps_range
        steps = int(lo + min(int(u[i, 3] * (hi - lo + 1)), hi - lo))
        reqs.append(dict(id=i, edge=edge, Tr=Tr, kind=kind, steps=steps, seed=seed + 1 + i,
                         noise=noise))
    return reqs


def request_fields(req, params=None):
    """Initial fields of one serving request (D3Q19, periodic cube of edge L)."""
    L = req["edge"]
    shape = (L, L, L)
    p = params or physics()
    rv, rl = coexistence(req["Tr"])
    if req["kind"] == "droplet":
        dist = sphere_distance(shape, round(0.1875 * L))
    else:
        dist = slab_distance(shape, round(0.3125 * L), axis=0)
    rho = with_uniform_noise(two_phase_smooth(dist, rl * p["rho_c"], rv * p["rho_c"]),
                             req["seed"], req["noise"])
    return dict(Q=19, params=p, rho0=rho, u0=uniform_velocity(shape, (0, 0, 0)),
                T0=np.full(shape, req["Tr"] * p["T_c"]))

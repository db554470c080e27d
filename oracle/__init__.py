"""FP64 CPU oracle of the thermal multiphase lattice Boltzmann method (arXiv:1705.10045).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP product library; the two meet only through the seeded inputs of
``paper_1705_10045_amd.inputs`` (pure data generation, none of the method's
arithmetic).

Field arrays are numpy float64 of shape (nz, ny, nx) (x fastest); vector fields
are (3, nz, ny, nx).  Populations are returned k-major, shape (Q, nz, ny, nx).
"""
import ctypes
import os

import numpy as np

from . import build as _build

WORK = 1
CONDUCTION = 2
LATENT = 4
PSEUDOFORCE = 8
BAROTROPIC = 16
ALL_TERMS = WORK | CONDUCTION | LATENT | PSEUDOFORCE

BGK = 0
MRT = 1

EOS_VDW = 0
EOS_TABLE = 1

WALL_T_BOTTOM = 1
WALL_T_TOP = 2

OK = 0
EINVAL = -1
EUNSTABLE = -3


class _Params(ctypes.Structure):
    _fields_ = [
        ("Q", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("tau", ctypes.c_double), ("tau_E", ctypes.c_double), ("A", ctypes.c_double),
        ("rho_c", ctypes.c_double), ("T_c", ctypes.c_double), ("p_c", ctypes.c_double),
        ("c_v", ctypes.c_double), ("chi", ctypes.c_double), ("rhoQ", ctypes.c_double),
        ("T0_baro", ctypes.c_double), ("flags", ctypes.c_uint),
        ("walls", ctypes.c_int), ("wall_heat", ctypes.c_uint),
        ("T_bottom", ctypes.c_double), ("T_top", ctypes.c_double),
        ("gravity", ctypes.c_double * 3),
        ("collision", ctypes.c_int),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double), ("s_q", ctypes.c_double),
        ("s_m", ctypes.c_double),
        ("eos", ctypes.c_int),
        ("eos_p", ctypes.POINTER(ctypes.c_double)), ("eos_coex", ctypes.POINTER(ctypes.c_double)),
        ("eos_nrho", ctypes.c_int), ("eos_nT", ctypes.c_int),
        ("eos_rho_min", ctypes.c_double), ("eos_rho_max", ctypes.c_double),
        ("eos_T_min", ctypes.c_double), ("eos_T_max", ctypes.c_double),
    ]


_LIB = None
_D = ctypes.POINTER(ctypes.c_double)


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        lib.orc_vdw_reduced.restype = ctypes.c_double
        lib.orc_vdw_reduced.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_table_reduced.restype = ctypes.c_double
        lib.orc_table_reduced.argtypes = [ctypes.POINTER(_Params), ctypes.c_double,
                                          ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        lib.orc_maxwell.argtypes = [ctypes.c_double, _D, _D, _D]
        lib.orc_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D, _D, _D]
        lib.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, _D, _D]
        lib.orc_mrt_basis.argtypes = [ctypes.c_int, _D, _D, ctypes.POINTER(ctypes.c_int)]
        lib.orc_force.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double, _D, _D]
        lib.orc_divergence.argtypes = [ctypes.c_int] * 4 + [_D, _D]
        lib.orc_conduction.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 2 + [_D, _D, _D]
        lib.orc_force_walls.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double, _D, _D]
        lib.orc_divergence_walls.argtypes = [ctypes.c_int] * 3 + [_D, _D]
        lib.orc_conduction_walls.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 2 + \
            [_D, _D, ctypes.c_uint, ctypes.c_double, ctypes.c_double, _D]
        lib.orc_create.restype = ctypes.c_void_p
        lib.orc_create.argtypes = [ctypes.POINTER(_Params), _D, _D, _D,
                                   ctypes.POINTER(ctypes.c_int)]
        lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        lib.orc_moments.argtypes = [ctypes.c_void_p, _D, _D, _D, _D]
        lib.orc_totals.argtypes = [ctypes.c_void_p, _D]
        lib.orc_last_sources.argtypes = [ctypes.c_void_p, _D, _D, _D]
        lib.orc_get_pops.argtypes = [ctypes.c_void_p, _D, _D]
        lib.orc_set_pops.argtypes = [ctypes.c_void_p, _D, _D]
        lib.orc_step_count.restype = ctypes.c_longlong
        lib.orc_step_count.argtypes = [ctypes.c_void_p]
        lib.orc_free.argtypes = [ctypes.c_void_p]
        _LIB = lib
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice(Q):
    """(c[Q,3] int, w[Q], G[Q], alpha, D) of the oracle's velocity set."""
    c = (ctypes.c_int * (3 * Q))()
    w = np.zeros(Q)
    G = np.zeros(Q)
    alpha = ctypes.c_double()
    D = _lib().orc_lattice(Q, c, _ptr(w), _ptr(G), ctypes.byref(alpha))
    if D < 0:
        raise ValueError("unsupported lattice Q=%d" % Q)
    return np.array(list(c), dtype=np.int64).reshape(Q, 3), w, G, alpha.value, D


def mrt_basis(Q):
    """(M[Q,Q], squared row norms[Q], group[Q]) of the MRT moment basis, rows in the oracle's
    velocity order; groups 0 conserved, 1 shear, 2 energy, 3 energy square and fourth order,
    4 energy flux, 5 third order."""
    M = np.zeros(Q * Q)
    n2 = np.zeros(Q)
    grp = (ctypes.c_int * Q)()
    if _lib().orc_mrt_basis(Q, _ptr(M), _ptr(n2), grp) != OK:
        raise ValueError("no MRT basis for Q=%d" % Q)
    return M.reshape(Q, Q), n2, np.array(list(grp))


def vdw_reduced(rr, Tr):
    return _lib().orc_vdw_reduced(float(rr), float(Tr))


def _table_fields(p, table):
    """Set the tabulated-EOS fields of a _Params from a dict with keys p (nT x nrho reduced
    pressures), coex (nT x 2 reduced band limits), rho_range and T_range; returns the arrays,
    which must stay alive while p is used."""
    tp = np.ascontiguousarray(table["p"], dtype=np.float64)
    tc = np.ascontiguousarray(table["coex"], dtype=np.float64)
    if tp.ndim != 2 or tc.shape != (tp.shape[0], 2):
        raise ValueError("table p must be (nT, nrho) and coex (nT, 2)")
    p.eos = EOS_TABLE
    p.eos_p = _ptr(tp)
    p.eos_coex = _ptr(tc)
    p.eos_nT, p.eos_nrho = tp.shape
    p.eos_rho_min, p.eos_rho_max = (float(v) for v in table["rho_range"])
    p.eos_T_min, p.eos_T_max = (float(v) for v in table["T_range"])
    return tp, tc


def table_reduced(table, rr, Tr):
    """Reduced pressure of a tabulated EOS (dict as for Sim's params["eos_table"]) at (rr, Tr),
    or None outside its grid."""
    p = _Params()
    keep = _table_fields(p, table)
    inside = ctypes.c_int()
    v = _lib().orc_table_reduced(ctypes.byref(p), float(rr), float(Tr), ctypes.byref(inside))
    del keep
    return v if inside.value else None


def maxwell(Tr):
    """Reduced (rho_v, rho_l, p_sat) of the van der Waals fluid at reduced temperature Tr."""
    rv, rl, ps = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    st = _lib().orc_maxwell(float(Tr), ctypes.byref(rv), ctypes.byref(rl), ctypes.byref(ps))
    if st != OK:
        raise ValueError("Maxwell construction needs 0 < Tr < 1")
    return rv.value, rl.value, ps.value


def equilibrium(Q, rho, u):
    out = np.zeros(Q)
    uu = _f64(list(u) + [0.0] * (3 - len(u)))
    _lib().orc_equilibrium(Q, float(rho), _ptr(uu), _ptr(out))
    return out


def force(Q, Phi, A):
    Phi = _f64(Phi)
    nz, ny, nx = Phi.shape
    F = np.zeros((3,) + Phi.shape)
    if _lib().orc_force(Q, nx, ny, nz, float(A), _ptr(Phi), _ptr(F)) != OK:
        raise ValueError("bad lattice")
    return F


def divergence(D, u):
    u = _f64(u)
    nz, ny, nx = u.shape[1:]
    out = np.zeros(u.shape[1:])
    _lib().orc_divergence(D, nx, ny, nz, _ptr(u), _ptr(out))
    return out


def conduction(D, c_v, chi, rho, T):
    rho, T = _f64(rho), _f64(T)
    nz, ny, nx = rho.shape
    out = np.zeros(rho.shape)
    _lib().orc_conduction(D, nx, ny, nz, float(c_v), float(chi), _ptr(rho), _ptr(T), _ptr(out))
    return out


def force_walls(Phi, A):
    """Force of section 3 on a D3Q19 box with walls normal to z (Phi mirrored beyond them)."""
    Phi = _f64(Phi)
    nz, ny, nx = Phi.shape
    F = np.zeros((3,) + Phi.shape)
    _lib().orc_force_walls(nx, ny, nz, float(A), _ptr(Phi), _ptr(F))
    return F


def divergence_walls(u):
    """Central-difference divergence with walls normal to z (u_z mirrored with opposite sign)."""
    u = _f64(u)
    nz, ny, nx = u.shape[1:]
    out = np.zeros(u.shape[1:])
    _lib().orc_divergence_walls(nx, ny, nz, _ptr(u), _ptr(out))
    return out


def conduction_walls(c_v, chi, rho, T, wall_heat, T_bottom, T_top):
    """Conduction increment with walls normal to z (adiabatic or held at T_bottom / T_top)."""
    rho, T = _f64(rho), _f64(T)
    nz, ny, nx = rho.shape
    out = np.zeros(rho.shape)
    _lib().orc_conduction_walls(nx, ny, nz, float(c_v), float(chi), _ptr(rho), _ptr(T),
                                int(wall_heat), float(T_bottom), float(T_top), _ptr(out))
    return out


_PARAM_KEYS = ("tau", "tau_E", "A", "rho_c", "T_c", "p_c", "c_v", "chi", "rhoQ", "T0_baro",
               "flags")


# walls, wall temperatures and the body force are optional keys of `params` (default: periodic
# box, no body force)
_WALL_DEFAULTS = {"walls": 0, "wall_heat": 0, "T_bottom": 0.0, "T_top": 0.0,
                  "gravity": (0.0, 0.0, 0.0)}

# the collision form is optional too (default BGK); the MRT rates matter only with MRT
_MRT_DEFAULTS = {"collision": BGK, "s_e": 1.0, "s_eps": 1.0, "s_q": 1.0, "s_m": 1.0}


class Sim:
    """One simulation on the CPU in FP64 (periodic, or with walls normal to z)."""

    def __init__(self, Q, params, rho0, u0, T0):
        rho0, u0, T0 = _f64(rho0), _f64(u0), _f64(T0)
        if rho0.ndim != 3 or u0.shape != (3,) + rho0.shape or T0.shape != rho0.shape:
            raise ValueError("rho0/T0 must be (nz,ny,nx) and u0 (3,nz,ny,nx)")
        nz, ny, nx = rho0.shape
        p = _Params(Q=Q, nx=nx, ny=ny, nz=nz)
        for k in _PARAM_KEYS:
            setattr(p, k, params[k] if k != "flags" else int(params[k]))
        p.walls = int(params.get("walls", _WALL_DEFAULTS["walls"]))
        p.wall_heat = int(params.get("wall_heat", _WALL_DEFAULTS["wall_heat"]))
        p.T_bottom = float(params.get("T_bottom", _WALL_DEFAULTS["T_bottom"]))
        p.T_top = float(params.get("T_top", _WALL_DEFAULTS["T_top"]))
        gv = params.get("gravity", _WALL_DEFAULTS["gravity"])
        for a in range(3):
            p.gravity[a] = float(gv[a])
        p.collision = int(params.get("collision", _MRT_DEFAULTS["collision"]))
        for k in ("s_e", "s_eps", "s_q", "s_m"):
            setattr(p, k, float(params.get(k, _MRT_DEFAULTS[k])))
        # optional tabulated equation of state: params["eos_table"] = dict(p=(nT, nrho) reduced
        # pressures, coex=(nT, 2) reduced band limits, rho_range=(min, max), T_range=(min, max))
        keep = _table_fields(p, params["eos_table"]) if params.get("eos_table") else None
        self.Q, self.shape = Q, rho0.shape
        self._p = p
        st = ctypes.c_int()
        h = _lib().orc_create(ctypes.byref(p), _ptr(rho0), _ptr(u0), _ptr(T0), ctypes.byref(st))
        del keep   # the oracle copied the table
        if not h:
            raise ValueError("oracle rejected the parameters or initial fields (status %d)"
                             % st.value)
        self._h = h

    def step(self, n=1):
        st = _lib().orc_step(self._h, int(n))
        if st != OK:
            raise FloatingPointError("oracle step failed with status %d" % st)

    def moments(self):
        """dict rho, u_star (3,...), E, T of the current state."""
        rho = np.zeros(self.shape)
        us = np.zeros((3,) + self.shape)
        E = np.zeros(self.shape)
        T = np.zeros(self.shape)
        st = _lib().orc_moments(self._h, _ptr(rho), _ptr(us), _ptr(E), _ptr(T))
        if st != OK:
            raise FloatingPointError("state outside the EOS domain")
        return {"rho": rho, "u_star": us, "E": E, "T": T}

    def totals(self):
        out = np.zeros(5)
        _lib().orc_totals(self._h, _ptr(out))
        return out

    def last_sources(self):
        w, c, l = (np.zeros(self.shape) for _ in range(3))
        _lib().orc_last_sources(self._h, _ptr(w), _ptr(c), _ptr(l))
        return {"work": w, "cond": c, "latent": l}

    def get_pops(self):
        N = np.zeros((self.Q,) + self.shape)
        g = np.zeros((self.Q,) + self.shape)
        _lib().orc_get_pops(self._h, _ptr(N), _ptr(g))
        return N, g

    def set_pops(self, N, g):
        N, g = _f64(N), _f64(g)
        _lib().orc_set_pops(self._h, _ptr(N), _ptr(g))

    @property
    def step_count(self):
        return _lib().orc_step_count(self._h)

    def close(self):
        if getattr(self, "_h", None):
            _lib().orc_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

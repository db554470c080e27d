"""Thin ctypes binding of the C ABI in include/lbm_mi355x.h (argument marshalling only).

Every function here has the name of the C entry point it calls; all arithmetic of the method
runs in the HIP library.  Fields are numpy float64 arrays of shape (nz, ny, nx) (x fastest)
or (3, nz, ny, nx) for vectors.  The library is loaded on first use; if it has not been built
(``python -m paper_1705_10045_amd.build``) every call raises ``LbmUnavailable``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EUNSTABLE, LBM_EDEVICE, LBM_EBUSY = 0, -1, -2, -3, -4, -5
LBM_WORK, LBM_CONDUCTION, LBM_LATENT, LBM_PSEUDOFORCE, LBM_BAROTROPIC = 1, 2, 4, 8, 16

_STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EUNSTABLE",
           -4: "LBM_EDEVICE", -5: "LBM_EBUSY"}


class LbmUnavailable(ImportError):
    pass


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("nz", ctypes.c_int), ("storage_bytes", ctypes.c_int),
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


LBM_COLLISION_BGK = 0
LBM_COLLISION_MRT = 1

LBM_EOS_VDW = 0
LBM_EOS_TABLE = 1

LBM_WALL_T_BOTTOM = 1
LBM_WALL_T_TOP = 2

_D = ctypes.POINTER(ctypes.c_double)
_P = ctypes.c_void_p
_ST = ctypes.c_int
_LIB = None

# (name, restype, argtypes) of every exported entry point
_SIGNATURES = [
    ("lbm_init", _ST, [ctypes.POINTER(lbm_params), _D, _D, _D, _P, ctypes.POINTER(_P)]),
    ("lbm_step", _ST, [_P, ctypes.c_int]),
    ("lbm_step_async", _ST, [_P, ctypes.c_int]),
    ("lbm_check", _ST, [_P]),
    ("lbm_moments", _ST, [_P, _D, _D, _D, _D]),
    ("lbm_moments_device", _ST, [_P, _P, _P, _P, _P]),
    ("lbm_moments_device_noalloc", _ST, [_P, _P, _P, _P, _P]),
    ("lbm_reduce", _ST, [_P, _D]),
    ("lbm_step_reduce", _ST, [_P, ctypes.c_int, _D]),
    ("lbm_step_count", ctypes.c_longlong, [_P]),
    ("lbm_footprint_bytes", ctypes.c_size_t, [ctypes.POINTER(lbm_params)]),
    ("lbm_checkpoint", _ST, [_P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    ("lbm_restore", _ST, [_P, _P, ctypes.c_size_t]),
    ("lbm_free", _ST, [_P]),
    ("lbm_last_error", ctypes.c_char_p, []),
    ("lbm_launch_info", _ST, [_P, ctypes.POINTER(ctypes.c_int)]),
    ("lbm_launch_plan", _ST, [ctypes.POINTER(lbm_params), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    ("lbm_set_launch", _ST, [_P, ctypes.c_int, ctypes.c_int]),
    ("lbm_lattice_info", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D, _D, _D]),
    ("lbm_coexistence", _ST, [ctypes.c_double, _D, _D]),
    ("lbm_pool_create", _ST, [ctypes.c_size_t, ctypes.c_int, ctypes.c_int, _P, ctypes.POINTER(_P)]),
    ("lbm_pool_submit", _ST, [_P, ctypes.POINTER(lbm_params), _D, _D, _D, ctypes.c_longlong,
                              ctypes.POINTER(ctypes.c_longlong)]),
    ("lbm_pool_run", _ST, [_P]),
    ("lbm_pool_run_async", _ST, [_P]),
    ("lbm_pool_poll", _ST, [_P, ctypes.c_longlong, ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_int)]),
    ("lbm_pool_collect", _ST, [_P, ctypes.c_longlong, _D, _D, _D, _D]),
    ("lbm_pool_stats", _ST, [_P, ctypes.POINTER(ctypes.c_longlong)]),
    ("lbm_pool_totals", _ST, [_P, ctypes.c_longlong, _D, _D]),
    ("lbm_pool_destroy", _ST, [_P]),
]


def library_path():
    return _build.LIB


def lib():
    """The loaded HIP library (raises LbmUnavailable if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            raise LbmUnavailable("HIP library %s is not built; run paper_1705_10045_amd/build.py"
                                 % _build.LIB)
        L = ctypes.CDLL(_build.LIB)
        for name, res, args in _SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(status):
    if status != LBM_OK:
        raise LbmError(status, lib().lbm_last_error().decode())
    return status


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), a.shape))
    return a


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def make_params(Q, shape, physics, storage_bytes=4):
    nz, ny, nx = shape
    p = lbm_params(lattice=Q, nx=nx, ny=ny, nz=nz, storage_bytes=storage_bytes)
    for k in ("tau", "tau_E", "A", "rho_c", "T_c", "p_c", "c_v", "chi", "rhoQ", "T0_baro"):
        setattr(p, k, float(physics[k]))
    p.flags = int(physics["flags"])
    # walls and body force are optional keys (default: periodic box, no body force)
    p.walls = int(physics.get("walls", 0))
    p.wall_heat = int(physics.get("wall_heat", 0))
    p.T_bottom = float(physics.get("T_bottom", 0.0))
    p.T_top = float(physics.get("T_top", 0.0))
    gv = physics.get("gravity", (0.0, 0.0, 0.0))
    for a in range(3):
        p.gravity[a] = float(gv[a])
    # the collision form is optional too (default BGK; the MRT rates matter only with MRT)
    p.collision = int(physics.get("collision", LBM_COLLISION_BGK))
    for k in ("s_e", "s_eps", "s_q", "s_m"):
        setattr(p, k, float(physics.get(k, 1.0)))
    # optional tabulated equation of state: physics["eos_table"] = dict(p=(nT, nrho) reduced
    # pressures, coex=(nT, 2) reduced band limits, rho_range=(min, max), T_range=(min, max));
    # the arrays are kept on the params object until lbm_init has read them
    table = physics.get("eos_table")
    if table:
        tp = np.ascontiguousarray(table["p"], dtype=np.float64)
        tc = np.ascontiguousarray(table["coex"], dtype=np.float64)
        if tp.ndim != 2 or tc.shape != (tp.shape[0], 2):
            raise ValueError("eos_table p must be (nT, nrho) and coex (nT, 2)")
        p.eos = LBM_EOS_TABLE
        p.eos_p, p.eos_coex = _dp(tp), _dp(tc)
        p.eos_nT, p.eos_nrho = tp.shape
        p.eos_rho_min, p.eos_rho_max = (float(v) for v in table["rho_range"])
        p.eos_T_min, p.eos_T_max = (float(v) for v in table["T_range"])
        p._keep = (tp, tc)
    return p


# ------------------------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ------------------------------------------------------------------------------------------
def lbm_init(params, rho0, u0, T0, stream=None):
    shape = (params.nz, params.ny, params.nx)
    rho0 = _f64(rho0, shape)
    u0 = _f64(u0, (3,) + shape)
    T0 = _f64(T0, shape)
    h = _P()
    _check(lib().lbm_init(ctypes.byref(params), _dp(rho0), _dp(u0), _dp(T0),
                          _P(stream) if stream else None, ctypes.byref(h)))
    return h


def lbm_step(h, nsteps):
    return _check(lib().lbm_step(h, int(nsteps)))


def lbm_step_async(h, nsteps):
    return _check(lib().lbm_step_async(h, int(nsteps)))


def lbm_check(h):
    return _check(lib().lbm_check(h))


def lbm_moments(h, shape):
    rho = np.empty(shape)
    us = np.empty((3,) + tuple(shape))
    E = np.empty(shape)
    T = np.empty(shape)
    _check(lib().lbm_moments(h, _dp(rho), _dp(us), _dp(E), _dp(T)))
    return {"rho": rho, "u_star": us, "E": E, "T": T}


def lbm_moments_device(h, rho_ptr, us_ptr, E_ptr, T_ptr):
    return _check(lib().lbm_moments_device(h, rho_ptr, us_ptr, E_ptr, T_ptr))


def lbm_moments_device_noalloc(h, rho_ptr, us_ptr, E_ptr, T_ptr):
    return _check(lib().lbm_moments_device_noalloc(h, rho_ptr, us_ptr, E_ptr, T_ptr))


def lbm_reduce(h):
    out = np.zeros(5)
    _check(lib().lbm_reduce(h, _dp(out)))
    return out


def lbm_step_reduce(h, nsteps):
    out = np.zeros(5)
    _check(lib().lbm_step_reduce(h, nsteps, _dp(out)))
    return out


def lbm_step_count(h):
    return lib().lbm_step_count(h)


def lbm_footprint_bytes(params):
    return lib().lbm_footprint_bytes(ctypes.byref(params))


def lbm_checkpoint(h):
    used = ctypes.c_size_t()
    _check(lib().lbm_checkpoint(h, None, 0, ctypes.byref(used)))
    buf = ctypes.create_string_buffer(used.value)
    _check(lib().lbm_checkpoint(h, buf, used.value, ctypes.byref(used)))
    return buf.raw


def lbm_restore(h, data):
    buf = ctypes.create_string_buffer(data, len(data))
    return _check(lib().lbm_restore(h, buf, len(data)))


def lbm_free(h):
    return _check(lib().lbm_free(h))


def lbm_last_error():
    return lib().lbm_last_error().decode()


def lbm_launch_info(h):
    info = (ctypes.c_int * 4)()
    _check(lib().lbm_launch_info(h, info))
    return {"tile_x": info[0], "tile_y": info[1], "chunk": info[2], "workgroups": info[3]}


def lbm_launch_plan(Q, shape, physics, storage_bytes=4, cus=256):
    """The launch lbm_init would choose for this box (host only, no device)."""
    params = make_params(Q, shape, physics, storage_bytes)
    info = (ctypes.c_int * 4)()
    _check(lib().lbm_launch_plan(ctypes.byref(params), int(cus), info))
    return {"tile_x": info[0], "tile_y": info[1], "chunk": info[2], "workgroups": info[3]}


def lbm_set_launch(h, variant, chunk=0):
    return _check(lib().lbm_set_launch(h, int(variant), int(chunk)))


def lbm_lattice_info(Q):
    c = (ctypes.c_int * (3 * Q))()
    w = np.zeros(Q)
    G = np.zeros(Q)
    alpha = ctypes.c_double()
    D = lib().lbm_lattice_info(Q, c, _dp(w), _dp(G), ctypes.byref(alpha))
    if D < 0:
        raise LbmError(D, "unsupported lattice")
    return np.array(list(c)).reshape(Q, 3), w, G, alpha.value, D


def lbm_coexistence(Tr):
    rv, rl = ctypes.c_double(), ctypes.c_double()
    _check(lib().lbm_coexistence(float(Tr), ctypes.byref(rv), ctypes.byref(rl)))
    return rv.value, rl.value


# ------------------------------------------------------------------------------------------
# Convenience wrapper
# ------------------------------------------------------------------------------------------
class Sim:
    """One simulation on the current HIP device (owns its lbm_sim handle)."""

    def __init__(self, Q, physics, rho0, u0, T0, storage_bytes=4, stream=None):
        rho0 = np.asarray(rho0)
        self.shape = tuple(rho0.shape)
        self.Q = Q
        self.params = make_params(Q, self.shape, physics, storage_bytes)
        self._h = lbm_init(self.params, rho0, u0, T0, stream)

    def step(self, n=1):
        lbm_step(self._h, n)

    def step_async(self, n=1):
        lbm_step_async(self._h, n)

    def check(self):
        lbm_check(self._h)

    def moments(self):
        return lbm_moments(self._h, self.shape)

    def reduce(self):
        return lbm_reduce(self._h)

    def step_reduce(self, n=1):
        return lbm_step_reduce(self._h, n)

    def checkpoint(self):
        return lbm_checkpoint(self._h)

    def restore(self, data):
        lbm_restore(self._h, data)

    def launch_info(self):
        return lbm_launch_info(self._h)

    def set_launch(self, variant, chunk=0):
        lbm_set_launch(self._h, variant, chunk)

    @property
    def step_count(self):
        return lbm_step_count(self._h)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lbm_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ------------------------------------------------------------------------------------------
# Serving pool
# ------------------------------------------------------------------------------------------
def lbm_pool_create(hbm_budget_bytes, max_slots, steps_per_run, stream=None):
    h = _P()
    _check(lib().lbm_pool_create(int(hbm_budget_bytes), int(max_slots), int(steps_per_run),
                                 _P(stream) if stream else None, ctypes.byref(h)))
    return h


def lbm_pool_submit(pool, params, rho0, u0, T0, nsteps):
    """Ticket of the admitted request, or None if the pool is busy (no slot / budget)."""
    shape = (params.nz, params.ny, params.nx)
    rho0 = _f64(rho0, shape)
    u0 = _f64(u0, (3,) + shape)
    T0 = _f64(T0, shape)
    t = ctypes.c_longlong()
    st = lib().lbm_pool_submit(pool, ctypes.byref(params), _dp(rho0), _dp(u0), _dp(T0),
                               int(nsteps), ctypes.byref(t))
    if st == LBM_EBUSY:
        return None
    _check(st)
    return t.value


def lbm_pool_run(pool):
    return _check(lib().lbm_pool_run(pool))


def lbm_pool_run_async(pool):
    return _check(lib().lbm_pool_run_async(pool))


def lbm_pool_poll(pool, ticket):
    done = ctypes.c_int()
    res = ctypes.c_int()
    _check(lib().lbm_pool_poll(pool, int(ticket), ctypes.byref(done), ctypes.byref(res)))
    return bool(done.value), res.value


def lbm_pool_collect(pool, ticket, shape):
    """Final fields of a finished request (dict as lbm_moments) and its status."""
    rho = np.empty(shape)
    us = np.empty((3,) + tuple(shape))
    E = np.empty(shape)
    T = np.empty(shape)
    st = lib().lbm_pool_collect(pool, int(ticket), _dp(rho), _dp(us), _dp(E), _dp(T))
    if st not in (LBM_OK, LBM_EUNSTABLE):
        _check(st)
    return {"rho": rho, "u_star": us, "E": E, "T": T}, st


def lbm_pool_totals(pool, ticket):
    """Totals (mass, momentum, energy) of a finished request at admission and at its end."""
    initial = np.zeros(5)
    final = np.zeros(5)
    _check(lib().lbm_pool_totals(pool, int(ticket), _dp(initial), _dp(final)))
    return initial, final


def lbm_pool_stats(pool):
    out = (ctypes.c_longlong * 4)()
    _check(lib().lbm_pool_stats(pool, out))
    return {"active": out[0], "bytes_in_use": out[1], "budget": out[2], "free_slots": out[3]}


def lbm_pool_destroy(pool):
    return _check(lib().lbm_pool_destroy(pool))


class Pool:
    """Serving pool of D3Q19 FP32 simulations resident on the current device."""

    def __init__(self, hbm_budget_bytes, max_slots=64, steps_per_run=10, stream=None):
        self._h = lbm_pool_create(hbm_budget_bytes, max_slots, steps_per_run, stream)
        self.steps_per_run = steps_per_run
        self._shapes = {}

    def submit(self, physics, rho0, u0, T0, nsteps):
        rho0 = np.asarray(rho0)
        params = make_params(19, rho0.shape, physics, 4)
        t = lbm_pool_submit(self._h, params, rho0, u0, T0, nsteps)
        if t is not None:
            self._shapes[t] = tuple(rho0.shape)
        return t

    def run(self):
        lbm_pool_run(self._h)

    def run_async(self):
        lbm_pool_run_async(self._h)

    def poll(self, ticket):
        return lbm_pool_poll(self._h, ticket)

    def collect(self, ticket):
        fields, st = lbm_pool_collect(self._h, ticket, self._shapes.pop(ticket))
        return fields, st

    def totals(self, ticket):
        return lbm_pool_totals(self._h, ticket)

    def stats(self):
        return lbm_pool_stats(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lbm_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

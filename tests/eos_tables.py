"""Tabulated equations of state for the tests: the reduced van der Waals EOS sampled on a
uniform grid by the oracle's own function, with the oracle's Maxwell band per row.  Used as an
input of both the oracle and the library (a table is data; the interpolation is what each side
implements)."""
import functools

import numpy as np

import oracle


@functools.lru_cache(maxsize=4)
def _vdw(rho_range, nrho, T_range, nT):
    rho = np.linspace(rho_range[0], rho_range[1], nrho)
    T = np.linspace(T_range[0], T_range[1], nT)
    p = np.array([[oracle.vdw_reduced(r, t) for r in rho] for t in T])
    coex = np.array([oracle.maxwell(t)[:2] if t < 0.999 else (1.0, 1.0) for t in T])
    p.setflags(write=False)
    coex.setflags(write=False)
    return p, coex


def vdw_table(rho_range=(0.01, 2.6), nrho=2048, T_range=(0.5, 1.0), nT=501):
    """dict(p=(nT, nrho), coex=(nT, 2), rho_range, T_range); the band is empty (1, 1) from
    T~ = 0.999 up."""
    p, coex = _vdw(tuple(rho_range), nrho, tuple(T_range), nT)
    return dict(p=p, coex=coex, rho_range=tuple(rho_range), T_range=tuple(T_range))

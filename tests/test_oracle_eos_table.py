"""The oracle's tabulated equation of state (section 3 names tabulated EOS of real fluids; the
library takes one as p~ on a uniform (rho~, T~) grid, cubic in rho~ and linear in T~, with the
coexistence band of the latent heat given per row).  Pinned by what interpolation fixes on its
own: exact reproduction of any polynomial cubic in rho~ and linear in T~ (the stencil, weights
and row blend), the Lagrange remainder bound against the analytic van der Waals EOS, and whole
runs of the tabulated van der Waals fluid against the analytic one.  Real-fluid tables (water,
Fig. 2) are not in this container: their results are parity unpinned."""
import numpy as np
import pytest

import eos_tables
from paper_1705_10045_amd import inputs as I


def vdw_table(orc, **kw):
    return eos_tables.vdw_table(**kw)


def test_reproduces_cubic_in_rho_linear_in_T_exactly(orc):
    """Cubic Lagrange interpolation in rho~ and linear in T~ is exact for p~ = a(rho~) + T~ b(rho~)
    with cubic a, b, anywhere on the grid, including the cells next to its edges where the
    stencil is shifted inward."""
    rng = np.random.default_rng(7)
    a, b = rng.normal(size=4), rng.normal(size=4)
    f = lambda r, t: np.polyval(a, r) + t * np.polyval(b, r)
    rho = np.linspace(0.2, 2.2, 37)
    T = np.linspace(0.55, 0.95, 9)
    table = dict(p=np.array([[f(r, t) for r in rho] for t in T]), coex=np.ones((9, 2)),
                 rho_range=(0.2, 2.2), T_range=(0.55, 0.95))
    pts = np.concatenate([rng.uniform(0.2, 2.2, 300), [0.2, 0.2001, 2.2, 2.1999, 0.25, 2.17]])
    for r in pts:
        t = rng.uniform(0.55, 0.95)
        got = orc.table_reduced(table, r, t)
        assert got == pytest.approx(f(r, t), rel=1e-12, abs=1e-12)
    for t in (0.55, 0.95):
        assert orc.table_reduced(table, 1.0, t) == pytest.approx(f(1.0, t), rel=1e-12)


def test_outside_the_grid_is_outside_the_domain(orc):
    table = vdw_table(orc)
    assert orc.table_reduced(table, 0.009, 0.8) is None
    assert orc.table_reduced(table, 2.61, 0.8) is None
    assert orc.table_reduced(table, 1.0, 0.49) is None
    assert orc.table_reduced(table, 1.0, 1.01) is None
    assert orc.table_reduced(table, 2.6, 1.0) is not None


def test_tabulated_vdw_within_the_lagrange_remainder(orc):
    """p~ of van der Waals is linear in T~, so only the rho~ interpolation errs.  The cubic
    through the grid densities x_{i-1} .. x_{i+2} around a point x_i + t h (0 <= t < 1) leaves
    |(t+1) t (t-1) (t-2)| h^4 / 24 times d4p/drho4 somewhere on the stencil, at most
    (9/16) h^4 / 24 max|d4p~/drho~4| with d4p~/drho~4 = 576 T~ / (3 - rho~)^5, largest at the
    stencil's top end x_{i+2}.  A stencil placed otherwise (not centred on the point's cell)
    can err up to (1) h^4 / 24 max|...| and reach x_{i+3}, beyond this bound."""
    table = vdw_table(orc)
    lo, hi, n = 0.01, 2.6, 2048
    h = (hi - lo) / (n - 1)
    rng = np.random.default_rng(3)
    worst = 0.0
    for r, t in zip(rng.uniform(lo + 1.5 * h, hi - 2.5 * h, 4000), rng.uniform(0.5, 1.0, 4000)):
        exact = orc.vdw_reduced(r, t)
        err = abs(orc.table_reduced(table, r, t) - exact)
        i = np.floor((r - lo) / h)
        top = lo + (i + 2) * h
        f4 = 576.0 * t / (3.0 - top) ** 5
        tt = (r - lo) / h - i
        bound = abs((tt + 1) * tt * (tt - 1) * (tt - 2)) * h ** 4 / 24.0 * f4
        # plus the rounding of the four products (weights sum to at most 1.25 in magnitude)
        assert err <= bound + 16 * 2.2e-16 * (abs(exact) + 1.0), (r, t)
        worst = max(worst, err / max(bound, 1e-300))
    assert worst > 0.1   # the comparison is not vacuous: the remainder is met, not undercut


def _case(table=None, flags=I.ALL_TERMS, shape=(20, 22, 24)):
    case = I.droplet_3d(shape=shape, radius=6.0, velocity=(0.03, 0.0, 0.0),
                        params=I.physics(flags=flags))
    if table is not None:
        case["params"] = dict(case["params"], eos_table=table)
    return case


def _run(orc, case, steps):
    s = orc.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"])
    s.step(steps)
    m = s.moments()
    s.close()
    return m


@pytest.mark.parametrize("flags,tol", [(I.WORK | I.CONDUCTION | I.PSEUDOFORCE, 1e-10),
                                       (I.ALL_TERMS, 1e-8)])
def test_tabulated_vdw_run_follows_the_analytic_one(orc, flags, tol):
    """40 steps of a moving droplet with the tabulated van der Waals EOS against the analytic
    EOS.  Without latent heat only the pressure interpolation differs (about 1e-12 of p~ here;
    measured field differences 2e-12); with it, the band limits are also interpolated linearly
    between rows 0.001 apart in T~ instead of cubically on the 4096-point Maxwell table
    (measured 1.1e-9)."""
    table = vdw_table(orc)
    a = _run(orc, _case(None, flags), 40)
    b = _run(orc, _case(table, flags), 40)
    for k in ("rho", "E", "T"):
        assert np.abs(a[k] - b[k]).max() / np.abs(a[k]).max() < tol, k
    assert np.abs(a["u_star"] - b["u_star"]).max() / max(np.abs(a["u_star"]).max(), 0.01) < tol


def test_table_band_drives_the_latent_source(orc):
    """The latent source of a tabulated EOS uses the table's own band: shifting the band to
    exclude the uniform density switches the source off, and narrowing it scales the source by
    the inverse width."""
    n = 48
    shape = (1, 1, n)
    x = np.arange(n, dtype=np.float64)
    u0 = np.zeros((3,) + shape)
    u0[0, 0, 0, :] = 0.01 * np.sin(2 * np.pi * x / n + 0.3)
    rho = np.full(shape, 1.1)
    base = vdw_table(orc)

    def latent(coex):
        table = dict(base, coex=coex)
        p = dict(I.physics(flags=I.LATENT | I.BAROTROPIC | I.PSEUDOFORCE, T0_baro=0.9,
                           rhoQ=0.01), eos_table=table)
        s = orc.Sim(9, p, rho, u0, np.full(shape, 0.9))
        s.step(1)
        lat = s.last_sources()["latent"].ravel()
        s.close()
        return lat

    wide = latent(np.tile([0.5, 1.5], (base["coex"].shape[0], 1)))
    narrow = latent(np.tile([0.9, 1.4], (base["coex"].shape[0], 1)))
    off = latent(np.tile([1.2, 1.5], (base["coex"].shape[0], 1)))
    assert np.all(off == 0.0) and np.count_nonzero(wide) == n
    np.testing.assert_allclose(narrow, wide * (1.0 / 0.5), rtol=1e-12)


def test_leaving_the_table_stops_the_run(orc):
    """A state whose density reaches beyond the table's grid has left the EOS domain."""
    table = vdw_table(orc, rho_range=(0.2, 2.6))
    case = _case(table, shape=(16, 16, 16))     # the vapour (0.24) sits just inside the grid
    s = orc.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"])
    s.step(1)
    s.close()
    low = dict(table, rho_range=(0.3, 2.6))      # now the vapour lies below it
    case = _case(low, shape=(16, 16, 16))
    s = orc.Sim(case["Q"], case["params"], case["rho0"], case["u0"], case["T0"])
    with pytest.raises(FloatingPointError):
        s.step(1)
    s.close()

"""Pins of the oracle's van der Waals equation of state and Maxwell-rule coexistence solver
(section 3 EOS; section 5 and Fig. 4b use the coexistence densities)."""
import numpy as np
import pytest
from scipy.integrate import quad


def test_critical_point(orc):
    """p~(1,1) = 1 with a horizontal inflection: dp/drho = d2p/drho2 = 0 at the critical point."""
    f = orc.vdw_reduced
    assert f(1.0, 1.0) == pytest.approx(1.0, abs=1e-15)
    h = 1e-4
    d1 = (f(1 + h, 1.0) - f(1 - h, 1.0)) / (2 * h)
    d2 = (f(1 + h, 1.0) - 2 * f(1.0, 1.0) + f(1 - h, 1.0)) / h ** 2
    assert abs(d1) < 1e-7 and abs(d2) < 1e-5


def test_ideal_gas_limit(orc):
    """rho -> 0: p~ -> (8/3) rho~ T~ (reduced vdW gas constant)."""
    for T in (0.5, 0.8, 1.3):
        r = 1e-7
        assert orc.vdw_reduced(r, T) / (8.0 / 3.0 * r * T) == pytest.approx(1.0, rel=1e-6)


@pytest.mark.parametrize("Tr", [0.45, 0.6, 0.75, 0.8, 0.85, 0.9, 0.95, 0.99])
def test_equal_area_rule(orc, Tr):
    """Maxwell's construction written independently in specific volume v = 1/rho:
    p(v_l) = p(v_v) = P and the integral of p dv from v_l to v_v equals P (v_v - v_l),
    evaluated with scipy's adaptive quadrature."""
    rv, rl, P = orc.maxwell(Tr)
    assert orc.vdw_reduced(rv, Tr) == pytest.approx(P, rel=1e-11)
    assert orc.vdw_reduced(rl, Tr) == pytest.approx(P, rel=1e-11)
    vl, vv = 1.0 / rl, 1.0 / rv
    p_of_v = lambda v: 8.0 * Tr / (3.0 * v - 1.0) - 3.0 / (v * v)
    area, _ = quad(p_of_v, vl, vv, epsabs=1e-13, epsrel=1e-13, limit=500)
    assert area == pytest.approx(P * (vv - vl), rel=1e-9)
    # vapour and liquid sit outside the spinodal 4 T = rho (3 - rho)^2
    spin = np.sort(np.roots([1.0, -6.0, 9.0, -4.0 * Tr]).real)
    assert rv < spin[0] < 1.0 < spin[1] < rl < 3.0


def test_textbook_values_at_0_9(orc):
    """Tabulated reduced vdW coexistence at T~ = 0.9 (standard result of the equal-area rule)."""
    rv, rl, P = orc.maxwell(0.9)
    assert rv == pytest.approx(0.425742, abs=2e-6)
    assert rl == pytest.approx(1.657270, abs=2e-6)
    assert P == pytest.approx(0.646998, abs=2e-6)


def test_near_critical_asymptotics(orc):
    """Close to T_c the coexistence branches open as rho_l - rho_v = 4 sqrt(1 - T~) (1 + O(1-T~))."""
    errs = []
    for eps in (1e-2, 1e-3, 1e-4):
        rv, rl, _ = orc.maxwell(1.0 - eps)
        errs.append(abs((rl - rv) / (4.0 * np.sqrt(eps)) - 1.0))
    assert errs[0] < 0.02 and errs[1] < 2e-3 and errs[2] < 2e-4
    assert errs[0] > errs[1] > errs[2]


def test_rejects_supercritical(orc):
    with pytest.raises(ValueError):
        orc.maxwell(1.0)
    with pytest.raises(ValueError):
        orc.maxwell(1.2)


def test_input_table_matches_solver(orc):
    """The coexistence data that places initial densities agrees with the oracle's solver."""
    from paper_1705_10045_amd import inputs
    for T, rv, rl in inputs.COEXISTENCE:
        ov, ol, _ = orc.maxwell(T)
        assert rv == pytest.approx(ov, abs=2e-9)
        assert rl == pytest.approx(ol, abs=2e-9)

"""The paper-scale experiment inputs (section 6) are what their captions state: checked on the
host, without a GPU, against the reduced van der Waals equation of state and the Maxwell
coexistence densities computed by the oracle."""
import numpy as np
import pytest

import scenarios as S


def test_hot_gas_layer_is_at_uniform_pressure_and_single_phase(orc):
    case = S.hot_gas_1d()
    rho, T = case["rho0"].ravel(), case["T0"].ravel()
    assert set(np.unique(T)) == {0.6, 0.947}
    p = S.vdw_reduced_pressure(rho, T)
    assert np.ptp(p) < 1e-12 * p.max()
    # both states are unsaturated gas: below the vapour coexistence density of their temperature
    for Tr in (0.6, 0.947):
        rv, _, _ = orc.maxwell(Tr)
        assert rho[T == Tr].max() < rv
    assert (T == 0.947).sum() == 200 and rho.size == 1000


def test_spinodal_states_lie_inside_the_spinodal():
    """(dp/drho)_T < 0 at the initial density and temperature (eq:sspeed's c_T is negative)."""
    for rho0 in (0.7, 1.0):
        cT = 24 * 0.8 / (3 - rho0) ** 2 - 6 * rho0
        assert cT < 0
    one = S.spinodal_1d()["rho0"].ravel()
    two = S.spinodal_2d()["rho0"].ravel()
    assert abs(one.mean() - 0.7) < 1e-3 and np.ptp(one) > 0.01
    assert abs(two.mean() - 1.0) < 1e-3 and two.size == 500 * 500


def test_moving_drop_is_at_coexistence_and_moves_diagonally(orc):
    case = S.moving_drop_2d(n=200, radius=40.0)
    rho = case["rho0"][0]
    rv, rl, _ = orc.maxwell(0.8)
    assert rho.max() == pytest.approx(rl, rel=1e-6)
    assert rho.min() == pytest.approx(rv, rel=1e-6)
    assert np.allclose(case["u0"][0], 0.1) and np.allclose(case["u0"][1], -0.1)
    assert np.allclose(case["u0"][2], 0.0)
    inside = (rho > 0.5 * (rv + rl)).sum()
    assert inside == pytest.approx(np.pi * 40.0 ** 2, rel=0.01)

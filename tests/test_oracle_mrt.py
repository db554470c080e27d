"""Pins of the oracle's multiple-relaxation-time collision (section 2 names it beside BGK; the
bases are those of Lallemand and Luo 2000, D2Q9, and d'Humieres et al. 2002, D3Q19).

  - the basis rows are orthogonal and span the population space;
  - the moments of the second-order equilibrium (eq:feq) take the published closed forms
    (a mistyped basis polynomial changes at least one of them);
  - with every rate equal to 1/tau the update is the BGK update;
  - mass and momentum are conserved exactly whatever the rates;
  - a shear wave decays at nu k^2 with nu = (tau - 1/2)/3 whatever the other rates, while the
    energy moment's rate s_e damps sound and leaves the shear decay alone (a moment placed in
    the wrong group fails one of these).
"""
import numpy as np
import pytest

import oracle
from paper_1705_10045_amd import inputs as I

D3Q19_RATES = dict(s_e=1.19, s_eps=1.4, s_q=1.2, s_m=1.98)


@pytest.mark.parametrize("Q", [9, 19])
def test_basis_is_orthogonal_and_complete(Q):
    M, n2, grp = oracle.mrt_basis(Q)
    G = M @ M.T
    assert np.array_equal(G, np.diag(n2))
    assert np.linalg.matrix_rank(M) == Q
    assert (grp == 0).sum() == (3 if Q == 9 else 4)          # rho and j
    assert (grp == 1).sum() == (2 if Q == 9 else 5)          # traceless stresses


def _equilibrium_moments(Q, rho, u):
    c, *_ = oracle.lattice(Q)
    M, _, _ = oracle.mrt_basis(Q)
    return M @ oracle.equilibrium(Q, rho, tuple(u))


def test_equilibrium_moments_d2q9():
    rho, (ux, uy) = 1.3, (0.05, -0.03)
    m = _equilibrium_moments(9, rho, (ux, uy, 0.0))
    u2 = ux * ux + uy * uy
    expected = [rho, rho * (-2 + 3 * u2), rho * (1 - 3 * u2), rho * ux, -rho * ux, rho * uy,
                -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy]
    assert np.allclose(m, expected, rtol=0, atol=1e-14)


def test_equilibrium_moments_d3q19():
    rho, (ux, uy, uz) = 0.9, (0.04, -0.02, 0.03)
    m = _equilibrium_moments(19, rho, (ux, uy, uz))
    u2 = ux * ux + uy * uy + uz * uz
    pxx3 = rho * (3 * ux * ux - u2)
    pww = rho * (uy * uy - uz * uz)
    expected = [rho, rho * (-11 + 19 * u2), rho * (3 - 5.5 * u2),
                rho * ux, -2 / 3 * rho * ux, rho * uy, -2 / 3 * rho * uy, rho * uz,
                -2 / 3 * rho * uz, pxx3, -0.5 * pxx3, pww, -0.5 * pww,
                rho * ux * uy, rho * uy * uz, rho * ux * uz, 0.0, 0.0, 0.0]
    assert np.allclose(m, expected, rtol=0, atol=1e-14)


def _droplet(Q, shape, tau):
    if Q == 19:
        case = I.droplet_3d(shape=shape, radius=3.0, velocity=(0.02, -0.01, 0.01))
    else:
        case = I.slab_2d(n=shape[1], width=shape[1] // 3)
        case["u0"][0] += 0.01
    case["params"] = dict(case["params"], tau=tau)
    return case


@pytest.mark.parametrize("Q,shape", [(19, (8, 10, 12)), (9, (1, 24, 24))])
def test_equal_rates_reduce_to_bgk(Q, shape):
    tau = 0.8
    case = _droplet(Q, shape, tau)
    bgk = oracle.Sim(Q, case["params"], case["rho0"], case["u0"], case["T0"])
    mrt_p = dict(case["params"], collision=oracle.MRT, s_e=1 / tau, s_eps=1 / tau, s_q=1 / tau,
                 s_m=1 / tau)
    mrt = oracle.Sim(Q, mrt_p, case["rho0"], case["u0"], case["T0"])
    bgk.step(40)
    mrt.step(40)
    a, b = bgk.moments(), mrt.moments()
    for k in a:
        assert np.abs(a[k] - b[k]).max() <= 1e-13 * max(np.abs(a[k]).max(), 0.01), k


@pytest.mark.parametrize("Q,shape", [(19, (8, 10, 12)), (9, (1, 24, 24))])
def test_mass_and_momentum_conserved_with_distinct_rates(Q, shape):
    case = _droplet(Q, shape, 0.7)
    p = dict(case["params"], collision=oracle.MRT, **D3Q19_RATES)
    s = oracle.Sim(Q, p, case["rho0"], case["u0"], case["T0"])
    t0 = s.totals()
    s.step(60)
    t1 = s.totals()
    assert abs(t1[0] - t0[0]) < 1e-13 * t0[0]
    for a in range(3):
        assert abs(t1[1 + a] - t0[1 + a]) < 1e-13 * t0[0]


def _wave_decay(kind, rates, tau=0.8, n=64, steps=400):
    """Amplitude ratio after `steps` of a small shear (u_y(x)) or sound (rho(x)) wave on a
    quasi-1D D3Q19 box of uniform density, barotropic EOS (no force from a uniform Phi)."""
    shape = (1, 1, n)
    x = np.arange(n)
    k = 2 * np.pi / n
    rho0 = 0.5
    rho = np.full(shape, rho0)
    u = np.zeros((3,) + shape)
    if kind == "shear":
        u[1, 0, 0] = 1e-4 * np.sin(k * x)
    else:
        rho = rho * (1 + 1e-4 * np.cos(k * x)).reshape(shape)
    p = I.physics(tau=tau, flags=oracle.BAROTROPIC | oracle.PSEUDOFORCE, T0_baro=0.9,
                  collision=oracle.MRT, **rates)
    s = oracle.Sim(19, p, rho, u, np.full(shape, 0.9))

    def amp():
        m = s.moments()
        f = m["u_star"][1].ravel() if kind == "shear" else m["rho"].ravel() - rho0
        basis = np.sin(k * x) if kind == "shear" else np.cos(k * x)
        return abs(2 * (f * basis).mean())

    a0 = amp()
    s.step(steps)
    return amp() / a0, k


def test_shear_wave_decays_at_nu_k2_whatever_the_other_rates():
    tau, steps = 0.8, 400
    nu = (tau - 0.5) / 3
    ratios = []
    for rates in (dict(s_e=1.0, s_eps=1.0, s_q=1.0, s_m=1.0), D3Q19_RATES,
                  dict(s_e=0.6, s_eps=1.8, s_q=0.7, s_m=1.1)):
        r, k = _wave_decay("shear", rates, tau, steps=steps)
        rate = -np.log(r) / steps
        assert rate == pytest.approx(nu * k * k, rel=0.01)
        ratios.append(r)
    assert np.ptp(ratios) < 1e-3                     # the other rates enter at O(k^4) only
    # and it follows tau: nu doubles from tau = 0.65 to 0.8
    r2, k = _wave_decay("shear", D3Q19_RATES, 0.65, steps=steps)
    assert -np.log(r2) / steps == pytest.approx((0.65 - 0.5) / 3 * k * k, rel=0.01)


def test_energy_rate_damps_sound_but_not_shear():
    base = dict(D3Q19_RATES)
    slow = dict(base, s_e=0.5)
    s_fast, _ = _wave_decay("sound", base)
    s_slow, _ = _wave_decay("sound", slow)
    assert s_slow < s_fast - 0.01                    # lower s_e: larger bulk viscosity
    h_fast, _ = _wave_decay("shear", base)
    h_slow, _ = _wave_decay("shear", slow)
    assert abs(h_fast - h_slow) < 1e-8                # e is not excited by a shear wave
    # the ghost rates leave sound alone to the same order
    s_ghost, _ = _wave_decay("sound", dict(base, s_eps=0.7, s_q=1.6, s_m=0.9))
    assert abs(s_ghost - s_fast) < 0.1 * abs(s_slow - s_fast)


@pytest.mark.parametrize("bad", [dict(collision=2), dict(collision=1, s_e=2.0),
                                 dict(collision=1, s_q=0.0)])
def test_mrt_parameters_are_validated(bad):
    case = _droplet(19, (6, 6, 6), 0.8)
    with pytest.raises(ValueError):
        oracle.Sim(19, dict(case["params"], **bad), case["rho0"], case["u0"], case["T0"])
    with pytest.raises(ValueError):     # no MRT basis for D1Q3
        oracle.Sim(3, I.physics(collision=1), np.full((1, 1, 8), 0.5), np.zeros((3, 1, 1, 8)),
                   np.full((1, 1, 8), 0.8))

"""Physics pins of the full oracle step on small (mostly quasi-1D) lattices, from what the paper
fixes in section 6: heat-conduction scaling and scheme diffusion (Figs. 5-6), the sound speed
against the heat-capacity ratio (eq:sspeed, Fig. 8), Galilean invariance (Figs. 5, 7), the
coexistence curve (section 3, Fig. 4b), the explicit-conduction stability bound (section 6.1)
and the direction of the pressure-work and latent-heat effects (Figs. 9-11)."""
import os

import numpy as np
import pytest
from scipy.optimize import curve_fit

from paper_1705_10045_amd import inputs as I

THETA = 1.0 / 3.0
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                key, val = line.split("=")
                vals[key.strip()] = float(val)
    return vals


# ---------------------------------------------------------------------------
# Heat conduction and scheme diffusion of energy
# ---------------------------------------------------------------------------
def _linear_update_eigenvalue(q, chi, tau_E):
    """Slowest eigenvalue of the energy-population update linearised about a uniform state at
    rest, for a Fourier mode exp(i q x) on the collapsed 1D velocity set {0, +1, -1} with
    weights {2/3, 1/6, 1/6}.  Collision: g' = g + (w E - g)/tau_E + w chi lap_q E (the
    conduction increment with uniform density, spread in proportion to g); streaming
    multiplies population k by exp(-i q c_k)."""
    c = np.array([0, 1, -1])
    w = np.array([2 / 3, 1 / 6, 1 / 6])
    om = 1.0 / tau_E
    lap = 2.0 * np.cos(q) - 2.0
    C = (1.0 - om) * np.eye(3) + np.outer(w, np.ones(3)) * (om + chi * lap)
    M = np.diag(np.exp(-1j * q * c)) @ C
    ev = np.linalg.eigvals(M)
    return ev[np.argmax(np.abs(ev))]


def _measured_decay(orc, L, chi, tau_E, steps=400, Q=9):
    """Per-step decay factor of a small temperature mode in a uniform fluid at rest
    (barotropic EOS so the mode cannot drive the density, pressure work off)."""
    shape = (1, 1, L)
    x = np.arange(L)
    k = 2 * np.pi / L
    T = (0.8 * (1.0 + 1e-6 * np.cos(k * x))).reshape(shape)
    p = I.physics(flags=I.BAROTROPIC | I.CONDUCTION | I.PSEUDOFORCE, T0_baro=0.8, chi=chi,
                  tau_E=tau_E)
    s = orc.Sim(Q, p, np.full(shape, 0.2), np.zeros((3,) + shape), T)
    amp = []
    for _ in range(2):
        s.step(steps // 2)
        Tm = s.moments()["T"].ravel()
        amp.append((Tm - Tm.mean()) @ np.cos(k * x))
    return (amp[1] / amp[0]) ** (1.0 / (steps // 2))


@pytest.mark.parametrize("L,chi,tau_E,steps,tol", [(16, 0.01, 0.53, 400, 1e-8),
                                                   (32, 0.1, 0.6, 400, 1e-8),
                                                   (24, 0.0, 0.7, 400, 1e-8),
                                                   (32, 0.1, 0.503, 2400, 1e-7)])
def test_temperature_mode_decays_at_linearised_rate(orc, L, chi, tau_E, steps, tol):
    """The oracle's nonlinear multi-pass step reproduces the eigenvalue of the linearised
    energy update computed independently here (numpy eigensolver).  Near tau_E = 1/2 the
    non-conserved modes decay only as |1 - 1/tau_E|^t (0.988 against 0.996 for the slow mode
    at tau_E = 0.503), so that case runs longer and is limited by rounding to ~3e-8."""
    lam = _linear_update_eigenvalue(2 * np.pi / L, chi, tau_E)
    assert abs(lam.imag) < 1e-12
    assert _measured_decay(orc, L, chi, tau_E, steps=steps) == pytest.approx(lam.real, rel=tol)


def test_scheme_diffusion_value_printed_in_paper(orc):
    """Section 6.1: with tau_E = 0.503 the scheme diffusion of energy is
    D_E = theta (tau_E - 1/2) = 0.001 h^2/dt; with chi = 0 a long temperature wave decays at
    exp(-D_E k^2 t)."""
    g = _golden("paper_values.txt")
    L = 64
    k = 2 * np.pi / L
    rate = -np.log(_measured_decay(orc, L, 0.0, g["tau_E_scheme_test"], steps=2000)) / k ** 2
    assert rate == pytest.approx(g["D_E_scheme_test"], rel=0.01)
    assert THETA * (g["tau_E_scheme_test"] - 0.5) == pytest.approx(g["D_E_scheme_test"])


def test_conduction_similarity_l_sqrt_chi_t(orc):
    """Fig. 6: l ~ sqrt(chi t).  The decay rate of a temperature wave scales as 1/L^2 and as
    (chi + D_E): halving the wavelength quadruples the rate."""
    r32 = -np.log(_measured_decay(orc, 32, 0.05, 0.53, steps=200))
    r64 = -np.log(_measured_decay(orc, 64, 0.05, 0.53, steps=600))
    assert r32 / r64 == pytest.approx(4.0, rel=0.01)
    k = 2 * np.pi / 64
    assert r64 / k ** 2 == pytest.approx(0.05 + THETA * 0.03, rel=0.01)


# ---------------------------------------------------------------------------
# Sound speed (section 6.2, eq:sspeed, Fig. 8)
# ---------------------------------------------------------------------------
def _sound_speed_sq(orc, flags, c_v, tau_E, L=128, rho0=0.01, T0=0.8, steps=1500):
    shape = (1, 1, L)
    x = np.arange(L)
    k = 2 * np.pi / L
    p = I.physics(flags=flags, c_v=c_v, chi=0.0, tau_E=tau_E)
    rho = (rho0 * (1 + 1e-3 * np.cos(k * x))).reshape(shape)
    s = orc.Sim(9, p, rho, np.zeros((3,) + shape), np.full(shape, T0))
    a = np.empty(steps)
    for t in range(steps):
        a[t] = s.moments()["rho"].ravel() @ np.cos(k * x) * 2 / L
        s.step(1)
    t = np.arange(steps)
    model = lambda t, A, w, ph, G, B, C: A * np.cos(w * t + ph) * np.exp(-G * t) + B + C * t
    popt, _ = curve_fit(model, t, a, p0=[a[0], 0.25 * k, 0, 1e-4, 0, 0], maxfev=20000)
    w, G = popt[1], popt[3]
    return (w * w + G * G) / k ** 2


def test_isothermal_and_adiabatic_sound_speed(orc):
    """Standing wave in the vapour at rho~ = 0.01, T~ = 0.8 (Fig. 8).  Without pressure work the
    isothermal speed c_T^2 = (p_c/rho_c) dp~/drho~ is independent of c_v; with it the model's
    adiabatic speed is c_S^2 = c_T^2 + (dp/dT)_rho p / (rho^2 c_v), linear in 1/c_v, which tends
    to the paper's 24 gamma T~/(3 - rho~)^2 - 6 rho~ (gamma = 1 + (8/3) p_c/(rho_c T_c c_v)) as
    rho -> 0."""
    pc, rho0, T0 = I.P_C, 0.01, 0.8
    cT2 = pc * (24 * T0 / (3 - rho0) ** 2 - 6 * rho0)
    dpdT = pc * 8 * rho0 / (3 - rho0)
    p = pc * (8 * rho0 * T0 / (3 - rho0) - 3 * rho0 ** 2)
    measured_T, measured_S = [], []
    for cv in (0.5 * I.P_C, 2 * I.P_C, 8 * I.P_C):
        c2T = _sound_speed_sq(orc, I.PSEUDOFORCE, cv, 1.0)
        c2S = _sound_speed_sq(orc, I.PSEUDOFORCE | I.WORK, cv, 0.53)
        gamma = 1 + (8.0 / 3.0) * pc / cv
        assert c2T == pytest.approx(cT2, rel=0.01)
        assert c2S == pytest.approx(cT2 + dpdT * p / (rho0 ** 2 * cv), rel=0.01)
        assert c2S == pytest.approx(pc * (24 * gamma * T0 / (3 - rho0) ** 2 - 6 * rho0), rel=0.015)
        measured_T.append(c2T)
        measured_S.append(c2S)
    # isothermal constant, adiabatic linear in 1/c_v
    assert np.ptp(measured_T) < 1e-4 * measured_T[0]
    inv = 1.0 / np.array([0.5 * I.P_C, 2 * I.P_C, 8 * I.P_C])
    fit = np.polyfit(inv, measured_S, 1)
    assert np.abs(np.polyval(fit, inv) - measured_S).max() < 2e-3 * max(measured_S)


# ---------------------------------------------------------------------------
# Galilean invariance (section 6.1, Figs. 5 and 7)
# ---------------------------------------------------------------------------
def _two_phase(orc, shape, u, steps, Q=9):
    rv, rl = I.coexistence(0.8)
    if shape[1] == 1:
        rho = I.two_phase_smooth(I.slab_distance(shape, shape[2] / 3, 0), rl, rv)
    else:
        rho = I.two_phase_smooth(I.sphere_distance(shape, shape[1] * 0.2), rl, rv)
    s = orc.Sim(Q, I.physics(), rho, I.uniform_velocity(shape, u), np.full(shape, 0.8))
    t0 = s.totals()
    s.step(steps)
    return s.moments(), s.totals(), t0


@pytest.mark.parametrize("shape,u,steps", [((1, 1, 192), 0.05, 2000), ((1, 48, 48), 0.05, 200)])
def test_moving_interface_matches_resting_one(orc, shape, u, steps):
    """A liquid slab/drop carried by a uniform flow reproduces the resting one shifted by u t
    (an integer number of nodes here): density within 3% of the liquid-vapour contrast and
    temperature within 0.3%.  The centre of mass moves exactly with the conserved momentum."""
    a, _, _ = _two_phase(orc, shape, (0, 0, 0), steps)
    b, tb, tb0 = _two_phase(orc, shape, (u, 0, 0), steps)
    sh = int(round(u * steps))
    contrast = a["rho"].max() - a["rho"].min()
    for key, tol in (("rho", 0.03 * contrast), ("T", 0.003 * 0.8)):
        assert np.abs(np.roll(b[key], -sh, axis=-1) - a[key]).max() < tol, key
    assert tb[1] == pytest.approx(tb0[1], rel=1e-12)
    assert tb[1] / tb[0] == pytest.approx(u, rel=1e-12)


# ---------------------------------------------------------------------------
# Coexistence (section 3, Fig. 4b)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("Tr,vap_tol", [(0.7, 0.04), (0.8, 0.02), (0.9, 0.01)])
def test_slab_coexistence_near_maxwell(orc, Tr, vap_tol):
    """A flat liquid layer relaxes to bulk densities close to the Maxwell construction (the
    paper reports < 0.2% with A = -0.152 at its own lattice scaling; here the liquid is within
    0.1% and the vapour within a few percent at p_c = 0.02, the deviation shrinking towards T_c)."""
    rv, rl, _ = orc.maxwell(Tr)
    n = 128
    shape = (1, 1, n)
    p = I.physics(flags=I.BAROTROPIC | I.PSEUDOFORCE, T0_baro=Tr)
    rho = I.two_phase_smooth(I.slab_distance(shape, 64, 0), rl, rv)
    s = orc.Sim(9, p, rho, np.zeros((3,) + shape), np.full(shape, Tr))
    s.step(12000)
    r = s.moments()["rho"].ravel()
    liq, vap = r[n // 2], r[0]
    assert abs(liq / rl - 1) < 1e-3
    assert 0 < vap / rv - 1 < vap_tol


def test_coexistence_depends_on_mixing_parameter(orc):
    """A enters only at second order (section 3): it changes the coexistence densities, and the
    paper's A = -0.152 lands closer to the Maxwell vapour density than A = 0."""
    Tr = 0.8
    rv, rl, _ = orc.maxwell(Tr)
    shape = (1, 1, 96)
    rho = I.two_phase_smooth(I.slab_distance(shape, 48, 0), rl, rv)
    err = {}
    for A in (-0.152, 0.0):
        p = I.physics(flags=I.BAROTROPIC | I.PSEUDOFORCE, T0_baro=Tr, A=A)
        s = orc.Sim(9, p, rho, np.zeros((3,) + shape), np.full(shape, Tr))
        s.step(8000)
        err[A] = abs(s.moments()["rho"].ravel()[0] / rv - 1)
    assert err[-0.152] < 0.5 * err[0.0]


# ---------------------------------------------------------------------------
# Stability bound of the explicit conduction (section 6.1)
# ---------------------------------------------------------------------------
def test_conduction_at_chi_0_49_in_1d_is_stable(orc):
    """One-dimensional runs with u = 0.1 and chi dt/h^2 = 0.49 are stable (section 6.1): a
    smoothed temperature step in a single-phase fluid stays bounded by its initial extremes."""
    n = 128
    shape = (1, 1, n)
    d = I.slab_distance(shape, 48, 0)
    s_ = 0.5 * (1 - np.tanh(d / 3.0))
    T = 0.7 + 0.2 * s_
    p = I.physics(flags=I.CONDUCTION | I.PSEUDOFORCE, chi=0.49)
    s = orc.Sim(9, p, np.full(shape, 0.05), I.uniform_velocity(shape, (0.1, 0, 0)), T)
    s.step(3000)
    Tm = s.moments()["T"]
    assert Tm.min() > 0.7 - 1e-3 and Tm.max() < 0.9 + 1e-3
    assert np.ptp(Tm) < 0.05  # and it has diffused


def test_conduction_bound_counts_extended_axes(orc):
    """chi < 0.5/d with d the number of axes the box extends along."""
    p = I.physics(chi=0.3)
    sh2 = (1, 8, 8)
    with pytest.raises(ValueError):
        orc.Sim(9, p, np.full(sh2, 0.3), np.zeros((3,) + sh2), np.full(sh2, 0.8))
    sh1 = (1, 1, 8)
    orc.Sim(9, p, np.full(sh1, 0.3), np.zeros((3,) + sh1), np.full(sh1, 0.8))


# ---------------------------------------------------------------------------
# Spinodal decomposition: pressure work and latent heat (section 6.2-6.3)
# ---------------------------------------------------------------------------
def _spinodal_1d(orc, flags, rhoQ=0.0, steps=6000, n=256):
    shape = (1, 1, n)
    rho = 0.7 * (1 + 0.01 * I.symmetric(17, n)).reshape(shape)
    p = I.physics(flags=flags, chi=0.0, rhoQ=rhoQ)
    s = orc.Sim(9, p, rho, np.zeros((3,) + shape), np.full(shape, 0.8))
    s.step(steps)
    return s.moments()


def test_pressure_work_cools_vapour_and_warms_liquid(orc):
    """Fig. 9: without pressure work the temperature stays at T0 (co-moving energy); with it
    the rarefied vapour cools markedly, roughly to T0 - (p/c_v)(1/rho_vap - 1/rho0), while the
    compressed liquid warms slightly."""
    off = _spinodal_1d(orc, I.PSEUDOFORCE)
    assert np.abs(off["T"] - 0.8).max() < 0.02
    on = _spinodal_1d(orc, I.PSEUDOFORCE | I.WORK)
    vap = on["rho"] < 0.5
    liq = on["rho"] > 1.2
    assert vap.any() and liq.any()
    Tv, Tl = on["T"][vap].mean(), on["T"][liq].mean()
    assert Tv < 0.8 - 0.02 and Tl > 0.8
    rho_v = on["rho"][vap].mean()
    pv = I.P_C * (8 * rho_v * Tv / (3 - rho_v) - 3 * rho_v ** 2)
    estimate = 0.8 - pv / I.physics()["c_v"] * (1 / rho_v - 1 / 0.7)
    assert Tv == pytest.approx(estimate, abs=0.25 * (0.8 - estimate))


def test_latent_heat_released_where_fluid_condenses(orc):
    """Section 5: inside the band rho_1(T) < rho < rho_2(T) energy is released where the fluid
    is being compressed into liquid and absorbed where it expands.  A liquid layer in
    supersaturated vapour, one step from rest: the latent source has the sign of the local
    density change at (nearly) every active node, and it is zero outside the band."""
    n = 128
    shape = (1, 1, n)
    rv, rl = I.coexistence(0.8)
    rho = I.two_phase_smooth(I.slab_distance(shape, 40, 0), rl, 1.15 * rv)
    s = orc.Sim(9, I.physics(), rho, np.zeros((3,) + shape), np.full(shape, 0.8))
    r0 = s.moments()["rho"].ravel()
    s.step(1)
    lat = s.last_sources()["latent"].ravel()
    d = s.moments()["rho"].ravel() - r0
    rv_o, rl_o, _ = orc.maxwell(0.8)
    outside = (r0 <= rv_o) | (r0 >= rl_o)
    assert np.all(lat[outside] == 0)
    m = (lat != 0) & (np.abs(d) > 1e-3 * np.abs(d).max())
    assert m.sum() > 20
    assert np.mean(np.sign(lat[m]) == np.sign(d[m])) > 0.9


def test_stepwise_hot_layer_needs_tau_e_above_0_503_without_conduction(orc):
    """The Fig. 4a state (stepwise T and rho at equal pressure) with the paper's tau_E = 0.503
    and no conduction leaves the EOS domain within 1000 steps: the temperature couples through
    the pressure into a growing short wave.  tau_E = 0.51 runs 1500 steps and keeps T inside
    its initial range; so do a temperature-independent (barotropic) pressure at 0.503 and
    chi = 0.1 at 0.503.  The paper-scale runs of Figs. 5 and 6 therefore use tau_E = 0.51."""
    import scenarios as S

    def run(steps, **kw):
        baro = kw.pop("baro", False)
        case = S.hot_gas_1d(**kw)
        p = dict(case["params"])
        if baro:
            p.update(flags=I.BAROTROPIC | I.PSEUDOFORCE, T0_baro=0.6)
        s = orc.Sim(9, p, case["rho0"], case["u0"], case["T0"])
        s.step(steps)
        return s.moments()["T"]

    with pytest.raises(FloatingPointError):
        run(1000, tau_E=0.503, chi=0.0)
    for kw in (dict(tau_E=0.51, chi=0.0), dict(tau_E=0.503, chi=0.1),
               dict(tau_E=0.503, chi=0.0, baro=True)):
        T = run(1500, **kw)
        assert T.min() > 0.59 and T.max() < 0.96, kw

"""Pins of two oracle functions against values that the mathematics fixes on its own:

- the physical velocity u* = (j + F/2)/rho of eq:ustar, through an exact property of the
  discrete steady state of a one-dimensional two-phase slab;
- the magnitude of the latent-heat source of section 5 on a constructed state whose
  central-difference divergence has a closed form, with the band limits from the textbook
  van der Waals coexistence densities (not from the oracle's own Maxwell solver).

Each test fails if the term it pins is dropped, doubled or has a wrong factor.
"""
import numpy as np
import pytest

from paper_1705_10045_amd import inputs as I

# Textbook van der Waals coexistence at T~ = 0.9 (equal-area rule): reduced vapour and liquid
# densities, the band limits rho_1 and rho_2 of section 5 at that temperature.
RHO1_T09 = 0.425742
RHO2_T09 = 1.657270
PHASE = 0.3


def _slab_1d(orc, Q, n=63, steps=6000):
    """Barotropic liquid slab in vapour on a quasi-1D box (n x 1 x 1), relaxed toward its
    steady state.  Returns the oracle's output u*, the populations' momentum j and rho.  The
    length is odd: on an even periodic box with tau = 1 a checkerboard mode of the momentum
    decays very slowly and would hide the steady state."""
    Tr = 0.8
    rv, rl = I.coexistence(Tr)
    shape = (1, 1, n)
    rho = I.two_phase_smooth(I.slab_distance(shape, n // 3, 0), rl, rv)
    phys = I.physics(flags=I.BAROTROPIC | I.PSEUDOFORCE, T0_baro=Tr, chi=0.0)
    s = orc.Sim(Q, phys, rho, np.zeros((3,) + shape), np.full(shape, Tr))
    s.step(steps)
    m = s.moments()
    N, _ = s.get_pops()
    c, _, _, _, _ = orc.lattice(Q)
    j = np.tensordot(c.T.astype(np.float64), N, axes=(1, 0))   # sum_k c_k N_k, (3, nz, ny, nx)
    s.close()
    return m["u_star"][0].ravel(), j[0].ravel(), m["rho"].ravel()


@pytest.mark.parametrize("Q", [3, 9, 19])
def test_ustar_vanishes_in_steady_1d_slab_while_j_does_not(orc, Q):
    """eq:ustar.  In a steady state of a one-dimensional periodic box, mass conservation makes
    the net population flux through every link equal, and the total momentum (conserved, zero
    from rest, since the force sums to zero) makes it zero.  The momentum a node pulls in is then
    minus the post-collision momentum it sends out, j = -(j + F), so j = -F/2 at every node: the
    physical velocity (j + F/2)/rho is exactly zero while j/rho is not (it is -F/(2 rho) at the
    interfaces).  A u* built with F/2 dropped (j/rho) or doubled ((j + F)/rho) equals -/+ F/(2 rho)
    there instead.  D1Q3, D2Q9 and D3Q19 on n x 1 x 1 boxes all obey this."""
    us, j, rho = _slab_1d(orc, Q)
    jr = np.abs(j / rho).max()
    assert jr > 1e-4                          # the interface force is present
    assert np.abs(us).max() < 1e-10 * jr     # and the physical velocity is zero to rounding


def test_ustar_relaxes_toward_zero_not_toward_j(orc):
    """The same property along the relaxation: |u*| decays with time, while j/rho converges to a
    nonzero profile (-F/(2 rho)); the ratio max|u*| / max|j/rho| falls by orders of magnitude."""
    ratios = []
    for steps in (1000, 3000, 6000):
        us, j, rho = _slab_1d(orc, 9, steps=steps)
        ratios.append(np.abs(us).max() / np.abs(j / rho).max())
    assert ratios[0] > ratios[1] > ratios[2]
    assert ratios[2] < 1e-6 * ratios[0]


def _latent_one_step(orc, rho_value, Tr, U=0.01, n=48, rhoQ=0.01):
    """Latent source of the first step from a uniform density rho_value, uniform temperature Tr
    (also the EOS temperature, barotropic) and u_x = U sin(k x + PHASE), k = 2 pi / n (the phase
    keeps every node off a zero of the divergence).  Uniform rho gives a uniform Phi, so F = 0
    and u* = u."""
    shape = (1, 1, n)
    x = np.arange(n, dtype=np.float64)
    k = 2.0 * np.pi / n
    u0 = np.zeros((3,) + shape)
    u0[0, 0, 0, :] = U * np.sin(k * x + PHASE)
    rho = np.full(shape, rho_value)
    phys = I.physics(flags=I.LATENT | I.BAROTROPIC | I.PSEUDOFORCE, T0_baro=Tr, rhoQ=rhoQ)
    s = orc.Sim(9, phys, rho, u0, np.full(shape, Tr))
    s.step(1)
    lat = s.last_sources()["latent"].ravel()
    s.close()
    return lat, x, k


@pytest.mark.parametrize("rho_value", [0.5, 1.3, 1.6])
def test_latent_source_magnitude_closed_form(orc, rho_value):
    """Section 5: inside the band rho_1(T) < rho < rho_2(T) the source is
    -rho_liq Q / (rho_2 - rho_1) * rho * div u*.  With u*_x = U sin(kx + a) the central
    difference gives div u* = U sin(k) cos(kx + a) exactly, so every node must carry
    -rhoQ rho U sin(k) cos(kx + a) / (rho_2 - rho_1), with rho_2 - rho_1 the textbook width of the
    coexistence band at T~ = 0.9.  Densities away from 1 catch a missing rho factor."""
    U, rhoQ = 0.01, 0.01
    lat, x, k = _latent_one_step(orc, rho_value, 0.9, U=U, rhoQ=rhoQ)
    expect = -rhoQ * rho_value * U * np.sin(k) * np.cos(k * x + PHASE) / (RHO2_T09 - RHO1_T09)
    # the textbook band limits carry 6 decimals
    np.testing.assert_allclose(lat, expect, rtol=2e-6, atol=1e-6 * np.abs(expect).max())


@pytest.mark.parametrize("rho_value", [RHO1_T09 * (1 - 1e-4), RHO2_T09 * (1 + 1e-4)])
def test_latent_source_zero_just_outside_band(orc, rho_value):
    """Outside the coexistence band (vapour below rho_1, liquid above rho_2) no latent heat."""
    lat, _, _ = _latent_one_step(orc, rho_value, 0.9)
    assert np.all(lat == 0.0)


@pytest.mark.parametrize("rho_value", [RHO1_T09 * (1 + 1e-4), RHO2_T09 * (1 - 1e-4)])
def test_latent_source_active_just_inside_band(orc, rho_value):
    lat, _, _ = _latent_one_step(orc, rho_value, 0.9)
    assert np.count_nonzero(lat) == lat.size


@pytest.mark.parametrize("Tr, active", [(0.3999, False), (0.4, True), (0.9989, True),
                                        (0.999, False)])
def test_latent_temperature_window_edges(orc, Tr, active):
    """The source acts for 0.4 <= T~ < 0.999 (the Maxwell table's range, a reading of
    section 5); rho = 1 lies inside the band at every temperature of the window."""
    lat, _, _ = _latent_one_step(orc, 1.0, Tr)
    assert (np.count_nonzero(lat) == lat.size) if active else np.all(lat == 0.0)

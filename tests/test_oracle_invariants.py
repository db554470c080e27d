"""Exact invariants of the full oracle step (sections 2-5): conservation of mass and momentum,
the internal-energy budget, the uniform fixed point, the co-moving invariant that the
pseudoforces of section 4 are built to keep, and exact reductions between lattices."""
import numpy as np
import pytest

from paper_1705_10045_amd import inputs as I


def _droplet2d(shape=(1, 40, 44), radius=9, Tr=0.8, u=(0.03, -0.02, 0.0), **over):
    p = I.physics(**over)
    rv, rl = I.coexistence(Tr)
    rho = I.with_uniform_noise(I.two_phase_smooth(I.sphere_distance(shape, radius), rl, rv), 7,
                               0.01)
    return 9, p, rho, I.uniform_velocity(shape, u), np.full(shape, Tr)


def _droplet3d(shape=(14, 16, 18), radius=4.5, Tr=0.8, u=(0.03, 0.01, -0.02), **over):
    p = I.physics(**over)
    rv, rl = I.coexistence(Tr)
    rho = I.with_uniform_noise(I.two_phase_smooth(I.sphere_distance(shape, radius), rl, rv), 8,
                               0.01)
    return 19, p, rho, I.uniform_velocity(shape, u), np.full(shape, Tr)


CASES = {"d2q9": _droplet2d, "d3q19": _droplet3d}


@pytest.mark.parametrize("case", sorted(CASES))
def test_mass_and_momentum_conserved(orc, case):
    """Collision and EDM conserve mass; EDM adds F per node and the force sums to zero on a
    periodic box; streaming permutes populations (eq:lbe, eq:edm, eq:hydro)."""
    Q, p, rho, u, T = CASES[case]()
    s = orc.Sim(Q, p, rho, u, T)
    t0 = s.totals()
    s.step(60)
    t1 = s.totals()
    assert t1[0] == pytest.approx(t0[0], rel=1e-13)
    scale = t0[0] * 0.05
    assert np.allclose(t1[1:4], t0[1:4], atol=1e-13 * scale)


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("tau_E", [0.53, 0.8, 1.0])
def test_energy_conserved_without_work_and_latent(orc, case, tau_E):
    """With the pressure work and latent heat off, sum E is exactly conserved: BGK and the
    pseudoforces conserve sum g_k, dg(1) injects the conduction term, which is a pure flux form."""
    Q, p, rho, u, T = CASES[case](tau_E=tau_E, flags=I.CONDUCTION | I.PSEUDOFORCE, chi=0.05)
    rng_T = T * (1.0 + 0.02 * I.symmetric(3, T.size).reshape(T.shape))
    s = orc.Sim(Q, p, rho, u, rng_T)
    e0 = s.totals()[4]
    s.step(40)
    assert s.totals()[4] == pytest.approx(e0, rel=1e-13)


@pytest.mark.parametrize("case", sorted(CASES))
def test_energy_budget_with_work_and_latent(orc, case):
    """With every term on, the change of sum E over a step equals the summed work and latent
    sources of that step: the LB transport and the conduction contribute exactly zero."""
    Q, p, rho, u, T = CASES[case](rhoQ=0.01)
    s = orc.Sim(Q, p, rho, u, T)
    s.step(5)
    total_latent = 0.0
    for _ in range(10):
        e0 = s.totals()[4]
        s.step(1)
        src = s.last_sources()
        de = s.totals()[4] - e0
        assert de == pytest.approx(src["work"].sum() + src["latent"].sum(), abs=1e-13 * e0)
        assert abs(src["cond"].sum()) < 1e-15 * e0
        total_latent += np.abs(src["latent"]).sum()
    assert total_latent > 0  # the interface band is actually exercised


@pytest.mark.parametrize("Q,shape", [(9, (1, 6, 7)), (19, (5, 6, 7))])
def test_uniform_state_is_a_fixed_point(orc, Q, shape):
    """Uniform rho, T, u: the force, every energy source and the collision increments vanish, so
    the moments stay put (the state only translates, which is invisible when uniform)."""
    p = I.physics()
    u = (0.04, -0.03, 0.02 if Q == 19 else 0.0)
    s = orc.Sim(Q, p, np.full(shape, 0.9), I.uniform_velocity(shape, u), np.full(shape, 0.85))
    s.step(25)
    m = s.moments()
    assert np.abs(m["rho"] - 0.9).max() < 1e-14
    assert np.abs(m["T"] - 0.85).max() < 1e-14
    for a in range(3):
        assert np.abs(m["u_star"][a] - u[a]).max() < 1e-15


@pytest.mark.parametrize("case", sorted(CASES))
def test_pseudoforces_keep_temperature_comoving(orc, case):
    """Section 4: with tau_E = tau, no work/conduction/latent and a uniform T0, the energy
    populations stay proportional to the density populations (g_k = c_v T0 N_k): the pseudoforce
    gives g the same kick as N, so T = T0 at every node and step.  Without the pseudoforces the
    energy leaks across the interface (the parasitic diffusion of Fig. 1)."""
    Q, p, rho, u, T = CASES[case](tau_E=1.0, flags=I.PSEUDOFORCE)
    s = orc.Sim(Q, p, rho, u, T)
    s.step(80)
    Tm = s.moments()["T"]
    assert np.abs(Tm - T).max() < 1e-13
    N, g = s.get_pops()
    assert np.allclose(g, p["c_v"] * T[None] * N, rtol=1e-12, atol=0)

    Q, p, rho, u, T = CASES[case](tau_E=1.0, flags=0)
    s = orc.Sim(Q, p, rho, u, T)
    s.step(5)
    dev = np.abs(s.moments()["T"] - T).max()
    assert dev > 0.05 * T.max()  # drifts by a few percent of T per step at the interface


def test_barotropic_eos_ignores_temperature(orc):
    """Section 4 barotropic variant: with the EOS at fixed T0, the density evolution does not
    depend on the energy populations at all."""
    Q, p, rho, u, T = _droplet2d(flags=I.BAROTROPIC | I.PSEUDOFORCE | I.CONDUCTION, T0_baro=0.8)
    s1 = orc.Sim(Q, p, rho, u, T)
    s2 = orc.Sim(Q, p, rho, u, T * 0.9)
    s1.step(30)
    s2.step(30)
    assert np.array_equal(s1.moments()["rho"], s2.moments()["rho"])
    assert not np.array_equal(s1.moments()["E"], s2.moments()["E"])


def _slab_1d(orc, Q, n, steps, axis, flags=I.ALL_TERMS):
    """Quasi-1D slab on an (n x 1 x 1) box with the slab normal along `axis`."""
    shape = [1, 1, 1]
    shape[2 - axis] = n
    shape = tuple(shape)
    rv, rl = I.coexistence(0.8)
    rho = I.two_phase_smooth(I.slab_distance(shape, n / 3, axis), rl, rv)
    rho = I.with_uniform_noise(rho, 21, 0.01)
    u = [0.0, 0.0, 0.0]
    u[axis] = 0.05
    T = np.full(shape, 0.8) * (1 + 0.01 * I.symmetric(5, n).reshape(shape))
    s = orc.Sim(Q, I.physics(flags=flags, rhoQ=0.005), rho, I.uniform_velocity(shape, u), T)
    s.step(steps)
    m = s.moments()
    return {k: (v.reshape(-1) if k != "u_star" else v[axis].reshape(-1)) for k, v in m.items()}


def test_dimension_reduction_d1q3_d2q9_d3q19(orc):
    """Fields uniform across the box: D3Q19 with ny = nz = 1 and D2Q9 with ny = 1 both collapse
    onto D1Q3 (weights {2/3, 1/6, 1/6}, force coefficients summing to alpha), so every moment
    agrees to rounding with the paper's own one-dimensional lattice, a separate velocity set
    with its own tables; and the result does not depend on which axis the slab is normal to."""
    a = _slab_1d(orc, 3, 64, 300, axis=0)
    b = _slab_1d(orc, 9, 64, 300, axis=0)
    c = _slab_1d(orc, 19, 64, 300, axis=0)
    d = _slab_1d(orc, 9, 64, 300, axis=1)
    e = _slab_1d(orc, 19, 64, 300, axis=2)
    for other in (b, c, d, e):
        for k in ("rho", "u_star", "E", "T"):
            assert np.allclose(a[k], other[k], rtol=1e-11, atol=1e-14), k


def test_population_roundtrip_continues_identically(orc):
    """The state is exactly {N, g}: copying the populations into a fresh simulation and
    continuing gives bit-identical results (checkpoint/restore)."""
    Q, p, rho, u, T = _droplet2d()
    s1 = orc.Sim(Q, p, rho, u, T)
    s1.step(20)
    N, g = s1.get_pops()
    s2 = orc.Sim(Q, p, rho, u, T)
    s2.set_pops(N, g)
    s1.step(15)
    s2.step(15)
    for k in ("rho", "u_star", "E", "T"):
        assert np.array_equal(s1.moments()[k], s2.moments()[k])


def test_rejects_invalid_parameters(orc):
    Q, p, rho, u, T = _droplet2d()
    bad = [dict(tau=0.5), dict(tau_E=0.4), dict(chi=0.25), dict(p_c=0.0)]
    for over in bad:
        with pytest.raises(ValueError):
            orc.Sim(Q, dict(p, **over), rho, u, T)
    # the explicit-conduction bound chi < 0.5/d (section 6.1) applies only with conduction on
    orc.Sim(Q, dict(p, chi=0.25, flags=I.PSEUDOFORCE), rho, u, T)
    with pytest.raises(ValueError):
        orc.Sim(Q, p, np.where(rho > 1, 3.5, rho), u, T)  # beyond the vdW co-volume
    with pytest.raises(ValueError):
        orc.Sim(Q, p, rho, u, -T)


def test_unstable_state_reported(orc):
    """A state driven outside the EOS domain (Phi^2 <= 0) stops with an error instead of
    producing NaNs; here a sharp voxel step at a large density ratio and a tiny tau."""
    shape = (1, 24, 24)
    rho = I.two_phase(I.sphere_mask(shape, 6), 2.9, 0.02)
    s = orc.Sim(9, I.physics(tau=0.501), rho, I.uniform_velocity(shape, (0.3, 0, 0)),
                np.full(shape, 0.6))
    with pytest.raises(FloatingPointError):
        s.step(200)

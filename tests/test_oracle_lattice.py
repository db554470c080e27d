"""Pins of the oracle's lattice tables and equilibrium (section 2, eq:feq; section 3 force
coefficients) against identities that any correct D1Q3 / D2Q9 / D3Q19 velocity set must
satisfy."""
import itertools

import numpy as np
import pytest

THETA = 1.0 / 3.0


@pytest.mark.parametrize("Q,D,alpha", [(3, 1, 1.0), (9, 2, 1.5), (19, 3, 3.0)])
def test_velocity_set_shape(orc, Q, D, alpha):
    c, w, G, a, d = orc.lattice(Q)
    assert d == D and a == alpha
    # distinct velocities, one rest particle, |c|^2 in {1, 2} otherwise
    assert len({tuple(v) for v in c}) == Q
    sq = (c * c).sum(1)
    assert sq[0] == 0 and set(sq[1:]) == ({1} if D == 1 else {1, 2})
    if D == 1:
        assert (c[:, 1:] == 0).all()
    elif D == 2:
        assert (c[:, 2] == 0).all()
        assert (sq == 1).sum() == 4 and (sq == 2).sum() == 4
    else:
        assert (sq == 1).sum() == 6 and (sq == 2).sum() == 12
        assert (np.abs(c).sum(1) <= 2).all()  # no (1,1,1) corners in D3Q19
    # every direction has its opposite with the same weight and force coefficient
    for k in range(Q):
        opp = [j for j in range(Q) if (c[j] == -c[k]).all()]
        assert len(opp) == 1
        assert w[opp[0]] == w[k] and G[opp[0]] == G[k]


@pytest.mark.parametrize("Q", [3, 9, 19])
def test_weight_moments_isotropic_to_fourth_order(orc, Q):
    """sum w = 1, sum w c = 0, sum w c c = theta I, odd moments vanish,
    sum w c_a c_b c_c c_d = theta^2 (d_ab d_cd + d_ac d_bd + d_ad d_bc) on the D active axes."""
    c, w, _, _, D = orc.lattice(Q)
    c = c[:, :D].astype(float)
    I = np.eye(D)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(np.einsum("k,ka->a", w, c), 0, atol=1e-15)
    assert np.allclose(np.einsum("k,ka,kb->ab", w, c, c), THETA * I, atol=1e-15)
    assert np.allclose(np.einsum("k,ka,kb,kc->abc", w, c, c, c), 0, atol=1e-15)
    m4 = np.einsum("k,ka,kb,kc,kd->abcd", w, c, c, c, c)
    iso = THETA ** 2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I)
                        + np.einsum("ad,bc->abcd", I, I))
    assert np.allclose(m4, iso, atol=1e-15)


@pytest.mark.parametrize("Q", [3, 9, 19])
def test_force_coefficients(orc, Q):
    """sum G e = 0, sum G e e e = 0 and sum G e e = 2 alpha I, so that the discrete force of
    section 3 reduces to grad(Phi^2) for smooth Phi."""
    c, _, G, alpha, D = orc.lattice(Q)
    c = c[:, :D].astype(float)
    assert G[0] == 0
    assert np.allclose(np.einsum("k,ka->a", G, c), 0)
    assert np.allclose(np.einsum("k,ka,kb->ab", G, c, c), 2 * alpha * np.eye(D))
    assert np.allclose(np.einsum("k,ka,kb,kc->abc", G, c, c, c), 0)
    # nearest neighbours G = 1, next-nearest 1/4 (D2Q9) or 1/2 (D3Q19) (section 3)
    sq = (c * c).sum(1)
    assert (G[sq == 1] == 1).all()
    assert (G[sq == 2] == (0.25 if Q == 9 else 0.5)).all()


@pytest.mark.parametrize("Q", [3, 9, 19])
def test_collapse_to_d1q3(orc, Q):
    """Grouping directions by c_x gives the D1Q3 weights {2/3, 1/6, 1/6} of section 2 and a
    force coefficient sum equal to alpha per side (alpha = 1 for D1Q3 after dividing)."""
    c, w, G, alpha, _ = orc.lattice(Q)
    for cx, wexp in ((0, 2 / 3), (1, 1 / 6), (-1, 1 / 6)):
        assert w[c[:, 0] == cx].sum() == pytest.approx(wexp, abs=1e-15)
    assert G[c[:, 0] == 1].sum() == pytest.approx(alpha)
    assert G[c[:, 0] == -1].sum() == pytest.approx(alpha)


@pytest.mark.parametrize("Q", [3, 9, 19])
def test_equilibrium_moments(orc, Q):
    """eq:feq has density rho, momentum rho u and momentum flux rho theta I + rho u u exactly
    (a consequence of the lattice identities above, evaluated on the oracle's function)."""
    c, _, _, _, D = orc.lattice(Q)
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho = rng.uniform(0.1, 2.5)
        u = np.zeros(3)
        u[:D] = rng.uniform(-0.2, 0.2, D)
        f = orc.equilibrium(Q, rho, u)
        cf = c.astype(float)
        assert f.sum() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(cf.T @ f, rho * u, atol=1e-15)
        Pi = np.einsum("k,ka,kb->ab", f, cf, cf)[:D, :D]
        assert np.allclose(Pi, rho * THETA * np.eye(D) + rho * np.outer(u[:D], u[:D]), atol=1e-14)


@pytest.mark.parametrize("Q", [3, 9, 19])
def test_edm_increment_moments(orc, Q):
    """eq:edm: dN = Neq(rho,u+du) - Neq(rho,u) adds no mass and exactly rho du of momentum."""
    c, _, _, _, D = orc.lattice(Q)
    rng = np.random.default_rng(5)
    rho = 0.7
    u = np.zeros(3)
    du = np.zeros(3)
    u[:D] = rng.uniform(-0.1, 0.1, D)
    du[:D] = rng.uniform(-0.05, 0.05, D)
    dN = orc.equilibrium(Q, rho, u + du) - orc.equilibrium(Q, rho, u)
    assert abs(dN.sum()) < 1e-15
    assert np.allclose(c.T.astype(float) @ dN, rho * du, atol=1e-15)


def test_equilibrium_at_rest_is_weights(orc):
    for Q in (9, 19):
        _, w, _, _, _ = orc.lattice(Q)
        assert np.allclose(orc.equilibrium(Q, 1.3, [0, 0, 0]), 1.3 * w, rtol=1e-15)


def test_lattices_are_symmetric_under_axis_permutation(orc):
    """The D3Q19 set maps onto itself under every permutation and reflection of axes."""
    c, w, G, _, _ = orc.lattice(19)
    table = {tuple(v): (w[k], G[k]) for k, v in enumerate(c)}
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            for k in range(19):
                v = tuple(signs[a] * c[k][perm[a]] for a in range(3))
                assert table[v] == (w[k], G[k])

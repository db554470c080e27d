"""Pins of the oracle's neighbourhood operators: the isotropic pseudopotential force (section 3),
the central-difference divergence (section 6.2) and the conservative conduction term (section 4),
against closed forms on polynomial fields and exact conservation identities."""
import numpy as np
import pytest

A = -0.152


def _coords(shape):
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(float), y.astype(float), z.astype(float)


def _interior(shape, margin):
    nz, ny, nx = shape
    sl = [slice(margin, nz - margin) if nz > 1 else slice(None),
          slice(margin, ny - margin), slice(margin, nx - margin)]
    return tuple(sl)


@pytest.mark.parametrize("Q,shape", [(9, (1, 12, 14)), (19, (10, 11, 12))])
@pytest.mark.parametrize("a_mix", [A, 0.0, 0.3])
def test_force_exact_for_linear_phi(orc, Q, shape, a_mix):
    """For Phi = a + b.x the discrete force equals 2 Phi grad Phi = grad(Phi^2) exactly,
    for any A (away from the periodic seam)."""
    x, y, z = _coords(shape)
    b = np.array([0.013, -0.021, 0.017 if Q == 19 else 0.0])
    Phi = 0.6 + b[0] * x + b[1] * y + b[2] * z
    F = orc.force(Q, Phi, a_mix)
    sl = _interior(shape, 1)
    for a in range(3):
        assert np.allclose(F[a][sl], 2 * Phi[sl] * b[a], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("Q,shape", [(9, (1, 4, 20)), (19, (4, 4, 20))])
def test_force_quadratic_phi_closed_form(orc, Q, shape):
    """For Phi = q X^2 varying along x only, the nearest and diagonal terms with e_x = +1 sum to
    alpha, giving F_x = A (Phi^2(x+1) - Phi^2(x-1)) + (1 - 2A) Phi (Phi(x+1) - Phi(x-1))
    = q^2 (4 X^3 + 8 A X): the continuum grad(Phi^2) = 4 q^2 X^3 plus an A-dependent lattice term."""
    x, _, _ = _coords(shape)
    q, x0 = 0.01, 9.5
    X = x - x0
    Phi = q * X ** 2 + 0.0
    F = orc.force(Q, Phi, A)
    sl = (slice(None), slice(None), slice(1, shape[2] - 1))
    assert np.allclose(F[0][sl], q * q * (4 * X[sl] ** 3 + 8 * A * X[sl]), rtol=1e-12, atol=1e-16)
    assert np.allclose(F[1], 0, atol=1e-16) and np.allclose(F[2], 0, atol=1e-16)


@pytest.mark.parametrize("Q,shape", [(9, (1, 9, 13)), (19, (7, 6, 5))])
def test_force_sums_to_zero_on_periodic_box(orc, Q, shape):
    """Pair antisymmetry: the total force on a periodic lattice vanishes (momentum conservation)."""
    Phi = np.random.default_rng(11).uniform(0.2, 0.8, shape)
    F = orc.force(Q, Phi, A)
    for a in range(3):
        assert abs(F[a].sum()) < 1e-13
    # and a uniform Phi exerts no force at all
    assert np.abs(orc.force(Q, np.full(shape, 0.4), A)).max() < 1e-15


def test_force_rotation_covariance(orc):
    """Rotating Phi by 90 degrees about z rotates F the same way (isotropy of the stencil)."""
    Phi = np.random.default_rng(2).uniform(0.2, 0.8, (1, 8, 8))
    F = orc.force(9, Phi, A)
    Pr = np.rot90(Phi, k=1, axes=(1, 2)).copy()   # (y, x) -> rotated
    Fr = orc.force(9, Pr, A)
    # np.rot90 on (y, x) axes maps a vector (vx, vy) to (vy, -vx) in array index terms
    assert np.allclose(Fr[0], np.rot90(F[1], k=1, axes=(1, 2)), atol=1e-15)
    assert np.allclose(Fr[1], -np.rot90(F[0], k=1, axes=(1, 2)), atol=1e-15)


@pytest.mark.parametrize("D,shape", [(2, (1, 10, 11)), (3, (9, 10, 11))])
def test_divergence_exact_for_quadratic(orc, D, shape):
    """Central differences are exact for quadratics: div(x^2, y^2, z^2) = 2(x + y + z)."""
    x, y, z = _coords(shape)
    u = np.stack([x ** 2, 0.5 * y ** 2, (z ** 2 if D == 3 else 0 * z)])
    div = orc.divergence(D, u)
    expect = 2 * x + y + (2 * z if D == 3 else 0)
    sl = _interior(shape, 1)
    assert np.allclose(div[sl], expect[sl], atol=1e-12)
    # a periodic field has zero total divergence
    r = np.random.default_rng(4).normal(size=(3,) + shape)
    assert abs(orc.divergence(D, r).sum()) < 1e-12


@pytest.mark.parametrize("D,shape", [(2, (1, 10, 12)), (3, (8, 9, 10))])
def test_conduction_closed_forms(orc, D, shape):
    x, y, z = _coords(shape)
    cv, chi = 0.08, 0.01
    sl = _interior(shape, 1)
    # uniform rho, T = x^2 + y^2: div(lam grad T) = lam * 4 exactly
    rho = np.full(shape, 0.7)
    T = x ** 2 + y ** 2
    out = orc.conduction(D, cv, chi, rho, T)
    assert np.allclose(out[sl], 0.7 * cv * chi * 4, rtol=1e-12)
    # linear rho and linear T along x: d/dx(lam dT/dx) = c_v chi rho' T' exactly
    rho = 0.5 + 0.02 * x
    T = 0.8 + 0.003 * x
    out = orc.conduction(D, cv, chi, rho, T)
    assert np.allclose(out[sl], cv * chi * 0.02 * 0.003, rtol=1e-9, atol=1e-18)
    # linear T and uniform rho: no heat flux divergence
    out = orc.conduction(D, cv, chi, np.full(shape, 1.1), 0.8 + 0.01 * y)
    assert np.abs(out[sl]).max() < 1e-15


def test_conduction_conserves_energy(orc):
    """Face fluxes cancel pairwise: the total over a periodic box is zero for any rho, T."""
    rng = np.random.default_rng(9)
    for D, shape in ((2, (1, 9, 10)), (3, (6, 7, 8))):
        rho = rng.uniform(0.2, 2.0, shape)
        T = rng.uniform(0.6, 0.95, shape)
        out = orc.conduction(D, 0.08, 0.1, rho, T)
        assert abs(out.sum()) < 1e-15 * np.abs(out).sum() * 100 + 1e-17
        # heat flows from hot to cold: the hottest node loses energy
        i = np.unravel_index(np.argmax(T), shape)
        assert out[i] < 0

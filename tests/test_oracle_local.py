"""Pins of the oracle's local operators (Sec. 2) against their defining
moment identities: the second-order equilibrium reproduces n, n u and
n (c_s^2 delta + u u); the Guo term has moments 0, F and u F + F u; BGK with
Guo forcing conserves each concentration and changes the local momentum by
exactly the total force when tau_A = tau_B (Sec. 2, after eq. lbm)."""
import numpy as np
import pytest

from oracle import oracle as O

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments(dim):
    rng = np.random.default_rng(11)
    xi, w = O.lattice(dim)
    for _ in range(20):
        n = rng.uniform(0.01, 2.0)
        u = rng.uniform(-0.1, 0.1, 3)
        if dim == 2:
            u[2] = 0.0
        feq = O.equilibrium(dim, n, u)
        assert abs(feq.sum() - n) < 1e-14
        np.testing.assert_allclose(xi.T @ feq, n * u, atol=1e-15)
        second = np.einsum("i,ia,ib->ab", feq, xi, xi)
        want = n * (CS2 * np.eye(3) + np.outer(u, u))
        if dim == 2:
            want[2, :] = 0.0
            want[:, 2] = 0.0
        np.testing.assert_allclose(second, want, atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_guo_source_moments(dim):
    rng = np.random.default_rng(12)
    xi, w = O.lattice(dim)
    for _ in range(20):
        u = rng.uniform(-0.1, 0.1, 3)
        F = rng.uniform(-0.05, 0.05, 3)
        if dim == 2:
            u[2] = F[2] = 0.0
        S = O.guo_source(dim, u, F)
        assert abs(S.sum()) < 1e-16
        np.testing.assert_allclose(xi.T @ S, F, atol=1e-16)
        second = np.einsum("i,ia,ib->ab", S, xi, xi)
        np.testing.assert_allclose(second, np.outer(u, F) + np.outer(F, u), atol=1e-16)


def _random_fields(shape, rng, lo=0.05, hi=1.0):
    return rng.uniform(lo, hi, shape), rng.uniform(lo, hi, shape)


@pytest.mark.parametrize("dim,order", [(2, 4), (2, 8), (3, 4), (3, 6)])
@pytest.mark.parametrize("tau", [0.7, 1.0, 1.7])
def test_collision_conserves_mass_and_adds_force(dim, order, tau):
    rng = np.random.default_rng(13)
    shape = (7, 9) if dim == 2 else (6, 5, 7)
    o = O.Oracle(dim, order, shape, tau=tau, g=((-0.3, 1.4), (1.4, 0.2)))
    f = rng.uniform(0.01, 0.1, (2, o.q) + o.shape)
    o.set_populations(f)
    n = o.density()
    F = o.force(n)
    xi, w = O.lattice(dim)
    for site in (0, 17, o.N - 1):
        z, y, x = np.unravel_index(site, o.shape)
        out = o.collide_site(site)
        fin = f[:, :, z, y, x]
        assert abs(out[0].sum() - fin[0].sum()) < 1e-15
        assert abs(out[1].sum() - fin[1].sum()) < 1e-15
        dmom = (out - fin).sum(axis=0) @ xi
        np.testing.assert_allclose(dmom, F[0, :, z, y, x] + F[1, :, z, y, x], atol=1e-15)


def test_collision_at_tau_one_is_equilibrium_plus_half_source():
    """With tau = 1 the update collapses to f* = f^eq + S/2 (eq. lbm)."""
    rng = np.random.default_rng(14)
    o = O.Oracle(3, 6, (5, 5, 6), tau=1.0, g=((0.0, 1.8), (1.8, -0.2)))
    f = rng.uniform(0.01, 0.1, (2, 19) + o.shape)
    o.set_populations(f)
    n = o.density()
    F = o.force(n)
    u = o.velocity()
    site = 31
    z, y, x = np.unravel_index(site, o.shape)
    out = o.collide_site(site)
    for J in range(2):
        want = (O.equilibrium(3, n[J, z, y, x], u[:, z, y, x])
                + 0.5 * O.guo_source(3, u[:, z, y, x], F[J, :, z, y, x]))
        np.testing.assert_allclose(out[J], want, atol=1e-16)

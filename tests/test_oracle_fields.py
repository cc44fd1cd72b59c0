"""Pins of the oracle's field operators and of its full time step.

* eq. sc_force: on a periodic lattice every coupling term is pairwise
  antisymmetric, so sum_x (F_A + F_B) = 0 for symmetric couplings; a uniform
  field feels no force; for a long-wave field the force tends to
  -g_AB n_A grad n_B - g_AA psi_A grad psi_A with the e2 = 1 normalisation.
* the full step against an independent brute-force stepper on tiny lattices.
* stream + collide with G = 0: a shear wave decays with the lattice viscosity
  nu = c_s^2 (tau - 1/2) (textbook BGK result).
* mass of each component and total momentum are conserved over long runs.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2112_02574_amd import inputs
from tests.naive_lbm import Naive

STENCILS = [(2, 4), (2, 6), (2, 8), (3, 4), (3, 6)]


def _shape(dim):
    return (9, 11) if dim == 2 else (7, 6, 9)


@pytest.mark.parametrize("dim,order", STENCILS)
@pytest.mark.parametrize("psi", [O.PSI_N, O.PSI_EXP])
def test_force_sums_to_zero(dim, order, psi):
    rng = np.random.default_rng(21)
    o = O.Oracle(dim, order, _shape(dim), g=((-0.7, 1.8), (1.8, 0.4)), psi_self=psi)
    n = rng.uniform(0.05, 1.1, (2,) + o.shape)
    F = o.force(n)
    tot = F.sum(axis=(2, 3, 4))
    assert np.abs(tot.sum(axis=0)).max() < 1e-12
    # individual components do not vanish, so the test is not vacuous
    assert np.abs(tot[0]).max() > 1e-3


@pytest.mark.parametrize("dim,order", STENCILS)
def test_uniform_field_has_no_force(dim, order):
    o = O.Oracle(dim, order, _shape(dim), g=((-0.7, 1.8), (1.8, 0.4)), psi_self=O.PSI_EXP)
    n = np.empty((2,) + o.shape)
    n[0] = 0.7
    n[1] = 0.3
    assert np.abs(o.force(n)).max() < 1e-15


@pytest.mark.parametrize("dim,order", STENCILS)
def test_long_wave_force_limit(dim, order):
    """F_A -> -g_AB n_A dn_B/dx - g_AA psi_A dpsi_A/dx for a sinusoid along x;
    the error falls like k^2, so doubling the wavelength cuts it ~4x."""
    gAB, gAA = 1.3, -0.6
    errs = []
    for L in (32, 64):
        shape = (3, L) if dim == 2 else (3, 3, L)
        o = O.Oracle(dim, order, shape, g=((gAA, gAB), (gAB, 0.0)), psi_self=O.PSI_EXP)
        x = np.arange(L)
        k = 2 * np.pi / L
        nA = 0.6 + 0.2 * np.sin(k * x)
        nB = 0.5 - 0.1 * np.cos(k * x)
        n = np.empty((2,) + o.shape)
        n[0] = nA
        n[1] = nB
        F = o.force(n)
        dnB = 0.1 * k * np.sin(k * x)
        psA = np.exp(-1.0 / nA)
        dpsA = psA / nA ** 2 * 0.2 * k * np.cos(k * x)
        want = -gAB * nA * dnB - gAA * psA * dpsA
        got = F[0, 0].reshape(-1, L)[0]
        errs.append(np.abs(got - want).max() / np.abs(want).max())
        assert np.abs(F[0, 1]).max() < 1e-15 and np.abs(F[0, 2]).max() < 1e-15
    assert errs[1] < 0.05
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def _vel_map(dim, naive):
    xi, _ = O.lattice(dim)
    order = [tuple(v) for v, _ in naive.vel]
    return [order.index(tuple(v)) for v in xi]


@pytest.mark.parametrize("dim,order,shape,psi", [
    (2, 4, (8, 8), O.PSI_N), (2, 8, (8, 8), O.PSI_N), (2, 6, (8, 7), O.PSI_EXP),
    (3, 4, (5, 6, 6), O.PSI_N), (3, 6, (6, 5, 6), O.PSI_EXP)])
def test_brute_force_agreement(dim, order, shape, psi):
    rng = np.random.default_rng(22)
    g = ((-0.2, 1.8), (1.8, 0.0)) if psi == O.PSI_N else ((-0.9, 1.2), (1.2, -0.5))
    tau = 1.0 if dim == 3 else 0.8
    nA = rng.uniform(0.2, 1.0, shape)
    nB = rng.uniform(0.2, 1.0, shape)
    o = O.Oracle(dim, order, shape, tau=tau, g=g, psi_self=psi)
    o.set_density(nA, nB)
    nv = Naive(dim, order, shape, tau, g, psi)
    nv.set_density(nA, nB)
    steps = 6 if dim == 3 else 12
    o.run(steps)
    for _ in range(steps):
        nv.step()
    fn = nv.populations()[:, _vel_map(dim, nv)]
    assert np.abs(o.f - fn.reshape(o.f.shape)).max() < 1e-13


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_shear_wave_viscosity(tau):
    """u_x(y) = U sin(k y) decays as exp(-nu k^2 t), nu = c_s^2 (tau - 1/2)."""
    L = 64
    # wave along y, 4 nodes in x
    o = O.Oracle(2, 4, (L, 4), tau=tau, g=((0.0, 0.0), (0.0, 0.0)))
    y = np.arange(L)[:, None] * np.ones((1, 4))
    k = 2 * np.pi / L
    U = 1e-4
    f = np.zeros((2, 9, 1, L, 4))
    for J, nJ in enumerate((0.6, 0.4)):
        for ix in range(4):
            for iy in range(L):
                u = np.array([U * np.sin(k * iy), 0.0, 0.0])
                f[J, :, 0, iy, ix] = O.equilibrium(2, nJ, u)
    o.set_populations(f)
    def amp():
        u = o.velocity()[0, 0, :, 0]
        return 2.0 / L * np.sum(u * np.sin(k * np.arange(L)))
    a0 = amp()
    steps = 400
    o.run(steps)
    a1 = amp()
    nu_meas = -np.log(a1 / a0) / (k * k * steps)
    nu = (tau - 0.5) / 3.0
    assert abs(nu_meas / nu - 1.0) < 2e-3, (nu_meas, nu)


@pytest.mark.parametrize("dim,order", [(2, 8), (3, 6)])
def test_conservation_over_run(dim, order):
    """Noisy droplet near coexistence (a deep quench from a mixed state is not
    a stable start for this coupling): masses and total momentum stay put."""
    from paper_2112_02574_amd import inputs
    rng = np.random.default_rng(23)
    L = 32 if dim == 2 else 16
    shape = (L, L) if dim == 2 else (L, L, L)
    o = O.Oracle(dim, order, shape, tau=1.0, g=((-0.05, 1.4), (1.4, 0.05)))
    nA, nB = inputs.droplet(L, L, None if dim == 2 else L, R=L / 4)
    nA = nA + 1e-3 * rng.uniform(-1, 1, shape)
    o.set_density(nA, nB)
    s0 = o.stats()
    o.run(400 if dim == 2 else 60)
    s1 = o.stats()
    np.testing.assert_allclose(s1["mass"], s0["mass"], rtol=1e-13)
    assert np.abs(s1["momentum"]).max() < 1e-11 * s0["mass"].sum()
    assert s1["n_nonfinite"] == 0
    assert s1["max_u"] > 1e-5


def test_delta_u_of_a_decaying_shear_wave():
    """Criterion (ii) of Sec. 4 on u_x(y) = U sin(k y) exp(-nu k^2 t): the mean
    of |u(t + dt) - u(t)| is (2/pi) U exp(-nu k^2 t) (1 - exp(-nu k^2 dt))
    (mean of |sin| over a period is 2/pi), and a state at rest gives 0."""
    L, tau = 64, 0.8
    o = O.Oracle(2, 4, (L, 4), tau=tau, g=((0.0, 0.0), (0.0, 0.0)))
    k, U = 2 * np.pi / L, 1e-4
    f = np.zeros((2, 9, 1, L, 4))
    for J, nJ in enumerate((0.6, 0.4)):
        for iy in range(L):
            f[J, :, 0, iy, :] = O.equilibrium(2, nJ, np.array([U * np.sin(k * iy), 0.0, 0.0]))[:, None]
    o.set_populations(f)
    o.run(200)
    u0 = o.velocity()
    o.run(400)
    u1 = o.velocity()
    nu = (tau - 0.5) / 3.0
    want = 2 / np.pi * U * np.exp(-nu * k * k * 200) * (1 - np.exp(-nu * k * k * 400))
    assert abs(O.delta_u(u1, u0) / want - 1) < 5e-3
    assert O.delta_u(u1, u1) == 0.0


def test_excess_com_locates_the_droplet():
    """A droplet centred on c = floor(L/2) has its centre there; the same
    droplet rolled by (2, -1, 1) nodes moves it by exactly that.  (With even
    L the cell [c - L/2, c + L/2) is one node short of symmetric; the tanh
    tails there, ~exp(-2 (L/2 - R - shift)), offset the centre slightly.)"""
    L = 32
    nA, nB = inputs.droplet(L, L, L, R=5.0)
    n = np.stack([nA, nB])
    com, rich = O.excess_com(n, (L, L, L))
    assert rich == 0 and np.abs(com - L // 2).max() < 1e-8
    n2 = np.roll(n, shift=(1, -1, 2), axis=(1, 2, 3))
    com2, _ = O.excess_com(n2, (L, L, L))
    assert np.abs(com2 - (L // 2 + np.array([2, -1, 1]))).max() < 1e-7
    com3, rich3 = O.excess_com(np.stack([nB, nA]), (L, L, L))
    assert rich3 == 1 and np.abs(com3 - L // 2).max() < 1e-8


@pytest.mark.parametrize("dim,order,shape,psi", [
    (2, 4, (8, 8), O.PSI_N), (2, 8, (8, 7), O.PSI_EXP), (3, 6, (5, 6, 6), O.PSI_N)])
def test_brute_force_agreement_unequal_tau(dim, order, shape, psi):
    """tau_A != tau_B: the brute-force stepper finds the common velocity as the
    one for which the collision changes the total momentum by exactly
    F_A + F_B (solving that linear condition, not using a formula)."""
    rng = np.random.default_rng(24)
    g = ((-0.2, 1.8), (1.8, 0.0)) if psi == O.PSI_N else ((-0.9, 1.2), (1.2, -0.5))
    tau = (0.7, 1.45)
    nA = rng.uniform(0.2, 1.0, shape)
    nB = rng.uniform(0.2, 1.0, shape)
    o = O.Oracle(dim, order, shape, tau=tau, g=g, psi_self=psi)
    o.set_density(nA, nB)
    nv = Naive(dim, order, shape, tau, g, psi)
    nv.set_density(nA, nB)
    steps = 5 if dim == 3 else 10
    o.run(steps)
    for _ in range(steps):
        nv.step()
    fn = nv.populations()[:, _vel_map(dim, nv)]
    assert np.abs(o.f - fn.reshape(o.f.shape)).max() < 1e-13


@pytest.mark.parametrize("dim,order", [(2, 8), (3, 6)])
def test_unequal_tau_conserves_momentum(dim, order):
    """With tau_A != tau_B the weighted common velocity keeps the total
    momentum (the forces sum to zero on the periodic lattice) and each
    component's mass; the unweighted velocity of Sec. 2 would not."""
    rng = np.random.default_rng(25)
    L = 24 if dim == 2 else 12
    shape = (L, L) if dim == 2 else (L, L, L)
    o = O.Oracle(dim, order, shape, tau=(0.65, 1.6), g=((-0.05, 1.4), (1.4, 0.05)))
    nA, nB = inputs.droplet(L, L, None if dim == 2 else L, R=L / 4)
    o.set_density(nA + 2e-3 * rng.uniform(-1, 1, shape), nB)
    s0 = o.stats()
    o.run(300 if dim == 2 else 60)
    s1 = o.stats()
    np.testing.assert_allclose(s1["mass"], s0["mass"], rtol=1e-13)
    assert np.abs(s1["momentum"]).max() < 1e-11 * s0["mass"].sum()
    assert s1["max_u"] > 1e-5


def test_shear_wave_of_one_component_with_unequal_tau():
    """Only component A present (n_B = 0): the weighted velocity is A's own,
    and a shear wave decays with A's viscosity c_s^2 (tau_A - 1/2) whatever
    tau_B is."""
    L, tauA = 64, 0.8
    o = O.Oracle(2, 4, (L, 4), tau=(tauA, 1.7), g=((0.0, 0.0), (0.0, 0.0)))
    k, U = 2 * np.pi / L, 1e-4
    f = np.zeros((2, 9, 1, L, 4))
    for iy in range(L):
        f[0, :, 0, iy, :] = O.equilibrium(2, 0.7, np.array([U * np.sin(k * iy), 0.0, 0.0]))[:, None]
    o.set_populations(f)

    def amp():
        u = o.velocity()[0, 0, :, 0]
        return 2.0 / L * np.sum(u * np.sin(k * np.arange(L)))
    a0 = amp()
    o.run(400)
    nu = -np.log(amp() / a0) / (k * k * 400)
    assert abs(nu / ((tauA - 0.5) / 3.0) - 1.0) < 2e-3

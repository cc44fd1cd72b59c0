"""Physics pins of the oracle.

* transverse-uniform 2D / 3D runs equal the exact D1Q3 reduction;
* the A<->B-symmetric slab keeps its symmetry (swap A and B, shift by L/2);
* with the fourth-order stencil and tau = 1 the normal pressure P_N = P^xx of a
  converged flat interface is constant to machine precision (Sec. 2, after
  eq. sm:pt);
* for uniform fields the lattice tensor is isotropic and equals the bulk
  pressure of eq. bulkp (e2 = 1);
* with psi = exp(-1/n) the single-component critical coupling is
  G_c c_s^2 = -e^2/3 = -2.463 (Sec. 2, after eq. self_p): dP/dn and
  d^2P/dn^2 vanish at n = 1;
* Laplace law: droplet pressure jumps scale as sigma / R_s and sigma_s tends
  to the flat sigma_0 (Sec. 3, Sec. 4).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2112_02574_amd import inputs
from tests.d1q3 import D1Q3


@pytest.mark.parametrize("dim,order", [(2, 4), (2, 6), (2, 8), (3, 4), (3, 6)])
@pytest.mark.parametrize("psi", [O.PSI_N, O.PSI_EXP])
def test_flat_runs_equal_d1q3(dim, order, psi):
    nx = 48
    g = ((0.0, 1.8), (1.8, 0.0)) if psi == O.PSI_N else ((-1.0, 0.5), (0.5, -0.6))
    tau = 1.0 if psi == O.PSI_N else 0.9
    shape = (3, nx) if dim == 2 else (2, 3, nx)
    o = O.Oracle(dim, order, shape, tau=tau, g=g, psi_self=psi)
    x = np.arange(nx)
    nA1 = np.where((x >= 12) & (x < 36), 1.0, 0.04) + 0.01 * np.sin(2 * np.pi * x / nx)
    nB1 = np.where((x >= 12) & (x < 36), 0.04, 1.0)
    if psi == O.PSI_EXP:
        nA1, nB1 = 0.6 + 0.3 * np.sin(2 * np.pi * x / nx), 0.7 - 0.2 * np.cos(2 * np.pi * x / nx)
    o.set_density(np.broadcast_to(nA1, shape), np.broadcast_to(nB1, shape))
    ref = D1Q3(order, nx, tau, g, psi)
    ref.set_density(nA1, nB1)
    o.run(300)
    for _ in range(300):
        ref.step()
    n = o.density()
    nref = ref.density()
    for J in range(2):
        assert np.isfinite(n[J]).all()
        assert np.abs(n[J] - nref[J]).max() < 1e-12
        assert np.abs(n[J] - n[J].reshape(-1, nx)[0]).max() < 1e-14  # stays transverse-uniform
    u = o.velocity()
    assert np.abs(u[1:]).max() < 1e-15


def test_symmetric_slab_keeps_swap_symmetry():
    L = 64
    o = O.Oracle(2, 4, (L, L), tau=1.0, g=((0.0, 1.8), (1.8, 0.0)))
    nA, nB = inputs.slab(L, L, x0=16, x1=48)
    # the 2D field is uniform along y; add a y-dependent but swap-symmetric
    # perturbation so the test is not one-dimensional
    y = np.arange(L)[:, None]
    pert = 1e-3 * np.sin(2 * np.pi * y / L) * np.cos(2 * np.pi * np.arange(L)[None, :] / L)
    nA = nA + pert
    nB = nB + np.roll(pert, -L // 2, axis=1)
    o.set_density(nA, nB)
    o.run(500)
    n = o.density()[:, 0]
    swapped = np.roll(n[1], L // 2, axis=1)
    assert np.abs(n[0] - swapped).max() < 1e-12
    assert np.abs(n[0] - n[0][:, ::-1]).max() > 1e-6  # not trivially uniform


def test_flat_normal_pressure_is_machine_constant():
    """E4, tau = 1: P_N(x) spread of a converged transverse-uniform slab."""
    L = 64
    o = O.Oracle(2, 4, (2, L), tau=1.0, g=((0.0, 1.8), (1.8, 0.0)))
    nA, nB = inputs.slab(L, 2, x0=16, x1=48)
    o.set_density(nA, nB)
    o.run(60000)
    s0, PN, PT = o.flat_sigma0()
    assert PN.max() - PN.min() < 1e-13 * abs(PN).max() * 10
    assert o.stats()["max_u"] < 1e-14
    # the tangential component is not constant: there is a surface tension
    assert s0 > 0.1 and (PT.max() - PT.min()) > 1e-2


@pytest.mark.parametrize("dim,order", [(2, 4), (2, 8), (3, 4), (3, 6)])
def test_uniform_tensor_is_bulk_pressure(dim, order):
    shape = (5, 6) if dim == 2 else (5, 5, 6)
    for psi, g in ((O.PSI_N, ((-0.2, 1.8), (1.8, 0.3))), (O.PSI_EXP, ((-2.0, 0.5), (0.5, -1.1)))):
        o = O.Oracle(dim, order, shape, g=g, psi_self=psi)
        n = np.empty((2,) + o.shape)
        n[0], n[1] = 0.83, 0.27
        P = o.pressure_tensor_site(n, 7)
        want = o.bulk_pressure(0.83, 0.27)
        assert abs(P[0] - want) < 1e-15 and abs(P[1] - want) < 1e-15
        if dim == 3:
            assert abs(P[2] - want) < 1e-15
        assert np.abs(P[3:]).max() < 1e-16
        # independent evaluation of eq. bulkp
        ps = (lambda v: v) if psi == O.PSI_N else (lambda v: np.exp(-1.0 / v))
        manual = (0.83 + 0.27) / 3 + g[0][1] * 0.83 * 0.27 + 0.5 * g[0][0] * ps(0.83) ** 2 + 0.5 * g[1][1] * ps(0.27) ** 2
        assert abs(want - manual) < 1e-15


def test_critical_coupling_of_exp_pseudopotential():
    gc = -np.exp(2.0) / 3.0
    assert abs(gc - (-2.463)) < 5e-4  # the value printed after eq. self_p
    o = O.Oracle(3, 4, (3, 3, 3), g=((gc, 0.0), (0.0, 0.0)), psi_self=O.PSI_EXP)
    P = lambda n: o.bulk_pressure(n, 0.0) - 0.0
    h = 1e-3
    d1 = (P(1 + h) - P(1 - h)) / (2 * h)
    d2 = (P(1 + h) - 2 * P(1) + P(1 - h)) / h ** 2
    assert abs(d1) < 1e-6 and abs(d2) < 1e-5
    # slightly weaker coupling is stable (dP/dn > 0 everywhere)
    o2 = O.Oracle(3, 4, (3, 3, 3), g=((0.9 * gc, 0.0), (0.0, 0.0)), psi_self=O.PSI_EXP)
    ns = np.linspace(0.2, 3.0, 200)
    Ps = np.array([o2.bulk_pressure(v, 0.0) for v in ns])
    assert np.all(np.diff(Ps) > 0)


@pytest.mark.parametrize("dim,order,gaa,guess", [
    (2, 4, 0.0, (1.0, 0.04, 0.04, 1.0)),
    (2, 8, 0.0, (1.0, 0.04, 0.04, 1.0)),
    (2, 4, -0.2, (1.0, 0.001, 0.001, 0.70)),
])
def test_flat_equilibrium_bulks_balance_pressure(dim, order, gaa, guess):
    """Stage one of the Sec. 4 initialisation.  At a flat steady state the
    pair forces cancel inside any slab of nodes, so the momentum balance
    leaves equal bulk pressures (eq. of the bulk pressure) on both sides of
    the interface, for every stencil; with symmetric couplings the two
    phases are mirror images (n_A in one = n_B in the other).  The asymmetric
    guess starts near pressure balance (n_A/3 - 0.1 n_A^2 = n_B/3): a guess far
    from it drives the attractive A phase towards its spinodal, where the
    strip splits and its centre is no longer a bulk phase (which this pin
    then flags)."""
    g = ((gaa, 1.8), (1.8, 0.0))
    bulk, steps = O.flat_equilibrium(dim, order, g, lx=64, guess=guess, tol=1e-13)
    assert steps < 200000
    o = O.Oracle(dim, order, (5, 64), g=g)
    p_in = o.bulk_pressure(bulk[0], bulk[1])
    p_out = o.bulk_pressure(bulk[2], bulk[3])
    assert abs(p_in - p_out) < 1e-8 * abs(p_in)
    # a genuine two-phase state, not the mixed one
    assert bulk[0] - bulk[2] > 0.5 and bulk[3] - bulk[1] > 0.5
    if gaa == 0.0:
        assert abs(bulk[0] - bulk[3]) < 1e-12 and abs(bulk[1] - bulk[2]) < 1e-12


def test_flat_equilibrium_negative_control():
    """An asymmetric state far from steady does not balance: guards the
    pressure-balance pin against a trivially passing check (a symmetric
    state balances by symmetry alone at any time)."""
    g = ((-0.2, 1.8), (1.8, 0.0))
    bulk, _ = O.flat_equilibrium(2, 4, g, lx=64, guess=(1.0, 0.001, 0.001, 0.70),
                                 tol=0.0, max_steps=256, chunk=128)
    o = O.Oracle(2, 4, (5, 64), g=g)
    p_in = o.bulk_pressure(bulk[0], bulk[1])
    p_out = o.bulk_pressure(bulk[2], bulk[3])
    assert abs(p_in - p_out) > 1e-6

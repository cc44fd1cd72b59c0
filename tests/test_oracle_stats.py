"""Pins of the oracle's global statistics (``Oracle.stats``): the minimum
concentration of each component, the largest speed |u| of the common
velocity (Sec. 2, Guo prescription), the count of non-finite populations and
the total momentum.

Each expected value is fixed by construction, independently of the oracle:
  * populations are built as equilibria f_i = w_i n (1 + 3 xi.u + 9/2 (xi.u)^2
    - 3/2 u.u) from the brute-force stepper's own velocity set, whose first
    moment is exactly n u;
  * minima and the fastest site are planted at known nodes, on different
    components and axes, so that a minimum over the wrong component or a
    maximum over one axis only gives a different number;
  * with couplings the rest state moves at u = (F_A + F_B) / (2 (n_A + n_B)),
    and F is summed here over the brute-force stepper's stencil.
The momentum statistic adds sum_x F_J / 2, which vanishes on any periodic
box (the force is pairwise antisymmetric), so only its population part can
be observed; it is pinned against sum_x n u.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.naive_lbm import stencil as naive_stencil
from tests.naive_lbm import velocities as naive_velocities


def _equilibrium_state(o, n, u):
    """(2, Q, *box) equilibria of the oracle's velocity order for the fields
    n[2, *box] and the common velocity u[3, *box]."""
    vel = dict(naive_velocities(o.dim))
    xi_o, _ = O.lattice(o.dim)
    f = np.zeros((2, o.q) + o.shape)
    uu = (u * u).sum(axis=0)
    for i, v in enumerate(xi_o):
        w = vel[tuple(int(c) for c in v)]
        xu = sum(v[c] * u[c] for c in range(3))
        for J in range(2):
            f[J, i] = w * n[J] * (1.0 + 3.0 * xu + 4.5 * xu * xu - 1.5 * uu)
    return f


def _box(dim):
    return (1, 9, 12) if dim == 2 else (6, 7, 9)


@pytest.mark.parametrize("dim", [2, 3])
def test_min_n_is_the_planted_minimum_of_each_component(dim):
    rng = np.random.default_rng(41)
    o = O.Oracle(dim, 4, _box(dim)[-dim:] if dim == 2 else _box(dim),
                 g=((0.0, 0.0), (0.0, 0.0)))
    n = rng.uniform(0.2, 0.9, (2,) + o.shape)
    sa = (0, 3, 5)
    sb = (o.shape[0] - 1, 1, 8)
    n[0][sa] = -0.0137     # a negative minority value, as at interfaces
    n[1][sb] = 0.0031
    o.set_populations(_equilibrium_state(o, n, np.zeros((3,) + o.shape)))
    st = o.stats()
    assert st["min_n"][0] == pytest.approx(-0.0137, abs=1e-15)
    assert st["min_n"][1] == pytest.approx(0.0031, abs=1e-15)
    assert st["n_nonfinite"] == 0


@pytest.mark.parametrize("dim", [2, 3])
def test_max_u_without_force_is_the_fastest_planted_site(dim):
    """G = 0: u is the barycentric velocity of the equilibria.  Everywhere
    |u_x| <= 0.01, and one site moves along the last axis at 0.03."""
    rng = np.random.default_rng(42)
    o = O.Oracle(dim, 4, _box(dim)[-dim:] if dim == 2 else _box(dim),
                 g=((0.0, 0.0), (0.0, 0.0)))
    n = rng.uniform(0.3, 1.0, (2,) + o.shape)
    u = np.zeros((3,) + o.shape)
    u[0] = rng.uniform(-0.01, 0.01, o.shape)
    u[1] = rng.uniform(-0.004, 0.004, o.shape)
    if dim == 3:
        u[2] = rng.uniform(-0.004, 0.004, o.shape)
    site = (0, 4, 2)
    u[(slice(None),) + site] = 0.0
    u[(dim - 1,) + site] = -0.03
    o.set_populations(_equilibrium_state(o, n, u))
    st = o.stats()
    assert st["max_u"] == pytest.approx(0.03, rel=1e-13)
    # the total momentum: sum_x (n_A + n_B) u (the force part is zero here)
    want = [(n.sum(axis=0) * u[c]).sum() for c in range(3)]
    assert np.abs(st["momentum"] - want).max() < 1e-13


@pytest.mark.parametrize("dim,order", [(2, 8), (3, 6)])
def test_max_u_at_rest_is_the_force_velocity(dim, order):
    """With couplings, populations at rest (f = w n) have a common velocity
    (F_A + F_B) / (2 (n_A + n_B)) (Sec. 2): the force enters with half its
    weight.  F is summed here over the brute-force stencil."""
    rng = np.random.default_rng(43)
    g = ((-0.3, 1.6), (1.6, 0.2))
    shape = (10, 11) if dim == 2 else (6, 7, 8)
    o = O.Oracle(dim, order, shape, g=g)
    n = rng.uniform(0.2, 1.0, (2,) + o.shape)
    o.set_populations(_equilibrium_state(o, n, np.zeros((3,) + o.shape)))
    F = np.zeros((2, 3) + o.shape)
    for e, W in naive_stencil(dim, order):
        sh = tuple(-e[2 - k] for k in range(3))   # n(x + e) on the (z, y, x) grid
        nb = [np.roll(n[K], sh, axis=(0, 1, 2)) for K in range(2)]
        for J in range(2):
            K = 1 - J
            for c in range(3):
                F[J, c] -= W * e[c] * (g[J][K] * n[J] * nb[K] + g[J][J] * n[J] * nb[J])
    u = (F[0] + F[1]) / (2.0 * n.sum(axis=0))
    speed = np.sqrt((u * u).sum(axis=0))
    st = o.stats()
    assert speed.max() > 1e-3
    assert st["max_u"] == pytest.approx(speed.max(), rel=1e-12)
    assert np.abs(st["momentum"]).max() < 1e-12


def test_nonfinite_populations_are_counted():
    rng = np.random.default_rng(44)
    o = O.Oracle(3, 4, (5, 6, 7), g=((0.0, 1.2), (1.2, 0.0)))
    n = rng.uniform(0.3, 0.9, (2,) + o.shape)
    f = _equilibrium_state(o, n, np.zeros((3,) + o.shape))
    o.set_populations(f)
    assert o.stats()["n_nonfinite"] == 0
    f1 = f.copy()
    f1[1, 7, 2, 3, 4] = np.nan
    o.set_populations(f1)
    assert o.stats()["n_nonfinite"] == 1
    f1[0, 0, 0, 0, 0] = np.inf
    f1[0, 18, 4, 5, 6] = -np.inf
    o.set_populations(f1)
    assert o.stats()["n_nonfinite"] == 3

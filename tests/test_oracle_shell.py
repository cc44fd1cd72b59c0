"""Pins of the oracle's shell-averaged pressure profiles (a variant of the
axis line of Sec. 3, not the paper's definition).

* a uniform state: the lattice tensor is isotropic, so every shell's normal
  and tangential pressures equal the bulk pressure of eq. bulkp and C_d = 0;
* a brute-force numpy evaluation on small boxes, written here from eq. sm:pt
  with the paper's fourth-order weights (3D: W(1) = 1/6, W(2) = 1/12; 2D:
  W(1) = 1/3, W(2) = 1/12): the tensor at every node, its projection on the
  radial unit vector and the shell means;
* exchanging the x and y axes of a cubic box maps every shell onto itself
  and the tensor onto its transpose, so the shell profiles do not change (a
  wrong component or index in the projection breaks this);
* the droplet analysis on the shell profile matches the closed form of
  eq. gen_sigma on a profile integrated here.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2112_02574_amd import inputs

CS2 = 1.0 / 3.0


def _e4_stencil(dim):
    """Vectors and weights of the fourth-order force stencil."""
    w = {1: 1.0 / 6, 2: 1.0 / 12} if dim == 3 else {1: 1.0 / 3, 2: 1.0 / 12}
    rng = range(-1, 2)
    out = []
    for ez in (rng if dim == 3 else [0]):
        for ey in rng:
            for ex in rng:
                s = ex * ex + ey * ey + ez * ez
                if s in w:
                    out.append(((ex, ey, ez), w[s]))
    return out


def _psi(n, psi_self):
    return n if psi_self == O.PSI_N else np.exp(-1.0 / n)


def _brute_force_shells(nA, nB, dim, g, psi_self):
    """Shell means of u.P.u and (tr P - u.P.u)/(d-1) from eq. sm:pt."""
    shape = nA.shape  # (nz, ny, nx) or (ny, nx)
    axes = {0: dim - 1, 1: dim - 2, 2: 0}  # x, y, z -> array axis
    pA, pB = _psi(nA, psi_self), _psi(nB, psi_self)

    def at(f, e):  # f(x + e) on the periodic box
        shift = tuple(-e[c] for c in range(dim))
        return np.roll(f, shift, axis=tuple(axes[c] for c in range(dim)))

    P = np.zeros((3, 3) + shape)
    for e, W in _e4_stencil(dim):
        inter = (g[0][1] * nA * at(nB, e) + g[1][0] * nB * at(nA, e)
                 + g[0][0] * pA * at(pA, e) + g[1][1] * pB * at(pB, e))
        for m in range(3):
            for n in range(3):
                if e[m] and e[n]:
                    P[m, n] += 0.5 * W * e[m] * e[n] * inter
    for m in range(dim):
        P[m, m] += CS2 * (nA + nB)
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    # distance vector from the centre node, components x, y, z
    v = [grids[axes[c]] - shape[axes[c]] // 2 for c in range(dim)]
    v += [np.zeros(shape)] * (3 - dim)
    r2 = sum(c * c for c in v).astype(float)
    tr = sum(P[c, c] for c in range(dim))
    with np.errstate(invalid="ignore", divide="ignore"):
        pn = sum(v[m] * v[n] * P[m, n] for m in range(3) for n in range(3)) / r2
    pn = np.where(r2 == 0, tr / dim, pn)
    pt = (tr - pn) / (dim - 1)
    k = np.floor(np.sqrt(r2) + 0.5).astype(int)
    rmax = min(shape) // 2
    keep = k <= rmax
    cnt = np.bincount(k[keep], minlength=rmax + 1)
    PN = np.bincount(k[keep], weights=pn[keep], minlength=rmax + 1) / cnt
    PT = np.bincount(k[keep], weights=pt[keep], minlength=rmax + 1) / cnt
    return PN, PT


def test_uniform_state_shells_equal_bulk_pressure():
    g = ((-0.2, 1.8), (1.8, 0.0))
    o = O.Oracle(3, 6, (12, 14, 16), g=g)
    nA, nB = 0.7, 0.3
    o.set_density(np.full(o.shape, nA), np.full(o.shape, nB))
    d = o.shell_observables(4.0)
    bulk = (nA + nB) * CS2 + g[0][1] * nA * nB + 0.5 * g[0][0] * nA * nA
    assert len(d["PT"]) == 12 // 2 + 1
    assert np.max(np.abs(d["PN"] - bulk)) < 1e-14
    assert np.max(np.abs(d["PT"] - bulk)) < 1e-14
    assert abs(d["C_d"]) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("psi_self", [O.PSI_N, O.PSI_EXP])
def test_shells_match_brute_force(dim, psi_self):
    """An off-centre, anisotropic droplet plus noise, so every tensor
    component and every shell carries a different value."""
    rng = np.random.default_rng(7)
    shape = (11, 14) if dim == 2 else (10, 11, 12)
    g = ((-0.2, 1.8), (1.8, 0.1)) if psi_self == O.PSI_N else ((-1.0, 0.5), (0.5, -0.6))
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    r = np.sqrt(sum((1.0 + 0.2 * a) * (gr - s / 2 + 0.7) ** 2
                    for a, (gr, s) in enumerate(zip(grids, shape))))
    nA = 0.55 - 0.45 * np.tanh(r - 3.0) + 0.02 * rng.random(shape)
    nB = 0.55 + 0.45 * np.tanh(r - 3.0) + 0.02 * rng.random(shape)
    o = O.Oracle(dim, 4, shape, g=g, psi_self=psi_self)
    o.set_density(nA, nB)
    d = o.shell_observables(3.0)
    n = o.density()  # the concentrations the oracle holds (sums of its populations)
    PN, PT = _brute_force_shells(n[0].reshape(shape), n[1].reshape(shape), dim, g, psi_self)
    assert np.max(np.abs(d["PN"] - PN)) < 1e-12
    assert np.max(np.abs(d["PT"] - PT)) < 1e-12


def test_shells_invariant_under_axis_exchange():
    rng = np.random.default_rng(3)
    L = 12
    shape = (L, L, L)
    nA = 0.5 + 0.3 * rng.random(shape)
    nB = 0.5 + 0.3 * rng.random(shape)
    g = ((-0.2, 1.8), (1.8, 0.0))
    o1 = O.Oracle(3, 6, shape, g=g)
    o1.set_density(nA, nB)
    o2 = O.Oracle(3, 6, shape, g=g)
    o2.set_density(nA.transpose(0, 2, 1), nB.transpose(0, 2, 1))  # x <-> y
    d1, d2 = o1.shell_observables(3.0), o2.shell_observables(3.0)
    assert np.max(np.abs(d1["PN"] - d2["PN"])) < 1e-13
    assert np.max(np.abs(d1["PT"] - d2["PT"])) < 1e-13
    # the axis line is not invariant: P^yy on the x axis becomes P^xx on y
    l1, l2 = o1.droplet_observables(3.0), o2.droplet_observables(3.0)
    assert np.max(np.abs(l1["PT"] - l2["PT"])) > 1e-3


def test_shell_droplet_analysis_closed_form():
    """C_d of the shell profile integrated here with the trapezoid-exact
    weights of a piecewise-linear interpolant, and R_s, sigma_s from
    eq. gen_sigma's minimum (Laplace law)."""
    L = 24
    o = O.Oracle(3, 6, (L, L, L), g=((0.0, 1.8), (1.8, 0.0)))
    nA, nB = inputs.droplet(L, L, L, R=6.0)
    o.set_density(nA, nB)
    o.run(300)  # past the initial pressure transient: dP > 0, C_d > 0
    d = o.shell_observables(6.0)
    assert d["dP"] > 0 and d["C_d"] > 0
    x = np.linspace(0.0, L // 2, 200001)
    pt = np.interp(x, np.arange(L // 2 + 1), d["PT"])
    f = x ** 2 * (d["P_out"] - pt)
    Cd = np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(x))
    assert abs(Cd - d["C_d"]) < 1e-6 * max(1.0, abs(Cd))
    Rs = (6.0 * d["C_d"] / d["dP"]) ** (1.0 / 3.0)
    assert abs(Rs - d["R_s"]) < 1e-12 * Rs
    assert abs(d["sigma_s"] - d["dP"] * Rs / 2.0) < 1e-12
    assert abs(d["R_s_grid"] - d["R_s"]) < 2e-3

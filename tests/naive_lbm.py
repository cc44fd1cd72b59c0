"""Brute-force two-component Shan-Chen stepper for tiny periodic lattices.

An independent, deliberately naive restatement of Sec. 2 of the paper, used
only to pin the oracle on 8^2 / 6^3 lattices.  It shares nothing with the
oracle: the velocity set is enumerated from the integer cube and weighted by
speed, the force stencil is enumerated from its shells, the equilibrium and the
Guo term are written as Hermite tensor contractions, and streaming is a pull
from dictionaries keyed by lattice coordinates.
"""
import itertools
from fractions import Fraction

import numpy as np

CS2 = 1.0 / 3.0

# lattice weights by squared speed (D2Q9 and D3Q19, c_s^2 = 1/3)
_W_LATTICE = {2: {0: Fraction(4, 9), 1: Fraction(1, 9), 2: Fraction(1, 36)},
              3: {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}}

# force-stencil weights by squared length (isotropy order 4, 6, 8)
_W_STENCIL = {
    (2, 4): {1: Fraction(1, 3), 2: Fraction(1, 12)},
    (2, 6): {1: Fraction(4, 15), 2: Fraction(1, 10), 4: Fraction(1, 120)},
    (2, 8): {1: Fraction(4, 21), 2: Fraction(4, 45), 4: Fraction(1, 60),
             5: Fraction(2, 315), 8: Fraction(1, 5040)},
    (3, 4): {1: Fraction(1, 6), 2: Fraction(1, 12)},
    (3, 6): {1: Fraction(2, 15), 2: Fraction(1, 15), 3: Fraction(1, 60),
             4: Fraction(1, 120)},
}


def velocities(dim):
    out = []
    for v in itertools.product((-1, 0, 1), repeat=dim):
        s = sum(c * c for c in v)
        if s <= 2:
            out.append((tuple(v) + (0,) * (3 - dim), float(_W_LATTICE[dim][s])))
    return out


def stencil(dim, order):
    table = _W_STENCIL[(dim, order)]
    out = []
    for v in itertools.product(range(-2, 3), repeat=dim):
        s = sum(c * c for c in v)
        if s in table:
            out.append((tuple(v) + (0,) * (3 - dim), float(table[s])))
    return out


def _psi(n, kind):
    return n if kind == 0 else np.exp(-1.0 / n)


class Naive:
    """state[J][(x, y, z)] -> dict {velocity: population} (pre-collision)."""

    def __init__(self, dim, order, shape, tau, g, psi_self=0):
        self.dim = dim
        self.vel = velocities(dim)
        self.sten = stencil(dim, order)
        nz, ny, nx = shape if dim == 3 else (1,) + tuple(shape)
        self.size = (nx, ny, nz)
        self.taus = (tau, tau) if np.isscalar(tau) else tuple(tau)
        self.g = g
        self.psi_self = psi_self
        self.nodes = [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
        self.f = [dict(), dict()]

    def _wrap(self, p):
        return tuple(p[a] % self.size[a] for a in range(3))

    def set_density(self, nA, nB):
        for J, nf in enumerate((nA, nB)):
            for (x, y, z) in self.nodes:
                val = nf[z, y, x] if nf.ndim == 3 else nf[y, x]
                self.f[J][(x, y, z)] = {v: w * val for v, w in self.vel}

    def density(self, J, node):
        return sum(self.f[J][node].values())

    def step(self):
        n = [{p: self.density(J, p) for p in self.nodes} for J in range(2)]
        post = [dict(), dict()]
        for p in self.nodes:
            F = []
            for J in range(2):
                K = 1 - J
                acc = np.zeros(3)
                for e, W in self.sten:
                    q = self._wrap((p[0] + e[0], p[1] + e[1], p[2] + e[2]))
                    acc -= self.g[J][K] * n[J][p] * W * n[K][q] * np.array(e, float)
                    acc -= (self.g[J][J] * _psi(n[J][p], self.psi_self) * W *
                            _psi(n[J][q], self.psi_self) * np.array(e, float))
                F.append(acc)
            def collide(u):
                res = []
                for J in range(2):
                    tau = self.taus[J]
                    out = {}
                    for v, w in self.vel:
                        xi = np.array(v, float)
                        H2 = np.outer(xi, xi) - CS2 * np.eye(3)
                        feq = n[J][p] * w * (1.0 + xi @ u / CS2 + np.sum(H2 * np.outer(u, u)) / (2 * CS2 ** 2))
                        S = w * (xi @ F[J] / CS2 + np.sum(H2 * np.outer(u, F[J])) / CS2 ** 2)
                        fv = self.f[J][p][v]
                        out[v] = fv + (-(fv - feq) / tau) + (1.0 - 1.0 / (2 * tau)) * S
                    res.append(out)
                return res

            if self.taus[0] == self.taus[1]:
                mom = np.zeros(3)
                for J in range(2):
                    for v, fv in self.f[J][p].items():
                        mom += fv * np.array(v, float)
                    mom += 0.5 * F[J]
                u = mom / (n[0][p] + n[1][p])
            else:
                # the velocity for which the collision changes the total
                # momentum by exactly F_A + F_B: the change is affine in u, so
                # probe it at u = 0 and the unit vectors and solve
                def excess(u):
                    out = collide(u)
                    d = -(F[0] + F[1])
                    for J in range(2):
                        for v, fv in out[J].items():
                            d = d + (fv - self.f[J][p][v]) * np.array(v, float)
                    return d
                d0 = excess(np.zeros(3))
                A = np.stack([excess(np.eye(3)[k]) - d0 for k in range(3)], axis=1)
                if self.dim == 2:
                    u = np.zeros(3)
                    u[:2] = np.linalg.solve(A[:2, :2], -d0[:2])
                else:
                    u = np.linalg.solve(A, -d0)
            post_p = collide(u)
            for J in range(2):
                post[J][p] = post_p[J]
        new = [dict(), dict()]
        for J in range(2):
            for p in self.nodes:
                new[J][p] = {}
                for v, _ in self.vel:
                    src = self._wrap((p[0] - v[0], p[1] - v[1], p[2] - v[2]))
                    new[J][p][v] = post[J][src][v]
        self.f = new

    def populations(self):
        """Array (2, Q, nz, ny, nx) in the order of self.vel."""
        nx, ny, nz = self.size
        out = np.zeros((2, len(self.vel), nz, ny, nx))
        for J in range(2):
            for k, (v, _) in enumerate(self.vel):
                for (x, y, z) in self.nodes:
                    out[J, k, z, y, x] = self.f[J][(x, y, z)][v]
        return out

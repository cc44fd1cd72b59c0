"""Exact one-dimensional reduction of the two-component Shan-Chen model.

For fields that are uniform across y (and z) and carry no transverse
momentum, summing D2Q9 / D3Q19 over the transverse velocity components gives
a D1Q3 lattice with weights 2/3, 1/6, 1/6 and c_s^2 = 1/3, and summing the
force stencil over its transverse offsets gives per-side weights: E4 {1: 1/2},
E6 {1: 7/15, 2: 1/120}, E8 {1: 8/21, 2: 5/168}.  This is an independent
second implementation (numpy, pull streaming via np.roll) used to pin the
oracle on flat-interface runs.
"""
import numpy as np

XI = np.array([0.0, 1.0, -1.0])
W = np.array([2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0])
SIDE = {4: {1: 0.5}, 6: {1: 7.0 / 15.0, 2: 1.0 / 120.0},
        8: {1: 8.0 / 21.0, 2: 5.0 / 168.0}}


class D1Q3:
    def __init__(self, order, nx, tau, g, psi_self=0):
        self.side = SIDE[order]
        self.nx = nx
        self.tau = tau
        self.g = np.array(g, dtype=float)
        self.psi_self = psi_self
        self.f = np.zeros((2, 3, nx))

    def psi(self, n):
        return n if self.psi_self == 0 else np.exp(-1.0 / n)

    def set_density(self, nA, nB):
        self.f[0] = W[:, None] * nA[None, :]
        self.f[1] = W[:, None] * nB[None, :]

    def density(self):
        return self.f.sum(axis=1)

    def grad_sum(self, phi):
        """sum over the 1D stencil of W_d phi(x + d) d"""
        out = np.zeros_like(phi)
        for d, w in self.side.items():
            out += w * d * (np.roll(phi, -d) - np.roll(phi, d))
        return out

    def force(self, n):
        F = np.zeros((2, self.nx))
        for J in range(2):
            K = 1 - J
            F[J] = (-self.g[J, K] * n[J] * self.grad_sum(n[K])
                    - self.g[J, J] * self.psi(n[J]) * self.grad_sum(self.psi(n[J])))
        return F

    def step(self):
        n = self.density()
        F = self.force(n)
        u = ((self.f * XI[None, :, None]).sum(axis=(0, 1)) + 0.5 * F.sum(axis=0)) / n.sum(axis=0)
        for J in range(2):
            for i in range(3):
                c = XI[i]
                feq = W[i] * n[J] * (1 + 3 * c * u + 4.5 * c * c * u * u - 1.5 * u * u)
                S = W[i] * (3 * c * F[J] + 9 * c * u * c * F[J] - 3 * u * F[J])
                post = self.f[J, i] - (self.f[J, i] - feq) / self.tau + (1 - 0.5 / self.tau) * S
                self.f[J, i] = np.roll(post, int(c))

"""Seeded synthetic initial conditions shared by the tests, the smoke check and
the benchmark.

This module holds no arithmetic of the lattice Boltzmann method itself: it
only builds the initial concentration fields n_A, n_B (float64 numpy arrays
shaped (nz, ny, nx), or (ny, nx) in 2D, x fastest) that both the oracle and
the GPU library receive unchanged.

Profiles:
  * ``slab``: sharp flat strip, n_A = n_hi inside x in [x0, x1), n_lo outside,
    n_B swapped, plus optional seeded uniform noise.
  * ``droplet``: the radial profile of Sec. 4,
    n_J(r) = (n_in + n_out)/2 - (n_in - n_out)/2 tanh(r - R), r measured from
    the centre node (floor(L/2) on every axis).
  * ``flat_strip``: the double-tanh strip of Sec. 4 with centre x0, width w.
  * ``batch_members``: the 48-droplet sweep (radii, box sizes, couplings).
"""
import math

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """splitmix64 (Steele, Lea, Flood 2014): state += 0x9E3779B97F4A7C15, then
    two xor-shift-multiply rounds.  ``uniform`` maps the top 53 bits to [0, 1)."""

    def __init__(self, seed):
        self.state = seed & MASK64

    def next(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self):
        return (self.next() >> 11) * (1.0 / (1 << 53))


def splitmix64_uniform_array(seed, count):
    """``count`` uniforms in [0, 1) from splitmix64(seed), vectorised."""
    i = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + i * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def _shape(nx, ny, nz):
    return (ny, nx) if nz is None else (nz, ny, nx)


def slab(nx, ny, nz=None, x0=16, x1=48, n_hi=1.0, n_lo=0.04, noise=0.0, seed=1):
    """Sharp strip along x; noise drawn per node per component, order J, z, y, x,
    noise = amplitude * (2u - 1) with u from splitmix64(seed)."""
    shp = _shape(nx, ny, nz)
    x = np.arange(nx)
    inside = (x >= x0) & (x < x1)
    nA = np.broadcast_to(np.where(inside, n_hi, n_lo), shp).astype(np.float64).copy()
    nB = np.broadcast_to(np.where(inside, n_lo, n_hi), shp).astype(np.float64).copy()
    if noise:
        cnt = nA.size
        u = splitmix64_uniform_array(seed, 2 * cnt)
        nA += noise * (2.0 * u[:cnt].reshape(shp) - 1.0)
        nB += noise * (2.0 * u[cnt:].reshape(shp) - 1.0)
    return nA, nB


def radius_field(nx, ny, nz=None):
    cx, cy = nx // 2, ny // 2
    if nz is None:
        y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        return np.sqrt((x - cx) ** 2.0 + (y - cy) ** 2.0)
    cz = nz // 2
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.sqrt((x - cx) ** 2.0 + (y - cy) ** 2.0 + (z - cz) ** 2.0)


def droplet(nx, ny, nz=None, R=None, n_in=1.0, n_out=0.04, a_rich=True, bulk=None):
    """tanh droplet of radius R (default L/4) centred on node floor(L/2).

    Either the rich component goes from n_in (inside) to n_out (outside) and
    the other the reverse, or ``bulk`` = (nA_in, nB_in, nA_out, nB_out) gives
    all four bulk values (e.g. those of a converged flat interface, with
    "in" the A-rich phase); ``a_rich`` then picks which phase is the droplet."""
    if R is None:
        R = nx / 4.0
    r = radius_field(nx, ny, nz)

    def prof(inside, outside):
        return 0.5 * (inside + outside) - 0.5 * (inside - outside) * np.tanh(r - R)

    if bulk is not None:
        a_in, b_in, a_out, b_out = bulk
        if not a_rich:
            a_in, b_in, a_out, b_out = a_out, b_out, a_in, b_in
        return prof(a_in, a_out), prof(b_in, b_out)
    rich = prof(n_in, n_out)
    poor = prof(n_out, n_in)
    return (rich, poor) if a_rich else (poor, rich)


def flat_strip(nx, ny, nz=None, x0=None, w=None, n_h=1.0, n_l=0.04, a_rich=True):
    """Double-tanh strip of Sec. 4 centred at x0 with width w (default nx/2)."""
    if x0 is None:
        x0 = nx / 2.0
    if w is None:
        w = nx / 2.0
    x = np.arange(nx, dtype=np.float64)

    def prof(nh, nl):
        return (0.5 * (nh + nl) - 0.5 * (nh - nl) * np.tanh(x - (x0 - w / 2.0))
                + 0.5 * (nh - nl) * (np.tanh(x - (x0 + w / 2.0)) + 1.0))

    shp = _shape(nx, ny, nz)
    # the profile is n_l inside the strip and n_h outside; the strip-rich
    # component is the one whose high value sits inside
    a = np.broadcast_to(prof(n_l, n_h) if a_rich else prof(n_h, n_l), shp).copy()
    b = np.broadcast_to(prof(n_h, n_l) if a_rich else prof(n_l, n_h), shp).copy()
    return a, b


def batch_members(count=48, seed=4):
    """The seeded droplet sweep: R0_i ~ U[8, 40]; L_i = clamp(8 ceil(4 R0_i / 8),
    48, 160) (aspect ratio L/R = 4 as in Sec. 4); g_AA = 0 for even i and -0.2
    for odd i, g_BB = 0, g_AB = 1.8.  Symmetric members alternate A-rich and
    B-rich droplets (A-rich when floor(i/2) is even); asymmetric members hold a
    B-rich droplet, because the attractive A phase sits close to its spinodal
    and an A-rich droplet of these sizes is driven over it by the Laplace
    pressure."""
    rng = SplitMix64(seed)
    out = []
    for i in range(count):
        R0 = 8.0 + 32.0 * rng.uniform()
        L = min(max(8 * math.ceil(4.0 * R0 / 8.0), 48), 160)
        sym = i % 2 == 0
        out.append({"index": i, "L": L, "R0": R0,
                    "g": ((0.0 if sym else -0.2, 1.8), (1.8, 0.0)),
                    "a_rich": sym and (i // 2) % 2 == 0})
    return out


# Starting guesses for the flat-interface stage, (nA_in, nB_in, nA_out, nB_out)
# with "in" the A-rich phase: close to pressure balance, n/3 + g_AA n^2 / 2 equal
# in both nearly pure phases.
FLAT_GUESS = {0.0: (1.0, 0.04, 0.04, 1.0), -0.2: (1.0, 0.001, 0.001, 0.70)}

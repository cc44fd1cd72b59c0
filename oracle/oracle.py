"""ctypes wrapper of the FP64 CPU oracle (``scmc_oracle.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module.  It never imports the GPU package
and the GPU package never imports it.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "scmc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

PSI_N = 0
PSI_EXP = 1


def build(force=True):
    """Compile the oracle with gcc (FP64, OpenMP over the site loops)."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("stencil", ctypes.c_int),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("tau", ctypes.c_double * 2), ("g", (ctypes.c_double * 2) * 2),
                ("psi_self", ctypes.c_int), ("nthreads", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(_Problem)
        L.orc_lattice.argtypes = [ctypes.c_int, dp, dp]
        L.orc_stencil.argtypes = [ctypes.c_int, ctypes.c_int, ip, dp]
        L.orc_check.argtypes = [pp]
        L.orc_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_guo_source.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_init_equilibrium.argtypes = [pp, dp, dp, dp]
        L.orc_density.argtypes = [pp, dp, dp]
        L.orc_pseudopotential.argtypes = [pp, dp, dp]
        L.orc_force.argtypes = [pp, dp, dp]
        L.orc_velocity.argtypes = [pp, dp, dp, dp, dp]
        L.orc_run.argtypes = [pp, dp, ctypes.c_long, dp]
        L.orc_work_doubles.argtypes = [pp]
        L.orc_work_doubles.restype = ctypes.c_long
        L.orc_collide_site.argtypes = [pp, dp, ctypes.c_long, dp]
        L.orc_pressure_tensor_site.argtypes = [pp, dp, ctypes.c_long, dp]
        L.orc_bulk_pressure.argtypes = [pp, ctypes.c_double, ctypes.c_double]
        L.orc_bulk_pressure.restype = ctypes.c_double
        L.orc_droplet_observables.argtypes = [pp, dp, ctypes.c_double, dp, dp, dp]
        L.orc_shell_observables.argtypes = [pp, dp, ctypes.c_double, dp, dp, dp]
        L.orc_flat_sigma0.argtypes = [pp, dp, dp, dp]
        L.orc_flat_sigma0.restype = ctypes.c_double
        L.orc_stats.argtypes = [pp, dp, dp]
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lattice(dim):
    xi = np.zeros(19 * 3)
    w = np.zeros(19)
    q = lib().orc_lattice(dim, _dp(xi), _dp(w))
    if q < 0:
        raise ValueError("bad dim")
    return xi[:3 * q].reshape(q, 3).astype(np.int64), w[:q].copy()


def stencil(dim, order):
    e = np.zeros(64 * 3, dtype=np.int32)
    W = np.zeros(64)
    n = lib().orc_stencil(dim, order, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(W))
    if n < 0:
        raise ValueError("unsupported stencil")
    return e[:3 * n].reshape(n, 3).astype(np.int64), W[:n].copy()


def equilibrium(dim, n, u):
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(3))
    out = np.zeros(19)
    lib().orc_equilibrium(dim, float(n), _dp(u), _dp(out))
    return out[:9 if dim == 2 else 19].copy()


def guo_source(dim, u, F):
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(3))
    F = np.ascontiguousarray(np.asarray(F, dtype=np.float64).reshape(3))
    out = np.zeros(19)
    lib().orc_guo_source(dim, _dp(u), _dp(F), _dp(out))
    return out[:9 if dim == 2 else 19].copy()


class Oracle:
    """One periodic two-component Shan-Chen problem on the CPU (FP64).

    Fields are numpy arrays shaped (nz, ny, nx) (x fastest); the population
    state has shape (2, Q, nz, ny, nx) and is the pre-collision state f(x, t).
    """

    def __init__(self, dim, stencil, shape, tau=1.0, g=((0.0, 1.8), (1.8, 0.0)),
                 psi_self=PSI_N, nthreads=0):
        if dim == 2:
            ny, nx = shape[-2], shape[-1]
            nz = 1
        else:
            nz, ny, nx = shape
        self.dim = dim
        self.q = 9 if dim == 2 else 19
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        p = _Problem()
        p.dim, p.stencil, p.nx, p.ny, p.nz = dim, stencil, nx, ny, nz
        taus = (tau, tau) if np.isscalar(tau) else tuple(tau)
        p.tau[0], p.tau[1] = float(taus[0]), float(taus[1])
        for J in range(2):
            for K in range(2):
                p.g[J][K] = float(g[J][K])
        p.psi_self = int(psi_self)
        p.nthreads = int(nthreads)
        if lib().orc_check(ctypes.byref(p)) != 0:
            raise ValueError("invalid oracle problem")
        self.p = p
        self.f = np.zeros((2, self.q) + self.shape)
        self._work = None
        self.t = 0

    # -- state ------------------------------------------------------------
    def set_density(self, nA, nB):
        nA = np.ascontiguousarray(np.asarray(nA, dtype=np.float64).reshape(self.shape))
        nB = np.ascontiguousarray(np.asarray(nB, dtype=np.float64).reshape(self.shape))
        self.f = np.zeros((2, self.q) + self.shape)
        lib().orc_init_equilibrium(ctypes.byref(self.p), _dp(nA), _dp(nB), _dp(self.f))
        self.t = 0

    def set_populations(self, f, t=0):
        self.f = np.ascontiguousarray(np.asarray(f, dtype=np.float64).reshape((2, self.q) + self.shape)).copy()
        self.t = t

    def run(self, nsteps):
        if self._work is None:
            self._work = np.zeros(lib().orc_work_doubles(ctypes.byref(self.p)))
        rc = lib().orc_run(ctypes.byref(self.p), _dp(self.f), int(nsteps), _dp(self._work))
        if rc != 0:
            raise RuntimeError("orc_run failed")
        self.t += nsteps

    # -- fields -----------------------------------------------------------
    def density(self):
        n = np.zeros((2,) + self.shape)
        lib().orc_density(ctypes.byref(self.p), _dp(self.f), _dp(n))
        return n

    def force(self, n=None):
        if n is None:
            n = self.density()
        n = np.ascontiguousarray(n)
        F = np.zeros((2, 3) + self.shape)
        lib().orc_force(ctypes.byref(self.p), _dp(n), _dp(F))
        return F

    def velocity(self):
        n = self.density()
        F = self.force(n)
        u = np.zeros((3,) + self.shape)
        lib().orc_velocity(ctypes.byref(self.p), _dp(self.f), _dp(n), _dp(F), _dp(u))
        return u

    def collide_site(self, site):
        out = np.zeros(2 * self.q)
        lib().orc_collide_site(ctypes.byref(self.p), _dp(self.f), int(site), _dp(out))
        return out.reshape(2, self.q)

    def pressure_tensor_site(self, n, site):
        n = np.ascontiguousarray(n)
        out = np.zeros(6)
        lib().orc_pressure_tensor_site(ctypes.byref(self.p), _dp(n), int(site), _dp(out))
        return out

    def bulk_pressure(self, nA, nB):
        return lib().orc_bulk_pressure(ctypes.byref(self.p), float(nA), float(nB))

    def droplet_observables(self, R0):
        obs = np.zeros(9)
        L = self.shape[2]
        PN = np.zeros(L // 2 + 1)
        PT = np.zeros(L // 2 + 1)
        rc = lib().orc_droplet_observables(ctypes.byref(self.p), _dp(self.f), float(R0),
                                           _dp(obs), _dp(PN), _dp(PT))
        if rc != 0:
            raise RuntimeError("orc_droplet_observables failed")
        keys = ["P_in", "P_out", "dP", "C_d", "R_s", "R_s_grid", "sigma_s",
                "sigma_grid_min", "max_PyyPzz"]
        d = dict(zip(keys, obs.tolist()))
        d["PN"] = PN
        d["PT"] = PT
        return d

    def shell_observables(self, R0):
        """The droplet analysis on shell-averaged profiles: PN[k], PT[k] are
        the means of the normal and tangential pressure over the shells
        k = floor(|x - c| + 1/2), k = 0..min(extent) // 2 (a variant of the
        axis line, not the paper's definition)."""
        dims = self.shape if self.dim == 3 else self.shape[-2:]
        rmax = min(dims) // 2
        obs = np.zeros(9)
        PN = np.zeros(rmax + 1)
        PT = np.zeros(rmax + 1)
        rc = lib().orc_shell_observables(ctypes.byref(self.p), _dp(self.f), float(R0),
                                         _dp(obs), _dp(PN), _dp(PT))
        if rc != 0:
            raise RuntimeError("orc_shell_observables failed")
        keys = ["P_in", "P_out", "dP", "C_d", "R_s", "R_s_grid", "sigma_s",
                "sigma_grid_min"]
        d = dict(zip(keys, obs.tolist()))
        d["PN"] = PN
        d["PT"] = PT
        return d

    def flat_sigma0(self):
        nx = self.shape[2]
        PN = np.zeros(nx)
        PT = np.zeros(nx)
        s0 = lib().orc_flat_sigma0(ctypes.byref(self.p), _dp(self.f), _dp(PN), _dp(PT))
        return s0, PN, PT

    def stats(self):
        out = np.zeros(9)
        lib().orc_stats(ctypes.byref(self.p), _dp(self.f), _dp(out))
        return {"mass": out[0:2].copy(), "momentum": out[2:5].copy(),
                "min_n": out[5:7].copy(), "max_u": out[7], "n_nonfinite": int(out[8])}


def flat_equilibrium(dim, stencil, g, psi_self=PSI_N, tau=1.0, lx=128,
                     guess=(1.0, 0.04, 0.04, 1.0), tol=1e-12, max_steps=200000,
                     chunk=2048, nthreads=1):
    """First stage of the two-stage initialisation of Sec. 4: relax a flat
    interface to its steady state and return the bulk concentrations.

    The box is lx x 5 (x 5 in 3D) periodic nodes; an A-rich strip
    x in [lx/4, 3 lx/4) starts at guess = (nA_in, nB_in, nA_out, nB_out) and the
    rest at the swapped phase.  The run goes in chunks of ``chunk`` steps until
    no bulk value (strip centre x = lx/2, box edge x = 0, on one transverse row)
    moves by more than ``tol`` over a chunk.  Returns ([nA_in, nB_in, nA_out,
    nB_out], steps); raises FloatingPointError if the run diverges."""
    shape = (5, lx) if dim == 2 else (5, 5, lx)
    o = Oracle(dim, stencil, shape, tau=tau, g=g, psi_self=psi_self, nthreads=nthreads)
    x = np.arange(lx)
    inside = (x >= lx // 4) & (x < 3 * lx // 4)
    nA = np.broadcast_to(np.where(inside, guess[0], guess[2]), o.shape).copy()
    nB = np.broadcast_to(np.where(inside, guess[1], guess[3]), o.shape).copy()
    o.set_density(nA, nB)
    prev = np.zeros(4)
    done = 0
    while done < max_steps:
        k = min(chunk, max_steps - done)
        o.run(k)
        done += k
        n = o.density()
        row = n[:, 2 if dim == 3 else 0, 2]
        cur = np.array([row[0, lx // 2], row[1, lx // 2], row[0, 0], row[1, 0]])
        if not np.all(np.isfinite(cur)):
            raise FloatingPointError("flat interface run diverged")
        change = np.max(np.abs(cur - prev))
        prev = cur
        if done > k and change <= tol:
            break
    return prev.tolist(), done


def delta_u(u1, u0):
    """Convergence criterion (ii) of Sec. 4: the mean over sites of
    sum_a |u_a(x, t + dt) - u_a(x, t)|; u arrays shaped (3, *box)."""
    u1 = np.asarray(u1, dtype=np.float64)
    u0 = np.asarray(u0, dtype=np.float64)
    n_sites = u1[0].size
    return float(np.abs(u1 - u0).sum() / n_sites)


def excess_com(n, shape):
    """Centre of a droplet (Sec. 4 requires it within 1e-3 of the box centre):
    the component richer at the centre node c = floor(L/2) per axis, its
    excess concentration over the value at the far node (c + floor(L/2)) mod L,
    and the excess-weighted mean of x - c per axis, plus c.  n has shape
    (2, nz, ny, nx); returns (com[3] as x, y, z; rich component)."""
    nz, ny, nx = shape
    c = (nz // 2, ny // 2, nx // 2)
    far = ((c[0] + nz // 2) % nz, (c[1] + ny // 2) % ny, (c[2] + nx // 2) % nx)
    rich = 1 if n[1][c] > n[0][c] else 0
    ex = n[rich] - n[rich][far]
    total = ex.sum()
    z, y, x = np.meshgrid(np.arange(nz) - c[0], np.arange(ny) - c[1], np.arange(nx) - c[2],
                          indexing="ij")
    com = [c[2] + (ex * x).sum() / total, c[1] + (ex * y).sum() / total,
           c[0] + (ex * z).sum() / total if nz > 1 else 0.0]
    return np.array(com), rich


def curvature_fit(curvature, sigma):
    """Curvature expansion of eq. sigma_c (Sec. 4): the quadratic
    sigma = c0 + c1 c + c2 c^2 in the signed curvature c = +-1/R_s (negative
    for droplets of the B-rich phase) fitted by least squares; sigma_0 = c0,
    the Tolman length delta = -c1 / (2 c0) and 2 kbar + k = c2 / c0."""
    c = np.asarray(curvature, dtype=np.float64)
    s = np.asarray(sigma, dtype=np.float64)
    A = np.stack([np.ones_like(c), c, c * c], axis=1)
    (c0, c1, c2), *_ = np.linalg.lstsq(A, s, rcond=None)
    return c0, -c1 / (2.0 * c0), c2 / c0

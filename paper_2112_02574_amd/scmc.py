"""Python binding of libscmc (ctypes; argument marshalling only).

Every function of the C ABI in ``include/scmc.h`` is exposed under the same
name; ``Sim`` and ``Batch`` wrap a handle together with its device workspace,
which is a PyTorch uint8 tensor on the GPU (PyTorch supplies device memory and
the HIP stream, nothing else).  Every step of the method runs in the HIP
library; when ``libscmc.so`` is missing or no GPU is present the calls fail
loudly instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libscmc.so")

# enums of scmc.h
D2Q9, D3Q19 = 0, 1
E4, E6, E8 = 4, 6, 8
PSI_N, PSI_EXP_NEG_INV = 0, 1
F64, F32, F16_OFF, BF16_OFF, F16_NODE, BF16_NODE = 0, 1, 2, 3, 4, 5
KERNEL_AUTO, KERNEL_TWO_PASS, KERNEL_FUSED, KERNEL_FUSED_REPULL, KERNEL_FUSED_PIPE = 0, 1, 2, 3, 4
KERNEL_FUSED_MOM, KERNEL_FUSED_MOM_PIPE, KERNEL_TWO_PASS_MOM = 5, 6, 7
ROUND_NEAREST, ROUND_STOCHASTIC = 0, 1
OBS_FLAT, OBS_DROPLET, OBS_SHELL = 0, 1, 2
STORAGE_NAMES = {F64: "f64", F32: "f32", F16_OFF: "f16", BF16_OFF: "bf16", F16_NODE: "f16_node",
                 BF16_NODE: "bf16_node"}

STATUS = {0: "SCMC_OK", -1: "SCMC_EINVAL", -2: "SCMC_EUNSUPPORTED",
          -3: "SCMC_ENOSPACE", -4: "SCMC_EDEVICE", -5: "SCMC_ENONFINITE",
          -6: "SCMC_ESTATE"}


class ScmcError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {msg}")


class Problem(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("stencil", ctypes.c_int),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("tau", ctypes.c_double * 2), ("g", (ctypes.c_double * 2) * 2),
                ("psi_self", ctypes.c_int), ("storage", ctypes.c_int),
                ("n0", ctypes.c_double * 2), ("kernel", ctypes.c_int),
                ("tile", ctypes.c_int * 3), ("rounding", ctypes.c_int),
                ("seed", ctypes.c_uint)]


class Stats(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double * 2), ("momentum", ctypes.c_double * 3),
                ("min_n", ctypes.c_double * 2), ("max_u", ctypes.c_double),
                ("n_nonfinite", ctypes.c_double), ("step", ctypes.c_int64)]

    def as_dict(self):
        return {"mass": np.array(self.mass[:]), "momentum": np.array(self.momentum[:]),
                "min_n": np.array(self.min_n[:]), "max_u": self.max_u,
                "n_nonfinite": int(self.n_nonfinite), "step": int(self.step)}


class Obs(ctypes.Structure):
    _fields_ = [("P_in", ctypes.c_double), ("P_out", ctypes.c_double),
                ("dP", ctypes.c_double), ("C_d", ctypes.c_double),
                ("R_s", ctypes.c_double), ("sigma_s", ctypes.c_double),
                ("R_s_grid", ctypes.c_double), ("sigma0", ctypes.c_double),
                ("max_PyyPzz", ctypes.c_double), ("step", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Convergence(ctypes.Structure):
    _fields_ = [("dP", ctypes.c_double), ("dP_change", ctypes.c_double),
                ("du", ctypes.c_double), ("com", ctypes.c_double * 3),
                ("com_offset", ctypes.c_double), ("rich", ctypes.c_int),
                ("converged", ctypes.c_int), ("step", ctypes.c_int64),
                ("prev_step", ctypes.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["com"] = np.array(self.com[:])
        d["converged"] = bool(self.converged)
        return d


_lib = None
_SYMBOLS = {
    "scmc_problem_init": ([ctypes.POINTER(Problem)], ctypes.c_int),
    "scmc_velocities": ([ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "scmc_workspace_bytes": ([ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "scmc_create": ([ctypes.POINTER(Problem), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                     ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "scmc_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "scmc_set_density": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "scmc_step": ([ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "scmc_set_graph_steps": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "scmc_synchronize": ([ctypes.c_void_p], ctypes.c_int),
    "scmc_get_fields": ([ctypes.c_void_p] + [ctypes.c_void_p] * 3, ctypes.c_int),
    "scmc_get_populations": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "scmc_set_populations": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "scmc_stats_get": ([ctypes.c_void_p, ctypes.POINTER(Stats)], ctypes.c_int),
    "scmc_observables": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.POINTER(Obs),
                          ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "scmc_batch_workspace_bytes": ([ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                                   ctypes.c_int),
    "scmc_batch_create": ([ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                           ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "scmc_batch_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "scmc_batch_set_density": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "scmc_batch_step": ([ctypes.c_void_p, ctypes.c_int64], ctypes.c_int),
    "scmc_batch_set_graph_steps": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "scmc_batch_get_fields": ([ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 3, ctypes.c_int),
    "scmc_batch_get_populations": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "scmc_batch_stats_get": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Stats)], ctypes.c_int),
    "scmc_batch_observables": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                ctypes.POINTER(Obs), ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "scmc_batch_config": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                          ctypes.c_int),
    "scmc_autotune": ([ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "scmc_batch_autotune": ([ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "scmc_config": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "scmc_pull_copy": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "scmc_convergence_check": ([ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.POINTER(Convergence)], ctypes.c_int),
    "scmc_run_to_convergence": ([ctypes.c_void_p, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_double, ctypes.c_double, ctypes.POINTER(Convergence)],
                                ctypes.c_int),
    "scmc_flat_workspace_bytes": ([ctypes.POINTER(Problem), ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                                  ctypes.c_int),
    "scmc_flat_equilibrium": ([ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "scmc_curvature_fit": ([ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "scmc_step_static": ([ctypes.POINTER(Problem), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                         ctypes.c_int),
    "scmc_last_error": ([ctypes.c_void_p], ctypes.c_char_p),
    "scmc_batch_last_error": ([ctypes.c_void_p], ctypes.c_char_p),
    "scmc_status_str": ([ctypes.c_int], ctypes.c_char_p),
}


def lib():
    """Load libscmc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: run __graft_entry__.build() first")
        # torch first: its HIP runtime must be the one libscmc binds to, or the
        # process holds two runtimes and neither sees the other's device memory
        import torch  # noqa: F401
        L = ctypes.CDLL(LIBPATH)
        for name, (args, res) in _SYMBOLS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SYMBOLS)


def _profile_len(p, kind):
    """Values of the PN / PT profiles of an observable kind."""
    if kind == OBS_DROPLET:
        return p.nx // 2 + 1
    if kind == OBS_SHELL:
        ext = [p.nx, p.ny] + ([p.nz] if p.lattice == D3Q19 else [])
        return min(ext) // 2 + 1
    return p.nx


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def problem(lattice=D3Q19, stencil=E6, shape=(64, 64, 64), tau=1.0,
            g=((0.0, 1.8), (1.8, 0.0)), psi_self=PSI_N, storage=F32, n0=(0.52, 0.52),
            kernel=KERNEL_AUTO, tile=(0, 0, 0), rounding=0, seed=0):
    """Problem struct; shape is (nz, ny, nx) in 3D or (ny, nx) in 2D."""
    p = Problem()
    lib().scmc_problem_init(ctypes.byref(p))
    p.lattice = lattice
    p.stencil = stencil
    if len(shape) == 2:
        p.nz, (p.ny, p.nx) = 1, shape
    else:
        p.nz, p.ny, p.nx = shape
    p.tau[0] = p.tau[1] = float(tau)
    for J in range(2):
        for K in range(2):
            p.g[J][K] = float(g[J][K])
    p.psi_self = psi_self
    p.storage = storage
    p.n0[0], p.n0[1] = n0
    p.kernel = kernel
    for a in range(3):
        p.tile[a] = int(tile[a])
    p.rounding = int(rounding)
    p.seed = int(seed) & 0xFFFFFFFF
    return p


def velocities(lattice):
    q = 9 if lattice == D2Q9 else 19
    xi = (ctypes.c_int * 57)()
    w = (ctypes.c_double * 19)()
    rc = lib().scmc_velocities(lattice, xi, w)
    if rc < 0:
        raise ScmcError(rc)
    return np.array(xi[:3 * q]).reshape(q, 3), np.array(w[:q])


def scmc_workspace_bytes(p):
    out = ctypes.c_size_t()
    rc = lib().scmc_workspace_bytes(ctypes.byref(p), ctypes.byref(out))
    if rc:
        raise ScmcError(rc, "scmc_workspace_bytes")
    return out.value


def _device_buffer(nbytes, device):
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libscmc needs a GPU (torch.cuda.is_available() is False)")
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def scmc_flat_equilibrium(p, lx=128, guess=None, max_steps=200000, tol=1e-12,
                          device="cuda:0", stream=None):
    """Bulk concentrations {nA_in, nB_in, nA_out, nB_out} of a converged flat
    interface with the problem's couplings (the paper's first stage)."""
    import torch
    need = ctypes.c_size_t()
    rc = lib().scmc_flat_workspace_bytes(ctypes.byref(p), int(lx), ctypes.byref(need))
    if rc:
        raise ScmcError(rc, "scmc_flat_workspace_bytes")
    ws = _device_buffer(need.value, device)
    with torch.cuda.device(ws.device):
        st = stream if stream is not None else torch.cuda.current_stream()
    g = None if guess is None else _f64(guess, 4)
    out = np.zeros(4)
    steps = ctypes.c_int64()
    rc = lib().scmc_flat_equilibrium(ctypes.byref(p), int(lx), _ptr(g), int(max_steps), float(tol),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     ctypes.c_void_p(st.cuda_stream), _ptr(out), ctypes.byref(steps))
    if rc:
        raise ScmcError(rc, "scmc_flat_equilibrium")
    return out, steps.value


STATIC_SCRATCH_BYTES = 64 << 20   # SCMC_STATIC_SCRATCH_BYTES


def state_bytes(p):
    """Bytes of one device population buffer of problem p (2 Q N values of
    the storage type)."""
    q = 9 if p.lattice == D2Q9 else 19
    return 2 * q * p.nx * p.ny * p.nz * {F64: 8, F32: 4}.get(p.storage, 2)


def scmc_step_static(p, src, dst, stream=None):
    """One allocation-free step of problem p from the device buffer src to dst
    (torch CUDA tensors of at least state_bytes(p) bytes, device layout)."""
    import torch
    need = state_bytes(p)
    for t in (src, dst):
        if not t.is_cuda or t.numel() * t.element_size() < need:
            raise ValueError(f"population buffers must be CUDA tensors of >= {need} bytes")
    if stream is None:
        with torch.cuda.device(src.device):
            stream = torch.cuda.current_stream()
    rc = lib().scmc_step_static(ctypes.byref(p), ctypes.c_void_p(src.data_ptr()),
                                ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
    if rc:
        raise ScmcError(rc, "scmc_step_static: " + lib().scmc_last_error(None).decode())


def scmc_curvature_fit(curvature, sigma):
    """(sigma_0, delta, 2 kbar + k) of eq. sigma_c fitted to signed
    curvatures 1/R_s (negative for B-rich droplets) and surface tensions."""
    k = _f64(curvature, len(curvature))
    sg = _f64(sigma, len(k))
    out = np.zeros(3)
    rc = lib().scmc_curvature_fit(len(k), _ptr(k), _ptr(sg), _ptr(out))
    if rc:
        raise ScmcError(rc, "scmc_curvature_fit")
    return tuple(float(v) for v in out)


class Sim:
    """One periodic lattice.  ``stream`` is a torch.cuda.Stream or None (the
    current stream)."""

    def __init__(self, p, device="cuda:0", stream=None):
        import torch
        self.p = p
        self.q = 9 if p.lattice == D2Q9 else 19
        self.shape = (p.nz, p.ny, p.nx)
        self.N = p.nx * p.ny * p.nz
        self.ws = _device_buffer(scmc_workspace_bytes(p), device)
        with torch.cuda.device(self.ws.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
        # the library queues its kernels on self.stream: tell the caching
        # allocator, so the workspace is not handed out again while they run
        self.ws.record_stream(self.stream)
        h = ctypes.c_void_p()
        rc = lib().scmc_create(ctypes.byref(p), ctypes.c_void_p(self.ws.data_ptr()),
                               self.ws.numel(), ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.byref(h))
        if rc:
            raise ScmcError(rc, "scmc_create")
        self.h = h

    def _check(self, rc, what):
        if rc:
            raise ScmcError(rc, f"{what}: {lib().scmc_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None):
            lib().scmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scmc_set_density(self, nA, nB):
        a, b = _f64(nA, self.N), _f64(nB, self.N)
        self._check(lib().scmc_set_density(self.h, _ptr(a), _ptr(b)), "scmc_set_density")

    def scmc_step(self, n):
        self._check(lib().scmc_step(self.h, int(n)), "scmc_step")

    def scmc_set_graph_steps(self, k):
        self._check(lib().scmc_set_graph_steps(self.h, int(k)), "scmc_set_graph_steps")

    def scmc_synchronize(self):
        self._check(lib().scmc_synchronize(self.h), "scmc_synchronize")

    def scmc_get_fields(self, velocity=False):
        nA = np.zeros(self.N)
        nB = np.zeros(self.N)
        u = np.zeros(3 * self.N) if velocity else None
        self._check(lib().scmc_get_fields(self.h, _ptr(nA), _ptr(nB), _ptr(u)), "scmc_get_fields")
        n = np.stack([nA, nB]).reshape((2,) + self.shape)
        return (n, u.reshape((3,) + self.shape)) if velocity else n

    def scmc_get_populations(self):
        f = np.zeros(2 * self.q * self.N)
        step = ctypes.c_int64()
        self._check(lib().scmc_get_populations(self.h, _ptr(f), ctypes.byref(step)),
                    "scmc_get_populations")
        return f.reshape((2, self.q) + self.shape), step.value

    def scmc_set_populations(self, f, step=0):
        a = _f64(f, 2 * self.q * self.N)
        self._check(lib().scmc_set_populations(self.h, _ptr(a), int(step)), "scmc_set_populations")

    def scmc_stats_get(self):
        s = Stats()
        self._check(lib().scmc_stats_get(self.h, ctypes.byref(s)), "scmc_stats_get")
        return s.as_dict()

    def scmc_observables(self, kind, R0=1.0):
        o = Obs()
        n = _profile_len(self.p, kind)
        PN = np.zeros(n)
        PT = np.zeros(n)
        self._check(lib().scmc_observables(self.h, kind, float(R0), ctypes.byref(o), _ptr(PN), _ptr(PT)),
                    "scmc_observables")
        d = o.as_dict()
        d["PN"], d["PT"] = PN, PT
        return d

    def scmc_convergence_check(self, R0, tol_dP=1e-5, tol_du=1e-12):
        o = Convergence()
        self._check(lib().scmc_convergence_check(self.h, float(R0), float(tol_dP), float(tol_du),
                                                  ctypes.byref(o)), "scmc_convergence_check")
        return o.as_dict()

    def scmc_run_to_convergence(self, R0, dt=2048, max_steps=200000, tol_dP=1e-5, tol_du=1e-12):
        o = Convergence()
        self._check(lib().scmc_run_to_convergence(self.h, float(R0), int(dt), int(max_steps),
                                                   float(tol_dP), float(tol_du), ctypes.byref(o)),
                    "scmc_run_to_convergence")
        return o.as_dict()

    def scmc_config(self):
        k = ctypes.c_int()
        t = (ctypes.c_int * 3)()
        self._check(lib().scmc_config(self.h, ctypes.byref(k), t), "scmc_config")
        return k.value, tuple(t)

    def scmc_pull_copy(self, reps):
        us = ctypes.c_double()
        self._check(lib().scmc_pull_copy(self.h, int(reps), ctypes.byref(us)), "scmc_pull_copy")
        return us.value

    def scmc_autotune(self, cache_path=None):
        t = (ctypes.c_int * 3)()
        self._check(lib().scmc_autotune(self.h, cache_path.encode() if cache_path else None, t),
                    "scmc_autotune")
        return tuple(t)


class Batch:
    """Many independent lattices stepped by one persistent launch per step."""

    def __init__(self, problems, device="cuda:0", stream=None):
        import torch
        self.problems = list(problems)
        self.count = len(self.problems)
        arr = (Problem * self.count)(*self.problems)
        self._arr = arr
        need = ctypes.c_size_t()
        rc = lib().scmc_batch_workspace_bytes(arr, self.count, ctypes.byref(need))
        if rc:
            raise ScmcError(rc, "scmc_batch_workspace_bytes")
        self.ws = _device_buffer(need.value, device)
        with torch.cuda.device(self.ws.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws.record_stream(self.stream)  # as in Sim
        h = ctypes.c_void_p()
        rc = lib().scmc_batch_create(arr, self.count, ctypes.c_void_p(self.ws.data_ptr()),
                                     self.ws.numel(), ctypes.c_void_p(self.stream.cuda_stream),
                                     ctypes.byref(h))
        if rc:
            raise ScmcError(rc, "scmc_batch_create")
        self.h = h

    def _check(self, rc, what):
        if rc:
            raise ScmcError(rc, f"{what}: {lib().scmc_batch_last_error(self.h).decode()}")

    def close(self):
        if getattr(self, "h", None):
            lib().scmc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _n(self, i):
        p = self.problems[i]
        return p.nx * p.ny * p.nz, (p.nz, p.ny, p.nx)

    def scmc_batch_set_density(self, i, nA, nB):
        N, _ = self._n(i)
        a, b = _f64(nA, N), _f64(nB, N)
        self._check(lib().scmc_batch_set_density(self.h, i, _ptr(a), _ptr(b)), "scmc_batch_set_density")

    def scmc_batch_step(self, n):
        self._check(lib().scmc_batch_step(self.h, int(n)), "scmc_batch_step")

    def scmc_batch_set_graph_steps(self, k):
        self._check(lib().scmc_batch_set_graph_steps(self.h, int(k)), "scmc_batch_set_graph_steps")

    def scmc_batch_get_fields(self, i, velocity=False):
        N, shp = self._n(i)
        nA, nB = np.zeros(N), np.zeros(N)
        u = np.zeros(3 * N) if velocity else None
        self._check(lib().scmc_batch_get_fields(self.h, i, _ptr(nA), _ptr(nB), _ptr(u)),
                    "scmc_batch_get_fields")
        n = np.stack([nA, nB]).reshape((2,) + shp)
        return (n, u.reshape((3,) + shp)) if velocity else n

    def scmc_batch_get_populations(self, i):
        N, shp = self._n(i)
        q = 9 if self.problems[i].lattice == D2Q9 else 19
        f = np.zeros(2 * q * N)
        step = ctypes.c_int64()
        self._check(lib().scmc_batch_get_populations(self.h, i, _ptr(f), ctypes.byref(step)),
                    "scmc_batch_get_populations")
        return f.reshape((2, q) + shp), step.value

    def scmc_batch_stats_get(self, i):
        s = Stats()
        self._check(lib().scmc_batch_stats_get(self.h, i, ctypes.byref(s)), "scmc_batch_stats_get")
        return s.as_dict()

    def scmc_batch_observables(self, i, kind, R0=1.0):
        o = Obs()
        p = self.problems[i]
        n = _profile_len(p, kind)
        PN, PT = np.zeros(n), np.zeros(n)
        self._check(lib().scmc_batch_observables(self.h, i, kind, float(R0), ctypes.byref(o),
                                                 _ptr(PN), _ptr(PT)), "scmc_batch_observables")
        d = o.as_dict()
        d["PN"], d["PT"] = PN, PT
        return d

    def scmc_batch_config(self):
        t = (ctypes.c_int * 3)()
        g = ctypes.c_int()
        self._check(lib().scmc_batch_config(self.h, t, ctypes.byref(g)), "scmc_batch_config")
        return tuple(t), g.value

    def scmc_batch_autotune(self, cache_path=None):
        t = (ctypes.c_int * 3)()
        self._check(lib().scmc_batch_autotune(self.h, cache_path.encode() if cache_path else None, t),
                    "scmc_batch_autotune")
        return tuple(t)

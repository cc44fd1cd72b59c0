"""The C ABI boundary without a GPU: libscmc.so loads, exports every function
that include/scmc.h declares, and its host-side validation rejects bad
problems with the documented status codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2112_02574_amd import scmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scmc_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = scmc.lib()
    names = declared_functions()
    assert len(names) >= 30
    for n in names:
        assert hasattr(L, n), n
    assert sorted(scmc.exported_symbols()) == names


def test_velocity_tables_match_the_oracle_sets():
    for lat, dim in ((scmc.D2Q9, 2), (scmc.D3Q19, 3)):
        xi, w = scmc.velocities(lat)
        oxi, ow = O.lattice(dim)
        assert {tuple(v) for v in xi} == {tuple(v) for v in oxi}
        wmap = {tuple(v): x for v, x in zip(oxi, ow)}
        for v, x in zip(xi, w):
            assert x == wmap[tuple(v)]


def _bytes(p):
    return scmc.scmc_workspace_bytes(p)


def test_workspace_planner():
    p = scmc.problem(scmc.D3Q19, scmc.E6, (128, 128, 128), storage=scmc.F32)
    n = _bytes(p)
    N = 128 ** 3
    pops = 2 * 2 * 19 * N * 4
    # two population buffers, the 7-field moment field (FP32), FP64 densities,
    # FP64 velocity and the monitor's previous velocity, plus small buffers
    assert pops < n < pops + (7 * 4 + 2 * 8 + 2 * 3 * 8) * N + (1 << 20)
    p16 = scmc.problem(scmc.D3Q19, scmc.E6, (128, 128, 128), storage=scmc.F16_OFF)
    assert _bytes(p16) < n
    p64 = scmc.problem(scmc.D3Q19, scmc.E6, (128, 128, 128), storage=scmc.F64)
    assert _bytes(p64) > n


@pytest.mark.parametrize("mutate,status", [
    (lambda p: setattr(p, "lattice", 7), -1),
    (lambda p: setattr(p, "stencil", 5), -1),
    (lambda p: setattr(p, "stencil", scmc.E8), -2),        # E8 is 2D only
    (lambda p: setattr(p, "nx", 4), -1),                   # < 2 r_F + 1 for E6
    (lambda p: p.tau.__setitem__(0, 0.5), -1),
    (lambda p: p.tau.__setitem__(1, 0.4), -1),
    (lambda p: (setattr(p, "kernel", scmc.KERNEL_TWO_PASS_MOM),
                p.tau.__setitem__(1, 0.9)), -2),          # tau = 1 design, tau_B != 1
    (lambda p: p.g[0].__setitem__(1, 1.7), -1),            # g_AB != g_BA
    (lambda p: p.g[0].__setitem__(0, float("nan")), -1),
    (lambda p: setattr(p, "storage", 9), -1),
    (lambda p: setattr(p, "psi_self", 3), -1),
    (lambda p: setattr(p, "kernel", 8), -1),
    (lambda p: setattr(p, "rounding", 2), -1),
    (lambda p: setattr(p, "rounding", scmc.ROUND_STOCHASTIC), -1),   # FP32 storage
    (lambda p: (setattr(p, "rounding", scmc.ROUND_STOCHASTIC), setattr(p, "storage", scmc.BF16_OFF),
                setattr(p, "kernel", scmc.KERNEL_FUSED)), -2),      # two-pass designs only
    (lambda p: (setattr(p, "kernel", scmc.KERNEL_FUSED_MOM), p.tau.__setitem__(0, 0.8),
                p.tau.__setitem__(1, 0.8)), -2),          # moment ring needs tau = 1
])
def test_invalid_problems(mutate, status):
    p = scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16))
    mutate(p)
    out = ctypes.c_size_t()
    assert scmc.lib().scmc_workspace_bytes(ctypes.byref(p), ctypes.byref(out)) == status
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: validation fails first
    assert scmc.lib().scmc_create(ctypes.byref(p), fake, 1 << 40, None, ctypes.byref(h)) == status
    assert not h.value


def test_2d_needs_nz_one():
    p = scmc.problem(scmc.D2Q9, scmc.E8, (32, 32))
    assert _bytes(p) > 0
    p.nz = 2
    out = ctypes.c_size_t()
    assert scmc.lib().scmc_workspace_bytes(ctypes.byref(p), ctypes.byref(out)) == -1


def test_small_workspace_and_null_arguments():
    p = scmc.problem(scmc.D2Q9, scmc.E4, (16, 16))
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)
    assert scmc.lib().scmc_create(ctypes.byref(p), fake, 1024, None, ctypes.byref(h)) == -3
    assert scmc.lib().scmc_create(ctypes.byref(p), None, 1 << 30, None, ctypes.byref(h)) == -1
    assert scmc.lib().scmc_create(ctypes.byref(p), ctypes.c_void_p((1 << 20) + 8), 1 << 30, None,
                                  ctypes.byref(h)) == -1  # misaligned
    assert scmc.lib().scmc_step(None, 1) == -1
    assert scmc.lib().scmc_status_str(-3) == b"workspace too small"


def test_batch_members_must_share_lattice():
    a = scmc.problem(scmc.D3Q19, scmc.E6, (48, 48, 48))
    b = scmc.problem(scmc.D3Q19, scmc.E4, (56, 56, 56))
    arr = (scmc.Problem * 2)(a, b)
    out = ctypes.c_size_t()
    assert scmc.lib().scmc_batch_workspace_bytes(arr, 2, ctypes.byref(out)) == -1
    c = scmc.problem(scmc.D3Q19, scmc.E6, (56, 64, 72), g=((-0.2, 1.8), (1.8, 0.0)))
    arr = (scmc.Problem * 2)(a, c)
    assert scmc.lib().scmc_batch_workspace_bytes(arr, 2, ctypes.byref(out)) == 0
    assert out.value > 2 * 2 * 19 * 4 * (48 ** 3 + 56 * 64 * 72)


def test_unequal_tau_is_accepted_by_the_tau_general_designs():
    for kernel in (scmc.KERNEL_AUTO, scmc.KERNEL_TWO_PASS, scmc.KERNEL_FUSED):
        p = scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16), kernel=kernel)
        p.tau[0], p.tau[1] = 0.7, 1.45
        out = ctypes.c_size_t()
        assert scmc.lib().scmc_workspace_bytes(ctypes.byref(p), ctypes.byref(out)) == 0
        assert out.value > 0


def test_node_storage_validation():
    """FP16 / BF16 offsets from the per-node reference: the moment two-pass on
    single D3Q19 lattices at tau = 1 with nearest rounding, nothing else."""
    out = ctypes.c_size_t()
    for st in (scmc.F16_NODE, scmc.BF16_NODE):
        for kernel in (scmc.KERNEL_AUTO, scmc.KERNEL_TWO_PASS_MOM):
            p = scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16), storage=st, kernel=kernel)
            assert scmc.lib().scmc_workspace_bytes(ctypes.byref(p), ctypes.byref(out)) == 0
        # a second (n_A, n_B) slot and the FP32 rest populations: 10 FP32
        # values per site in the moment field instead of 7
        n_node = out.value
        p = scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16), storage=scmc.F16_OFF)
        assert scmc.lib().scmc_workspace_bytes(ctypes.byref(p), ctypes.byref(out)) == 0
        assert n_node == out.value + 3 * 16 ** 3 * 4
        bad = [
            scmc.problem(scmc.D2Q9, scmc.E8, (32, 32), storage=st),
            scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16), storage=st, tau=0.8),
            scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16), storage=st, kernel=scmc.KERNEL_FUSED),
            scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16), storage=st, kernel=scmc.KERNEL_TWO_PASS),
            scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16), storage=st,
                         rounding=scmc.ROUND_STOCHASTIC),
        ]
        for q in bad:
            assert scmc.lib().scmc_workspace_bytes(ctypes.byref(q), ctypes.byref(out)) == -2
        q = scmc.problem(scmc.D3Q19, scmc.E6, (16, 16, 16), storage=st)
        arr = (scmc.Problem * 2)(q, q)
        assert scmc.lib().scmc_batch_workspace_bytes(arr, 2, ctypes.byref(out)) == -2
        fake_src, fake_dst = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21)  # never dereferenced
        assert scmc.lib().scmc_step_static(ctypes.byref(q), fake_src, fake_dst, None) == -2

"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances (FP64 is the oracle's precision; the others follow from the
storage precision, unit roundoff u, over the number of steps run):
  * FP64 storage: populations within 1e-12 after tens of steps.
  * FP32 storage: populations within 2e-6 after tens of steps (u = 6e-8,
    O(10) roundings per update, errors grow slowly with the step count).
  * FP16 / BF16 offset storage: every stored value is rounded to 11 / 8
    significant bits of |f - w n0| <= w * 0.5; a single step is checked to
    half an ulp of the largest offset, longer runs are reported elsewhere.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2112_02574_amd import inputs
from paper_2112_02574_amd import scmc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _perm(lattice, dim):
    xi, _ = scmc.velocities(lattice)
    oxi, _ = O.lattice(dim)
    okeys = [tuple(v) for v in oxi]
    return [okeys.index(tuple(v)) for v in xi]


def _random_state(shape, seed):
    rng = np.random.default_rng(seed)
    nA = rng.uniform(0.3, 0.9, shape)
    nB = rng.uniform(0.3, 0.9, shape)
    return nA, nB


CASES = [
    # lattice, stencil, shape (nz, ny, nx) or (ny, nx), psi, couplings, initial state
    (scmc.D2Q9, scmc.E4, (37, 70), scmc.PSI_N, ((0.0, 1.2), (1.2, 0.0)), "random"),
    (scmc.D2Q9, scmc.E6, (21, 67), scmc.PSI_EXP_NEG_INV, ((-1.0, 0.5), (0.5, -0.6)), "random"),
    (scmc.D2Q9, scmc.E8, (33, 129), scmc.PSI_N, ((-0.1, 1.4), (1.4, 0.05)), "random"),
    (scmc.D3Q19, scmc.E4, (9, 13, 70), scmc.PSI_N, ((0.0, 1.2), (1.2, 0.0)), "random"),
    (scmc.D3Q19, scmc.E6, (11, 7, 67), scmc.PSI_EXP_NEG_INV, ((-1.0, 0.5), (0.5, -0.6)), "random"),
    (scmc.D3Q19, scmc.E6, (6, 9, 130), scmc.PSI_N, ((-0.1, 1.4), (1.4, 0.05)), "random"),
    # the benchmark's instantiation (E6, psi = n, symmetric g_AB = 1.8) on a
    # ragged box: a droplet between the bulk values of the flat stage
    (scmc.D3Q19, scmc.E6, (10, 12, 66), scmc.PSI_N, ((0.0, 1.8), (1.8, 0.0)), "droplet"),
]

# designs: (kernel, tile); the moment designs run tau = 1 only, the fused and
# LDS-staged ones D3Q19 with FP32-compute storage only
DESIGNS = {
    "two_pass": (scmc.KERNEL_TWO_PASS, (0, 0, 0)),
    "auto": (scmc.KERNEL_AUTO, (0, 0, 0)),
    "two_pass_mom": (scmc.KERNEL_TWO_PASS_MOM, (0, 0, 0)),
    "two_pass_mom_lds": (scmc.KERNEL_TWO_PASS_MOM, (64, 8, 8)),
    "fused_mom": (scmc.KERNEL_FUSED_MOM, (64, 8, 16)),
}
TAU_GENERAL = ("two_pass", "auto")


def _oracle_for(lattice, stencil, shape, psi, g, tau=1.0):
    dim = 2 if lattice == scmc.D2Q9 else 3
    return O.Oracle(dim, stencil, shape, tau=tau, g=g, psi_self=psi)


def _initial_state(case):
    lattice, _, shape, _, _, init = CASES[case]
    if init == "random":
        return _random_state(shape, 100 + case)
    if lattice == scmc.D2Q9:
        return inputs.droplet(shape[1], shape[0], R=shape[0] / 4)
    nz, ny, nx = shape
    return inputs.droplet(nx, ny, nz, R=min(shape) / 3, bulk=(1.06, -0.001, -0.001, 1.06))


@pytest.mark.parametrize("design", list(DESIGNS))
@pytest.mark.parametrize("tau", [1.0, 0.8])
@pytest.mark.parametrize("storage,tol,steps", [(scmc.F64, 1e-12, 25), (scmc.F32, 2e-6, 25)])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_populations_match_oracle(case, storage, tol, steps, tau, design):
    """Every design at tau = 1 (the configurations of the benchmark), and the
    tau-general designs also at tau = 0.8, against the oracle: populations,
    fields and statistics after 25 steps."""
    lattice, stencil, shape, psi, g, _ = CASES[case]
    kernel, tile = DESIGNS[design]
    if tau != 1.0 and design not in TAU_GENERAL:
        pytest.skip("moment designs need tau = 1")
    if design in ("fused_mom", "two_pass_mom_lds") and (lattice == scmc.D2Q9 or storage == scmc.F64):
        pytest.skip("fused and LDS-staged designs are D3Q19 with FP32-compute storage")
    print(f"case {case} storage {storage} tau {tau} design {design} shape {shape}", flush=True)
    nA, nB = _initial_state(case)
    p = scmc.problem(lattice, stencil, shape, tau=tau, g=g, psi_self=psi, storage=storage,
                     kernel=kernel, tile=tile)
    sim = scmc.Sim(p)
    if kernel != scmc.KERNEL_AUTO:
        assert sim.scmc_config() == (kernel, tile)
    elif tau == 1.0:
        assert sim.scmc_config() == (scmc.KERNEL_TWO_PASS_MOM, (0, 0, 0))
    sim.scmc_set_density(nA, nB)
    sim.scmc_step(steps)
    f, step = sim.scmc_get_populations()
    assert step == steps
    o = _oracle_for(lattice, stencil, shape, psi, g, tau)
    o.set_density(nA, nB)
    o.run(steps)
    dim = 2 if lattice == scmc.D2Q9 else 3
    fo = o.f[:, _perm(lattice, dim)].reshape(f.shape)
    err = np.abs(f - fo).max()
    assert np.isfinite(f).all()
    assert err < tol, err
    # fields and statistics of the same state
    n, u = sim.scmc_get_fields(velocity=True)
    assert np.abs(n - o.density()).max() < tol * 10
    assert np.abs(u - o.velocity()).max() < tol * 10
    st, so = sim.scmc_stats_get(), o.stats()
    np.testing.assert_allclose(st["mass"], so["mass"], rtol=1e-12 if storage == scmc.F64 else 1e-6)
    if storage == scmc.F64:
        assert np.abs(st["momentum"] - so["momentum"]).max() < 1e-11
    np.testing.assert_allclose(st["min_n"], so["min_n"], atol=tol * 10)
    assert abs(st["max_u"] - so["max_u"]) < tol * 10
    # the FP64 reductions against the oracle's statistics of the very same
    # (GPU-produced) state: FP32 storage breaks exact conservation by its
    # rounding, so momentum is compared state for state
    o.set_populations(f[:, np.argsort(_perm(lattice, dim))].reshape(o.f.shape))
    so2 = o.stats()
    np.testing.assert_allclose(st["mass"], so2["mass"], rtol=1e-13)
    assert np.abs(st["momentum"] - so2["momentum"]).max() < 1e-10
    assert abs(st["max_u"] - so2["max_u"]) < 1e-12
    np.testing.assert_array_equal(st["min_n"], so2["min_n"])
    sim.close()


@pytest.mark.parametrize("design", ["auto", "two_pass_mom_lds"])
@pytest.mark.parametrize("storage,bits", [(scmc.F16_OFF, 11), (scmc.BF16_OFF, 8)])
def test_offset_storage_single_step(storage, bits, design):
    """One step from an equilibrium start: the stored h = f* - w n0 carries the
    rounding of the storage format only.  Both forms of the moment two-pass:
    direct stencil gathers and the LDS-staged collision pass."""
    shape = (10, 12, 66)
    nA, nB = inputs.droplet(66, 12, 10, R=5.0)
    g = ((0.0, 1.8), (1.8, 0.0))
    kernel, tile = DESIGNS[design]
    p = scmc.problem(scmc.D3Q19, scmc.E6, shape, g=g, storage=storage, n0=(0.52, 0.52),
                     kernel=kernel, tile=tile)
    sim = scmc.Sim(p)
    assert sim.scmc_config() == (scmc.KERNEL_TWO_PASS_MOM, tile)
    sim.scmc_set_density(nA, nB)
    f0, _ = sim.scmc_get_populations()
    sim.scmc_step(1)
    f1, _ = sim.scmc_get_populations()
    o = O.Oracle(3, 6, shape, g=g)
    o.set_populations(f0[:, np.argsort(_perm(scmc.D3Q19, 3))])  # GPU order -> oracle order
    o.run(1)
    fo = o.f[:, _perm(scmc.D3Q19, 3)]
    _, w = scmc.velocities(scmc.D3Q19)
    half_ulp = 0.5 * 2.0 ** (1 - bits) * (w * 0.52 + 0.1)  # |h| < w n0 + margin
    err = np.abs(f1 - fo)
    assert (err <= half_ulp[None, :, None, None, None] * 1.05 + 1e-7).all(), err.max()
    sim.close()


def test_stats_and_observables_match_oracle_fp64():
    L, R0 = 32, 8.0
    nA, nB = inputs.droplet(L, L, L, R=R0)
    g = ((0.0, 1.8), (1.8, 0.0))
    p = scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), g=g, storage=scmc.F64)
    sim = scmc.Sim(p)
    sim.scmc_set_density(nA, nB)
    sim.scmc_step(400)
    o = O.Oracle(3, 6, (L, L, L), g=g)
    o.set_density(nA, nB)
    o.run(400)
    ob, oo = sim.scmc_observables(scmc.OBS_DROPLET, R0), o.droplet_observables(R0)
    assert oo["dP"] > 0 and oo["C_d"] > 0  # a settled droplet
    for k in ("P_in", "P_out", "dP", "C_d", "R_s", "R_s_grid", "sigma_s"):
        assert abs(ob[k] - oo[k]) < 1e-10 * max(1.0, abs(oo[k])), (k, ob[k], oo[k])
    assert np.abs(ob["PN"] - oo["PN"]).max() < 1e-12
    assert np.abs(ob["PT"] - oo["PT"]).max() < 1e-12
    assert ob["max_PyyPzz"] < 1e-13
    sim.close()


def test_flat_sigma0_matches_oracle():
    nA, nB = inputs.slab(64, 64, noise=1e-3, seed=1)
    g = ((0.0, 1.8), (1.8, 0.0))
    for storage, tol in ((scmc.F64, 1e-11), (scmc.F32, 2e-5)):
        p = scmc.problem(scmc.D2Q9, scmc.E4, (64, 64), g=g, storage=storage)
        sim = scmc.Sim(p)
        sim.scmc_set_density(nA, nB)
        sim.scmc_step(200)
        o = O.Oracle(2, 4, (64, 64), g=g)
        o.set_density(nA, nB)
        o.run(200)
        ob = sim.scmc_observables(scmc.OBS_FLAT)
        s0, PN, PT = o.flat_sigma0()
        assert abs(ob["sigma0"] - s0) < tol, (storage, ob["sigma0"], s0)
        assert np.abs(ob["PN"] - PN).max() < tol
        assert np.abs(ob["PT"] - PT).max() < tol
        sim.close()


def test_checkpoint_resume_is_bitwise():
    shape = (12, 10, 40)
    nA, nB = _random_state(shape, 7)
    g = ((-0.1, 1.4), (1.4, 0.05))
    for storage in (scmc.F32, scmc.F64):
        p = scmc.problem(scmc.D3Q19, scmc.E6, shape, g=g, storage=storage)
        a = scmc.Sim(p)
        a.scmc_set_density(nA, nB)
        a.scmc_step(20)
        fa, _ = a.scmc_get_populations()
        b = scmc.Sim(p)
        b.scmc_set_density(nA, nB)
        b.scmc_step(10)
        ck, st = b.scmc_get_populations()
        c = scmc.Sim(p)
        c.scmc_set_populations(ck, st)
        c.scmc_step(10)
        fc, stc = c.scmc_get_populations()
        assert stc == 20
        assert np.array_equal(fa, fc)
        for s in (a, b, c):
            s.close()


def test_deterministic_reductions():
    shape = (16, 16, 16)
    nA, nB = inputs.droplet(16, 16, 16, R=4.0)
    p = scmc.problem(scmc.D3Q19, scmc.E6, shape, storage=scmc.F32)
    runs = []
    for _ in range(2):
        s = scmc.Sim(p)
        s.scmc_set_density(nA, nB)
        s.scmc_step(30)
        runs.append((s.scmc_get_populations()[0], s.scmc_stats_get(),
                     s.scmc_observables(scmc.OBS_DROPLET, 4.0)))
        s.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    assert runs[0][1]["momentum"].tolist() == runs[1][1]["momentum"].tolist()
    assert runs[0][2]["R_s"] == runs[1][2]["R_s"]


def test_graph_replay_matches_direct_launches():
    shape = (12, 20, 36)
    nA, nB = _random_state(shape, 9)
    p = scmc.problem(scmc.D3Q19, scmc.E6, shape, g=((-0.1, 1.4), (1.4, 0.05)), storage=scmc.F32)
    a = scmc.Sim(p)
    a.scmc_set_density(nA, nB)
    a.scmc_step(23)
    fa, _ = a.scmc_get_populations()
    b = scmc.Sim(p)
    b.scmc_set_graph_steps(5)
    b.scmc_set_density(nA, nB)
    for k in (7, 11, 5):   # graph replays with odd offsets in between
        b.scmc_step(k)
        b.scmc_synchronize()
    fb, st = b.scmc_get_populations()
    assert st == 23
    assert np.isfinite(fa).all()
    assert np.array_equal(fa, fb)


def test_nonfinite_state_is_reported():
    shape = (8, 8, 8)
    nA, nB = _random_state(shape, 3)
    p = scmc.problem(scmc.D3Q19, scmc.E4, shape, g=((0.0, 5.0), (5.0, 0.0)), storage=scmc.F32)
    s = scmc.Sim(p)
    s.scmc_set_density(nA * 4.0, nB * 4.0)   # far beyond the stable coupling
    s.scmc_step(400)
    with pytest.raises(scmc.ScmcError) as e:
        s.scmc_stats_get()
    assert e.value.status == -5
    bad = nA.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(scmc.ScmcError):
        s.scmc_set_density(bad, nB)


def test_batch_matches_single_runs():
    members = [(48, 8.0, ((0.0, 1.8), (1.8, 0.0)), True),
               (40, 7.0, ((0.0, 1.8), (1.8, 0.0)), False),
               (56, 10.0, ((0.0, 1.8), (1.8, 0.0)), True)]
    ps, inits = [], []
    for L, R0, g, arich in members:
        ps.append(scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), g=g, storage=scmc.F32))
        inits.append(inputs.droplet(L, L, L, R=R0, a_rich=arich))
    b = scmc.Batch(ps)
    for i, (nA, nB) in enumerate(inits):
        b.scmc_batch_set_density(i, nA, nB)
    b.scmc_batch_step(30)
    for i, (nA, nB) in enumerate(inits):
        s = scmc.Sim(ps[i])
        s.scmc_set_density(nA, nB)
        s.scmc_step(30)
        assert np.array_equal(b.scmc_batch_get_fields(i), s.scmc_get_fields())
        ob = b.scmc_batch_observables(i, scmc.OBS_DROPLET, members[i][1])
        os_ = s.scmc_observables(scmc.OBS_DROPLET, members[i][1])
        assert ob["R_s"] == os_["R_s"]
        s.close()


@pytest.mark.parametrize("storage", [scmc.F32, scmc.F16_OFF])
@pytest.mark.parametrize("graph_steps", [0, 4])
def test_batch_in_member_chunks_matches_single_runs(graph_steps, storage):
    """Members whose moment fields exceed the chunk budget (48 MB: here
    128^3 | 128^3 | 112^3 + 48^3) run the moment two-pass chunk by chunk, the
    128^3 ones each alone with the single-lattice kernels, several steps per
    chunk; direct launches and graphs must still equal single-lattice runs
    bit for bit, in FP32 and with FP16 offsets."""
    members = [(128, 24.0, True), (128, 20.0, False), (112, 18.0, True), (48, 8.0, False)]
    ps = [scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), storage=storage) for L, _, _ in members]
    inits = [inputs.droplet(L, L, L, R=R0, a_rich=a) for L, R0, a in members]
    b = scmc.Batch(ps)
    for i, (nA, nB) in enumerate(inits):
        b.scmc_batch_set_density(i, nA, nB)
    b.scmc_batch_set_graph_steps(graph_steps)
    b.scmc_batch_step(10)
    for i, (nA, nB) in enumerate(inits):
        print(f"member {i} graph_steps {graph_steps} storage {storage}", flush=True)
        s = scmc.Sim(ps[i])
        s.scmc_set_density(nA, nB)
        s.scmc_step(10)
        assert np.array_equal(b.scmc_batch_get_fields(i), s.scmc_get_fields())
        s.close()
    b.close()


@pytest.mark.parametrize("graph_steps", [0, 5])
def test_batch_long_call_matches_single_runs(graph_steps):
    """One call of 70 steps runs chunk by chunk in blocks (direct launches: 64
    steps and then 6; graphs of 5: fourteen replays), the 128^3 member alone
    in its chunk, the others together; every member equals its single run
    bit for bit."""
    members = [(128, 24.0, True), (40, 8.0, False), (24, 6.0, True)]
    ps = [scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), storage=scmc.F32) for L, _, _ in members]
    inits = [inputs.droplet(L, L, L, R=R0, a_rich=a) for L, R0, a in members]
    b = scmc.Batch(ps)
    for i, (nA, nB) in enumerate(inits):
        b.scmc_batch_set_density(i, nA, nB)
    b.scmc_batch_set_graph_steps(graph_steps)
    b.scmc_batch_step(70)
    for i, (nA, nB) in enumerate(inits):
        s = scmc.Sim(ps[i])
        s.scmc_set_density(nA, nB)
        s.scmc_step(70)
        assert np.array_equal(b.scmc_batch_get_fields(i), s.scmc_get_fields()), i
        s.close()
    assert b.scmc_batch_get_populations(2)[1] == 70
    b.close()


G_SYM = ((0.0, 1.8), (1.8, 0.0))
G_ASYM = ((-0.2, 1.8), (1.8, 0.0))


@pytest.mark.parametrize("graph_steps", [0, 4])
@pytest.mark.parametrize("storage,tol", [(scmc.F64, 1e-12), (scmc.F32, 2e-6)])
def test_batch_members_match_oracle(storage, tol, graph_steps):
    """The batched sweep (Sec. 4's sweep over droplet sizes and couplings) in
    its benchmark design against the oracle, member by member: uneven boxes
    (one with rows that are not a multiple of 64), symmetric couplings and the
    asymmetric g_AA = -0.2 with B-rich droplets between the flat-stage guess
    values, and a 128^3 member whose moment field passes the 48 MB chunk
    budget, so the tile list runs as three chunks ([0, 1], [2], [3]).  Every
    population after 25 steps, with direct launches and with graphs of 4
    steps (six replays and one direct step)."""
    members = [((20, 20, 20), G_SYM, True, 5.0),
               ((18, 22, 70), G_ASYM, False, 6.0),
               ((128, 128, 128), G_SYM, False, 24.0),
               ((24, 24, 24), G_ASYM, False, 6.0)]
    ps, inits = [], []
    for shape, g, a_rich, R0 in members:
        nz, ny, nx = shape
        ps.append(scmc.problem(scmc.D3Q19, scmc.E6, shape, g=g, storage=storage))
        bulk = inputs.FLAT_GUESS[g[0][0]]
        inits.append(inputs.droplet(nx, ny, nz, R=R0, a_rich=a_rich, bulk=bulk))
    b = scmc.Batch(ps)
    for i, (nA, nB) in enumerate(inits):
        b.scmc_batch_set_density(i, nA, nB)
    b.scmc_batch_set_graph_steps(graph_steps)
    b.scmc_batch_step(25)
    perm = _perm(scmc.D3Q19, 3)
    for i, ((shape, g, _, R0), (nA, nB)) in enumerate(zip(members, inits)):
        f, step = b.scmc_batch_get_populations(i)
        o = O.Oracle(3, 6, shape, g=g)
        o.set_density(nA, nB)
        o.run(25)
        fo = o.f[:, perm]
        err = np.abs(f - fo).max()
        print(f"member {i} shape {shape} g_AA {g[0][0]} storage {storage} graph {graph_steps}: "
              f"max |f - f_oracle| = {err:.3g}", flush=True)
        assert step == 25 and np.isfinite(f).all()
        assert err < tol, (i, err)
        st, so = b.scmc_batch_stats_get(i), o.stats()
        np.testing.assert_allclose(st["mass"], so["mass"],
                                   rtol=1e-12 if storage == scmc.F64 else 1e-6)
    b.close()


def test_full_size_sampled_single_step():
    """128^3 D3Q19 / E6 FP32 (the benchmark workload and launch): one step from
    the droplet start; the post-collision populations at sampled sites against
    the oracle computed site by site."""
    L, R0 = 128, 24.0
    nA, nB = inputs.droplet(L, L, L, R=R0)
    p = scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), storage=scmc.F32)
    sim = scmc.Sim(p)
    # the design and tile the benchmark runs (same tuner and cache file)
    sim.scmc_autotune(os.path.join(os.environ.get("TMPDIR", "/tmp"), "scmc_autotune.txt"))
    sim.scmc_set_density(nA, nB)
    sim.scmc_step(1)
    f1, _ = sim.scmc_get_populations()
    o = O.Oracle(3, 6, (L, L, L))
    o.set_density(nA, nB)
    xi, _ = scmc.velocities(scmc.D3Q19)
    perm = _perm(scmc.D3Q19, 3)
    rng = np.random.default_rng(5)
    sites = [(64, 64, 64 + 24), (0, 0, 0), (127, 127, 127), (64, 40, 64)]
    sites += [tuple(v) for v in rng.integers(0, L, (8, 3))]
    worst = 0.0
    for (z, y, x) in sites:
        want = o.collide_site((z * L + y) * L + x)[:, perm]
        got = np.array([[f1[J, i, (z + xi[i, 2]) % L, (y + xi[i, 1]) % L, (x + xi[i, 0]) % L]
                         for i in range(19)] for J in range(2)])
        worst = max(worst, np.abs(got - want).max())
    assert worst < 1e-6, worst
    sim.close()


_GC = -np.e ** 2 / 3.0


@pytest.mark.parametrize("stencil,psi,g", [
    (scmc.E6, scmc.PSI_N, ((0.0, 1.8), (1.8, 0.0))),
    (scmc.E6, scmc.PSI_N, ((-0.2, 1.8), (1.8, 0.0))),
    (scmc.E4, scmc.PSI_EXP_NEG_INV, ((_GC * 0.6, 0.5), (0.5, _GC * 0.6)))])
def test_slab_pipelined_moment_pass_single_step(stencil, psi, g):
    """An FP32 lattice whose moment field (288 MB) exceeds the slab threshold
    (264 MiB in FP32) runs the moment two-pass in z-slabs (24 of 8-9 planes),
    pass 2 of each slab beside pass 1 of the slab after next in one launch.
    One step from a droplet against the oracle
    site by site, on every plane (so on both sides of every slab boundary),
    on the interface and in the bulk.  The asymmetric coupling g_AA = -0.2
    holds a B-rich droplet, as the 256^3 workload does."""
    nz, ny, nx, R0 = 208, 240, 240, 30.0
    if g[0][0] == -0.2:
        nA, nB = inputs.droplet(nx, ny, nz, R=R0, a_rich=False, bulk=inputs.FLAT_GUESS[-0.2])
    else:
        nA, nB = inputs.droplet(nx, ny, nz, R=R0)
    sim = scmc.Sim(scmc.problem(scmc.D3Q19, stencil, (nz, ny, nx), g=g, psi_self=psi,
                                storage=scmc.F32))
    sim.scmc_set_density(nA, nB)
    sim.scmc_step(1)
    f1, _ = sim.scmc_get_populations()
    sim.close()
    o = O.Oracle(3, stencil, (nz, ny, nx), g=g,
                 psi_self=O.PSI_EXP if psi == scmc.PSI_EXP_NEG_INV else O.PSI_N)
    o.set_density(nA, nB)
    xi, _ = scmc.velocities(scmc.D3Q19)
    perm = _perm(scmc.D3Q19, 3)
    sites = []
    for z in range(nz):
        dz = abs(z - nz // 2)
        rxy = np.sqrt(max(R0 * R0 - dz * dz, 0.0))
        sites += [(z, ny // 2, int(nx // 2 + rxy)), (z, ny // 2 + int(rxy), nx // 2), (z, 0, 0)]
    worst = 0.0
    for (z, y, x) in sites:
        want = o.collide_site((z * ny + y) * nx + x)[:, perm]
        got = np.array([[f1[J, i, (z + xi[i, 2]) % nz, (y + xi[i, 1]) % ny, (x + xi[i, 0]) % nx]
                         for i in range(19)] for J in range(2)])
        worst = max(worst, np.abs(got - want).max())
    assert worst < 1e-6, worst


def test_nt_all_pass1_single_step_graph_and_batch():
    """A lattice whose moment field (88 MB) is past the size from which pass 1
    loads every population non-temporally, and below the slab threshold: one
    step against the oracle site by site on every plane; 7 steps in graphs of
    3 and in a batch (graphs of 3) beside a small member, whose chunk keeps the
    default pass 1, give the bits of direct launches."""
    nz, ny, nx, R0 = 144, 160, 160, 28.0
    g = ((0.0, 1.8), (1.8, 0.0))
    nA, nB = inputs.droplet(nx, ny, nz, R=R0)
    p = scmc.problem(scmc.D3Q19, scmc.E6, (nz, ny, nx), g=g, storage=scmc.F32,
                     kernel=scmc.KERNEL_TWO_PASS_MOM)
    sim = scmc.Sim(p)
    sim.scmc_set_density(nA, nB)
    sim.scmc_step(1)
    f1, _ = sim.scmc_get_populations()
    sim.scmc_step(6)
    direct = sim.scmc_get_fields()
    sim.close()
    o = O.Oracle(3, 6, (nz, ny, nx), g=g)
    o.set_density(nA, nB)
    xi, _ = scmc.velocities(scmc.D3Q19)
    perm = _perm(scmc.D3Q19, 3)
    worst = 0.0
    for z in range(nz):
        dz = abs(z - nz // 2)
        rxy = np.sqrt(max(R0 * R0 - dz * dz, 0.0))
        for (y, x) in ((ny // 2, int(nx // 2 + rxy)), (ny // 2 + int(rxy), nx // 2), (0, 0)):
            want = o.collide_site((z * ny + y) * nx + x)[:, perm]
            got = np.array([[f1[J, i, (z + xi[i, 2]) % nz, (y + xi[i, 1]) % ny,
                                (x + xi[i, 0]) % nx] for i in range(19)] for J in range(2)])
            worst = max(worst, np.abs(got - want).max())
    assert worst < 1e-6, worst
    del f1, o
    gs = scmc.Sim(p)
    gs.scmc_set_graph_steps(3)
    gs.scmc_set_density(nA, nB)
    gs.scmc_step(7)
    assert np.array_equal(gs.scmc_get_fields(), direct)
    gs.close()
    q = scmc.problem(scmc.D3Q19, scmc.E6, (24, 28, 32), g=g, storage=scmc.F32,
                     kernel=scmc.KERNEL_TWO_PASS_MOM)
    bt = scmc.Batch([p, q])
    bt.scmc_batch_set_graph_steps(3)
    bt.scmc_batch_set_density(0, nA, nB)
    bt.scmc_batch_set_density(1, *inputs.droplet(32, 28, 24, R=6.0))
    bt.scmc_batch_step(7)
    assert np.array_equal(bt.scmc_batch_get_fields(0), direct)
    bt.close()


def test_slab_pipelined_asymmetric_droplet_matches_oracle():
    """The 256^3 workload's arithmetic (D3Q19 / E6, psi = n, g_AA = -0.2,
    B-rich droplet, FP32) in its slab schedule on a 208 x 240 x 240 box, 200
    steps (in graphs of 8) against the oracle: every concentration, and
    Delta P, C_d and the pressure-tensor line.  FP32 rounding over 200
    steps of a relaxing droplet: 1e-5 in n, 1e-4 relative in the pressures."""
    nz, ny, nx, R0, steps = 208, 240, 240, 30.0, 200
    g = ((-0.2, 1.8), (1.8, 0.0))
    nA, nB = inputs.droplet(nx, ny, nz, R=R0, a_rich=False, bulk=inputs.FLAT_GUESS[-0.2])
    sim = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, (nz, ny, nx), g=g, storage=scmc.F32))
    sim.scmc_set_graph_steps(8)
    sim.scmc_set_density(nA, nB)
    sim.scmc_step(steps)
    n = sim.scmc_get_fields()
    ob = sim.scmc_observables(scmc.OBS_DROPLET, R0)
    sim.close()
    o = O.Oracle(3, 6, (nz, ny, nx), g=g)
    o.set_density(nA, nB)
    o.run(steps)
    # the line observables of a non-cubic box run along +x from the centre
    # node (nz/2, ny/2, nx/2) out to nx/2
    oo = o.droplet_observables(R0)
    dn = np.abs(n - o.density()).max()
    print(f"max |dn| {dn:.3g}, dP {ob['dP']:.9g} ({oo['dP']:.9g}), C_d {ob['C_d']:.9g} "
          f"({oo['C_d']:.9g})", flush=True)
    assert dn < 1e-5
    assert abs(ob["dP"] - oo["dP"]) < 1e-4 * abs(oo["dP"])
    assert abs(ob["C_d"] - oo["C_d"]) < 1e-4 * abs(oo["C_d"])
    assert np.abs(ob["PT"] - oo["PT"]).max() < 1e-4 * np.abs(oo["PT"]).max()


def test_slab_pipelined_moment_pass_graph_and_fused():
    """The slab schedule in captured graphs equals direct launches bit for bit,
    and 20 steps agree with the fused moment-ring design (one launch per step,
    no slabs) to FP32 rounding."""
    nz, ny, nx, R0 = 208, 240, 240, 30.0
    nA, nB = inputs.droplet(nx, ny, nz, R=R0)
    runs = {}
    for name, kernel, tile, graph in (("direct", scmc.KERNEL_AUTO, (0, 0, 0), 0),
                                      ("graph", scmc.KERNEL_AUTO, (0, 0, 0), 3),
                                      ("fused", scmc.KERNEL_FUSED_MOM, (64, 8, 16), 0)):
        print(name, flush=True)
        sim = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, (nz, ny, nx), storage=scmc.F32,
                                    kernel=kernel, tile=tile))
        sim.scmc_set_graph_steps(graph)
        sim.scmc_set_density(nA, nB)
        sim.scmc_step(20)
        runs[name] = sim.scmc_get_fields()
        sim.close()
    assert np.array_equal(runs["direct"], runs["graph"])
    assert np.abs(runs["direct"] - runs["fused"]).max() < 1e-5


@pytest.mark.parametrize("kernel,tile", [
    (scmc.KERNEL_FUSED, (128, 4, 8)), (scmc.KERNEL_FUSED, (32, 16, 16)),
    (scmc.KERNEL_FUSED, (64, 4, 32)), (scmc.KERNEL_FUSED_REPULL, (64, 8, 16)),
    (scmc.KERNEL_FUSED_PIPE, (32, 8, 16)), (scmc.KERNEL_FUSED_PIPE, (64, 8, 8)),
    (scmc.KERNEL_FUSED_MOM, (64, 8, 16)), (scmc.KERNEL_FUSED_MOM, (128, 8, 8)),
    (scmc.KERNEL_FUSED_MOM, (64, 16, 32)), (scmc.KERNEL_FUSED_MOM, (32, 8, 8)),
    (scmc.KERNEL_FUSED_MOM_PIPE, (32, 8, 16)), (scmc.KERNEL_FUSED_MOM_PIPE, (64, 8, 8)),
    (scmc.KERNEL_TWO_PASS_MOM, (64, 8, 8))])
@pytest.mark.parametrize("stencil", [scmc.E4, scmc.E6])
def test_fused_designs_match_two_pass(kernel, tile, stencil):
    """Every fused design and tile (ragged x, y and z chunks included) gives
    the two-pass result to FP32 roundoff."""
    shape = (21, 22, 150) if tile[0] == 128 else (19, 37, 70)
    if kernel == scmc.KERNEL_FUSED_PIPE and stencil == scmc.E6 and tile[1] == 8 and tile[0] == 64:
        pytest.skip("64x8 halo does not fit one node per thread for E6")
    nA, nB = _random_state(shape, 31)
    g = ((-0.1, 1.4), (1.4, 0.05))
    ref = scmc.Sim(scmc.problem(scmc.D3Q19, stencil, shape, g=g, storage=scmc.F32,
                                kernel=scmc.KERNEL_TWO_PASS))
    ref.scmc_set_density(nA, nB)
    ref.scmc_step(12)
    fr, _ = ref.scmc_get_populations()
    s = scmc.Sim(scmc.problem(scmc.D3Q19, stencil, shape, g=g, storage=scmc.F32,
                              kernel=kernel, tile=tile))
    assert s.scmc_config() == (kernel, tile)   # TWO_PASS_MOM + tile: LDS-staged pass 2
    s.scmc_set_density(nA, nB)
    s.scmc_step(12)
    f, _ = s.scmc_get_populations()
    assert np.isfinite(f).all()
    assert np.abs(f - fr).max() < 2e-6


def test_autotune_picks_a_working_design(tmp_path):
    shape = (40, 48, 64)
    nA, nB = inputs.droplet(64, 48, 40, R=8.0)
    cache = str(tmp_path / "tune.txt")
    s = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, storage=scmc.F32))
    tile = s.scmc_autotune(cache)
    kernel, t2 = s.scmc_config()
    assert t2 == tile and kernel in (scmc.KERNEL_FUSED, scmc.KERNEL_FUSED_REPULL,
                                     scmc.KERNEL_FUSED_PIPE, scmc.KERNEL_FUSED_MOM,
                                     scmc.KERNEL_FUSED_MOM_PIPE, scmc.KERNEL_TWO_PASS_MOM)
    assert open(cache).read().count("->") == 1
    with pytest.raises(scmc.ScmcError):   # the tuner's scratch state is not kept
        s.scmc_step(1)
    s.scmc_set_density(nA, nB)
    s.scmc_step(20)
    ref = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, storage=scmc.F32,
                                kernel=scmc.KERNEL_TWO_PASS))
    ref.scmc_set_density(nA, nB)
    ref.scmc_step(20)
    assert np.abs(s.scmc_get_fields() - ref.scmc_get_fields()).max() < 1e-5
    # a second tuner call reads the cache
    s2 = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, storage=scmc.F32))
    assert s2.scmc_autotune(cache) == tile
    assert open(cache).read().count("->") == 1


def test_batch_autotune_and_graph():
    members = [(48, 8.0, True), (56, 10.0, False)]
    ps = [scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), storage=scmc.F32) for L, _, _ in members]
    inits = [inputs.droplet(L, L, L, R=R0, a_rich=a) for L, R0, a in members]
    b = scmc.Batch(ps)
    tile = b.scmc_batch_autotune(None)
    assert b.scmc_batch_config()[0] == tile
    for i, (nA, nB) in enumerate(inits):
        b.scmc_batch_set_density(i, nA, nB)
    b.scmc_batch_set_graph_steps(4)
    b.scmc_batch_step(13)
    for i, (nA, nB) in enumerate(inits):
        s = scmc.Sim(ps[i])
        s.scmc_set_density(nA, nB)
        s.scmc_step(13)
        assert np.abs(b.scmc_batch_get_fields(i) - s.scmc_get_fields()).max() < 1e-5


@pytest.mark.parametrize("lattice,stencil,gaa,lx", [
    (scmc.D3Q19, scmc.E6, 0.0, 32), (scmc.D2Q9, scmc.E8, 0.0, 48),
    (scmc.D2Q9, scmc.E4, -0.2, 64)])
def test_flat_equilibrium_matches_oracle(lattice, stencil, gaa, lx):
    """Stage one of the two-stage initialisation: the GPU flat-interface run
    (FP64 storage) and the oracle's reach the same bulk concentrations after
    the same number of steps."""
    dim = 2 if lattice == scmc.D2Q9 else 3
    g = ((gaa, 1.8), (1.8, 0.0))
    guess = inputs.FLAT_GUESS[gaa]
    want, wsteps = O.flat_equilibrium(dim, stencil, g, lx=lx, guess=guess, tol=1e-12)
    p = scmc.problem(lattice, stencil, (lx, lx, lx)[:dim], g=g, storage=scmc.F64)
    got, steps = scmc.scmc_flat_equilibrium(p, lx=lx, guess=guess, tol=1e-12)
    # FP64 on both sides: the same stopping chunk and the same values, unless
    # roundoff moves the stop by one chunk (then both sit within the slow
    # mode's tail, well under 1e-10, of the common fixed point)
    err = np.abs(np.array(got) - np.array(want)).max()
    if steps == wsteps:
        # FP64 roundoff, at most a few ulp per step, accumulated over the run
        assert err < 4 * 2.0 ** -53 * steps, err
    else:
        assert abs(steps - wsteps) == 2048 and err < 1e-10, (steps, wsteps, err)


@pytest.mark.parametrize("storage,mant", [(scmc.BF16_OFF, 8), (scmc.F16_OFF, 11)])
def test_stochastic_rounding_single_step(storage, mant):
    """One step with stochastic rounding of the FP16 / BF16 offsets against
    the same step in FP32 from the same (decoded) state: every stored value is
    one of the two neighbours of the exact one, the rounding is unbiased on
    average (where nearest-even rounding keeps a half-ulp spread), and the
    stream is reproducible for a seed and differs between seeds."""
    shape = (20, 24, 32)
    nA, nB = inputs.droplet(32, 24, 20, R=6.0)
    g = ((-0.2, 1.8), (1.8, 0.0))

    def run(seed, rounding=scmc.ROUND_STOCHASTIC):
        s = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, g=g, storage=storage,
                                  rounding=rounding, seed=seed))
        s.scmc_set_density(nA, nB)
        f0, _ = s.scmc_get_populations()
        s.scmc_step(1)
        f1, _ = s.scmc_get_populations()
        s.close()
        return f0, f1

    f0, f1 = run(7)
    _, f1b = run(7)
    _, f1c = run(8)
    _, f1n = run(7, scmc.ROUND_NEAREST)
    assert np.array_equal(f1, f1b)
    assert not np.array_equal(f1, f1c)
    ref = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, g=g, storage=scmc.F32))
    ref.scmc_set_populations(f0, 0)
    ref.scmc_step(1)
    fr, _ = ref.scmc_get_populations()
    xi, w = scmc.velocities(scmc.D3Q19)
    h = np.abs(fr - (np.array(w)[None, :, None, None, None] * 0.52))  # |offset|, n0 = 0.52
    ulp = 2.0 ** (np.floor(np.log2(np.maximum(h, 1e-30))) - (mant - 1))
    big = h > 1e-3   # normal range of both formats, away from zero offsets
    # the rest population closes the mass balance of all 2Q inputs, whose
    # host-decoded (reference) and device-decoded values differ in the last
    # FP32 bit: compare the moving populations, which depend on n_J and u only
    big[:, 0] = False
    e_sr = ((f1 - fr) / ulp)[big]
    e_rn = ((f1n - fr) / ulp)[big]
    # the FP32 reference itself carries up to 2^-24 |f| of rounding, which is
    # up to 2^-8 of an FP16 ulp at the smallest offsets kept here
    slack = (2.0 ** -23 * np.abs(fr) / ulp)[big]
    assert (np.abs(e_sr) <= 1.0 + slack).all()
    assert (np.abs(e_rn) <= 0.5 + slack).all()
    assert abs(e_sr.mean()) < 0.01
    # really rounds up and down, not to nearest: for a fraction f of an ulp the
    # expected |error| is 2 f (1 - f) >= min(f, 1 - f), the nearest-even error
    assert np.abs(e_sr).mean() > np.abs(e_rn).mean()
    assert (f1 != f1n).mean() > 0.05


def test_autotune_cache_respects_rounding(tmp_path):
    """A cached choice made for nearest-even rounding (possibly a fused
    design) is not reused for stochastic rounding, which runs two-pass only."""
    cache = str(tmp_path / "tune.txt")
    shape = (24, 32, 40)
    s = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, storage=scmc.BF16_OFF))
    s.scmc_autotune(cache)
    s2 = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, storage=scmc.BF16_OFF,
                               rounding=scmc.ROUND_STOCHASTIC, seed=3))
    s2.scmc_autotune(cache)
    assert s2.scmc_config()[0] == scmc.KERNEL_TWO_PASS_MOM


def test_convergence_check_matches_oracle():
    """The Sec. 4 monitor on a 24^3 E6 droplet (FP64 storage): no comparison
    on the first call; after 64 steps the relative change of Delta P, the
    velocity criterion du and the droplet centre against the oracle's own
    run of the same steps."""
    L, R0 = 24, 6.0
    nA, nB = inputs.droplet(L, L, L, R=R0)
    s = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), storage=scmc.F64))
    s.scmc_set_density(nA, nB)
    s.scmc_step(64)   # the symmetric start has Delta P = 0: begin later
    c0 = s.scmc_convergence_check(R0)
    assert np.isnan(c0["du"]) and np.isnan(c0["dP_change"]) and not c0["converged"]
    s.scmc_step(64)
    c1 = s.scmc_convergence_check(R0)
    o = O.Oracle(3, 6, (L, L, L))
    o.set_density(nA, nB)
    o.run(64)
    u0, d0 = o.velocity(), o.droplet_observables(R0)["dP"]
    o.run(64)
    u1, d1 = o.velocity(), o.droplet_observables(R0)["dP"]
    com, rich = O.excess_com(o.density(), (L, L, L))
    assert c1["rich"] == rich and c1["step"] == 128 and c1["prev_step"] == 64
    assert abs(c1["du"] - O.delta_u(u1, u0)) < 1e-10 * O.delta_u(u1, u0)
    want = abs(d1 - d0) / abs(d0)
    assert abs(c1["dP_change"] - want) < 1e-9 * want
    assert np.abs(c1["com"] - com).max() < 1e-10
    # (while pressure waves cross the box the far-field excess is not zero,
    # and with even L the cell is one node short of symmetric: the centre is
    # off c by a few 1e-3 here, in the oracle as on the GPU)
    assert abs(c1["com_offset"] - np.abs(com - L // 2).max()) < 1e-10
    s.close()


def test_run_to_convergence_stops_on_criterion():
    """A 32^3 droplet between flat-interface bulk values runs until Delta P
    changes by less than the tolerance over dt; a state set afresh forgets
    the previous check."""
    L, R0 = 32, 8.0
    p = scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), storage=scmc.F32)
    bulk, _ = scmc.scmc_flat_equilibrium(
        scmc.problem(scmc.D3Q19, scmc.E6, (L, L, L), storage=scmc.F64), lx=32,
        guess=inputs.FLAT_GUESS[0.0], tol=1e-10)
    s = scmc.Sim(p)
    s.scmc_set_density(*inputs.droplet(L, L, L, R=R0, bulk=bulk))
    c = s.scmc_run_to_convergence(R0, dt=512, max_steps=40960, tol_dP=1e-4, tol_du=1e-12)
    assert c["converged"] and c["dP_change"] < 1e-4
    assert c["step"] % 512 == 0 and c["step"] - c["prev_step"] == 512
    assert c["com_offset"] < 1e-3
    s.scmc_set_density(*inputs.droplet(L, L, L, R=R0, bulk=bulk))
    assert np.isnan(s.scmc_convergence_check(R0)["du"])
    s.close()


@pytest.mark.parametrize("tile", [(0, 0, 0), (64, 8, 8)])
def test_stochastic_rounding_graph_replay(tile):
    """The rounding stream advances with the device step counter, so graph
    replays (several runs of k steps, with odd remainders in between) give
    the same bits as direct launches, and a checkpoint resumed at its step
    continues the same stream."""
    shape = (12, 20, 36)
    nA, nB = inputs.droplet(36, 20, 12, R=4.0)
    p = scmc.problem(scmc.D3Q19, scmc.E6, shape, storage=scmc.BF16_OFF,
                     kernel=scmc.KERNEL_TWO_PASS_MOM, tile=tile,
                     rounding=scmc.ROUND_STOCHASTIC, seed=99)
    a = scmc.Sim(p)
    a.scmc_set_density(nA, nB)
    a.scmc_step(23)
    fa, _ = a.scmc_get_populations()
    b = scmc.Sim(p)
    b.scmc_set_graph_steps(5)
    b.scmc_set_density(nA, nB)
    for k in (7, 11, 5):
        b.scmc_step(k)
        b.scmc_synchronize()
    fb, st = b.scmc_get_populations()
    assert st == 23 and np.array_equal(fa, fb)
    c = scmc.Sim(p)
    c.scmc_set_density(nA, nB)
    c.scmc_step(10)
    f10, s10 = c.scmc_get_populations()
    d = scmc.Sim(p)
    d.scmc_set_populations(f10, s10)
    d.scmc_step(13)
    fd, _ = d.scmc_get_populations()
    assert np.array_equal(fa, fd)


def test_stochastic_rounding_batch():
    """A batch draws each member's rounding stream from its seed, the shared
    step counter and the member's offset in the batch buffers: member 0 (at
    offset 0) gives the bits of the same problem run alone, and member 1 does
    round stochastically (it differs from nearest-even rounding, by a few
    ulp of the offsets)."""
    shapes = [(16, 20, 24), (12, 16, 20)]
    ps = [scmc.problem(scmc.D3Q19, scmc.E6, sh, storage=scmc.F16_OFF,
                       kernel=scmc.KERNEL_TWO_PASS_MOM, rounding=scmc.ROUND_STOCHASTIC, seed=5)
          for sh in shapes]
    dens = [inputs.droplet(*sh[::-1], R=4.0) for sh in shapes]
    bt = scmc.Batch(ps)
    for i, d in enumerate(dens):
        bt.scmc_batch_set_density(i, *d)
    bt.scmc_batch_step(9)
    a = scmc.Sim(ps[0])
    a.scmc_set_density(*dens[0])
    a.scmc_step(9)
    fa, sa = a.scmc_get_populations()
    fb, sb = bt.scmc_batch_get_populations(0)
    assert sa == sb == 9 and np.array_equal(fa, fb)
    n = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shapes[1], storage=scmc.F16_OFF,
                              kernel=scmc.KERNEL_TWO_PASS_MOM))
    n.scmc_set_density(*dens[1])
    n.scmc_step(9)
    fn, _ = n.scmc_get_populations()
    f1, _ = bt.scmc_batch_get_populations(1)
    assert not np.array_equal(f1, fn) and np.abs(f1 - fn).max() < 1e-2
    for s in (a, n, bt):
        s.close()


@pytest.mark.parametrize("design", ["two_pass", "auto", "fused"])
@pytest.mark.parametrize("storage,tol", [(scmc.F64, 1e-12), (scmc.F32, 4e-6)])
@pytest.mark.parametrize("case", [2, 4, 5])
def test_unequal_tau_matches_oracle(case, storage, tol, design):
    """tau_A != tau_B with the 1/tau_J-weighted common velocity (the form that
    keeps the collision's momentum balance; the oracle pins it against a
    brute-force stepper that solves that balance): populations, the velocity
    field and the conserved momentum after 25 steps.  FP32 bound: tau_A = 0.7
    damps the non-conserved modes by only |1 - 1/tau_A| = 0.43 per step
    (0.25 at tau = 0.8), so rounding errors of the far-from-equilibrium
    random start persist longer; 4e-6 is about 64 u."""
    lattice, stencil, shape, psi, g, _ = CASES[case]
    kernel, tile = {"two_pass": (scmc.KERNEL_TWO_PASS, (0, 0, 0)),
                    "auto": (scmc.KERNEL_AUTO, (0, 0, 0)),
                    "fused": (scmc.KERNEL_FUSED, (64, 4, 16))}[design]
    if design == "fused" and (lattice == scmc.D2Q9 or storage == scmc.F64):
        pytest.skip("fused designs are D3Q19 with FP32-compute storage")
    print(f"case {case} storage {storage} design {design}", flush=True)
    tau = (0.7, 1.45)
    nA, nB = _random_state(shape, 300 + case)
    p = scmc.problem(lattice, stencil, shape, g=g, psi_self=psi, storage=storage,
                     kernel=kernel, tile=tile)
    p.tau[0], p.tau[1] = tau
    sim = scmc.Sim(p)
    sim.scmc_set_density(nA, nB)
    st0 = sim.scmc_stats_get()
    sim.scmc_step(25)
    f, _ = sim.scmc_get_populations()
    o = _oracle_for(lattice, stencil, shape, psi, g, tau)
    o.set_density(nA, nB)
    o.run(25)
    dim = 2 if lattice == scmc.D2Q9 else 3
    fo = o.f[:, _perm(lattice, dim)].reshape(f.shape)
    assert np.abs(f - fo).max() < tol
    n, u = sim.scmc_get_fields(velocity=True)
    assert np.abs(u - o.velocity()).max() < tol * 10
    st = sim.scmc_stats_get()
    sim.close()
    # the total momentum is conserved (to FP32 rounding with FP32 storage)
    mtol = 1e-11 if storage == scmc.F64 else 1e-4
    assert np.abs(st["momentum"] - st0["momentum"]).max() < mtol

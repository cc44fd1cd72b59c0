"""The allocation-free step (scmc_step_static) against the handle's step
(scmc_step) through the C ABI: two calls in a row on one GPU, the second with
a smaller lattice (and another design) than the first, so the second reuses
the static scratch array that the first left full.  The two entry points run
the same kernels on the same state, so the populations must agree bit for
bit; a lattice beyond the array is refused with SCMC_ENOSPACE."""
import numpy as np
import pytest

from paper_2112_02574_amd import inputs
from paper_2112_02574_amd import scmc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _run_static(p, nA, nB, steps):
    """Steps by the static entry point, ping-ponging between the workspace
    start (where scmc_set_density leaves the state) and a second buffer;
    returns the populations read back through the handle."""
    sim = scmc.Sim(p)
    sim.scmc_set_density(nA, nB)
    nbytes = scmc.state_bytes(p)
    a = sim.ws[:nbytes]
    b = torch.empty(nbytes, dtype=torch.uint8, device=sim.ws.device)
    for k in range(steps):
        src, dst = (a, b) if k % 2 == 0 else (b, a)
        scmc.scmc_step_static(p, src, dst, sim.stream)
    if steps % 2:
        with torch.cuda.stream(sim.stream):
            a.copy_(b)
    sim.scmc_synchronize()
    f, _ = sim.scmc_get_populations()
    sim.close()
    return f


def _run_handle(p, nA, nB, steps):
    sim = scmc.Sim(p)
    sim.scmc_set_density(nA, nB)
    sim.scmc_step(steps)
    f, st = sim.scmc_get_populations()
    sim.close()
    assert st == steps
    return f


def test_static_step_matches_handle_step():
    rng = np.random.default_rng(17)
    cases = [
        # 40 x 48 x 64 FP32 droplet, tau = 1: the moment two-pass (7 FP32
        # planes of scratch), three steps
        (scmc.problem(scmc.D3Q19, scmc.E6, (40, 48, 64), storage=scmc.F32),
         inputs.droplet(64, 48, 40, R=9.0), 3),
        # then a smaller FP64 lattice at tau = 0.8: the density two-pass
        (scmc.problem(scmc.D3Q19, scmc.E4, (12, 20, 36), tau=0.8, storage=scmc.F64,
                      g=((-0.1, 1.4), (1.4, 0.05)), kernel=scmc.KERNEL_TWO_PASS),
         (rng.uniform(0.3, 0.9, (12, 20, 36)), rng.uniform(0.3, 0.9, (12, 20, 36))), 2),
    ]
    for p, (nA, nB), steps in cases:
        print(f"static step: box {(p.nz, p.ny, p.nx)} storage {p.storage} tau {p.tau[0]} "
              f"steps {steps}", flush=True)
        fs = _run_static(p, nA, nB, steps)
        fh = _run_handle(p, nA, nB, steps)
        assert np.isfinite(fs).all()
        assert np.array_equal(fs, fh)


def test_static_step_refuses_lattices_beyond_the_array():
    p = scmc.problem(scmc.D3Q19, scmc.E6, (160, 160, 160), storage=scmc.F32)
    nbytes = scmc.state_bytes(p)
    buf = torch.empty(2 * nbytes, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(scmc.ScmcError) as e:
        scmc.scmc_step_static(p, buf[:nbytes], buf[nbytes:])
    assert e.value.status == -3
    assert "static array" in str(e.value)

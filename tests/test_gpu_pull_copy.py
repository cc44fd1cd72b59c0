"""The bandwidth-ceiling copy (scmc_pull_copy): the streaming half of the
step without arithmetic.  After an odd number of copies the second buffer
holds every population plane shifted by its velocity (periodic), i.e. the
state of one pure streaming step; checked against numpy rolls of the
populations the host put in."""
import numpy as np
import pytest

from paper_2112_02574_amd import inputs
from paper_2112_02574_amd import scmc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("storage", [scmc.F64, scmc.F32, scmc.F16_OFF])
def test_pull_copy_is_one_streaming_step(storage):
    shape = (6, 9, 14)
    nA, nB = inputs.droplet(14, 9, 6, R=3.0)
    sim = scmc.Sim(scmc.problem(scmc.D3Q19, scmc.E6, shape, storage=storage))
    sim.scmc_set_density(nA, nB)
    f0, _ = sim.scmc_get_populations()
    # buffer 0 holds g_i(x) = f_i(x + xi_i); one copy leaves g_i(x - xi_i) in
    # buffer 1, which read as a state of buffer 0 is f_i(x - xi_i)
    us = sim.scmc_pull_copy(1)
    assert us > 0
    with pytest.raises(scmc.ScmcError):
        sim.scmc_step(1)  # the state is unset after a copy
    raw = sim.ws.clone()
    sim.close()
    dt = {scmc.F64: np.float64, scmc.F32: np.float32, scmc.F16_OFF: np.uint16}[storage]
    N = int(np.prod(shape))
    pop = ((2 * 19 * N * np.dtype(dt).itemsize + 255) // 256) * 256
    b = raw.cpu().numpy()
    buf0 = b[:2 * 19 * N * np.dtype(dt).itemsize].view(dt).reshape(2, 19, *shape)
    buf1 = b[pop:pop + 2 * 19 * N * np.dtype(dt).itemsize].view(dt).reshape(2, 19, *shape)
    xi, _ = scmc.velocities(scmc.D3Q19)
    for i in range(19):
        want = np.roll(buf0[:, i], shift=(xi[i, 2], xi[i, 1], xi[i, 0]), axis=(1, 2, 3))
        np.testing.assert_array_equal(buf1[:, i], want)
    assert np.isfinite(f0).all()

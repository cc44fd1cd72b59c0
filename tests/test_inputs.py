"""The seeded input generators: splitmix64 against its published reference
outputs, and the initial profiles of Sec. 4 against their definitions."""
import numpy as np

from paper_2112_02574_amd import inputs


def test_splitmix64_reference_outputs():
    # first outputs of the reference splitmix64 for seed 0
    g = inputs.SplitMix64(0)
    assert [g.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                            0x06C45D188009454F]


def test_vectorised_stream_matches_scalar():
    g = inputs.SplitMix64(1)
    a = np.array([g.uniform() for _ in range(1000)])
    b = inputs.splitmix64_uniform_array(1, 1000)
    assert np.array_equal(a, b)
    assert 0.0 <= b.min() and b.max() < 1.0


def test_slab_noise_recipe():
    nA, nB = inputs.slab(64, 64, noise=1e-3, seed=1)
    clean_A, clean_B = inputs.slab(64, 64)
    u = inputs.splitmix64_uniform_array(1, 2 * 4096)
    assert np.array_equal(nA, clean_A + 1e-3 * (2 * u[:4096].reshape(64, 64) - 1))
    assert np.array_equal(nB, clean_B + 1e-3 * (2 * u[4096:].reshape(64, 64) - 1))
    assert clean_A[0, 16] == 1.0 and clean_A[0, 15] == 0.04 and clean_A[0, 48] == 0.04
    assert clean_B[0, 16] == 0.04 and clean_B[0, 47] == 0.04


def test_droplet_profile():
    nA, nB = inputs.droplet(33, 33, 33, R=8.0)
    assert nA.shape == (33, 33, 33)
    c = 16
    assert abs(nA[c, c, c] - (0.52 + 0.48 * np.tanh(8.0))) < 1e-15
    assert abs(nA[c, c, c + 8] - 0.52) < 1e-15  # r = R
    assert np.allclose(nA + nB, 1.04)
    a2, b2 = inputs.droplet(32, 32, R=8.0, a_rich=False)
    assert a2[16, 16] < 0.05 and b2[16, 16] > 0.99


def test_flat_strip_profile():
    nA, nB = inputs.flat_strip(127, 5, 5)
    x0 = 63.5
    assert nA[0, 0, int(x0)] > 0.99 and nA[0, 0, 0] < 0.05
    assert nB[0, 0, int(x0)] < 0.05 and nB[0, 0, 0] > 0.99


def test_batch_members_recipe():
    m = inputs.batch_members()
    assert len(m) == 48
    for i, d in enumerate(m):
        assert 8.0 <= d["R0"] < 40.0
        assert d["L"] % 8 == 0 and 48 <= d["L"] <= 160
        assert d["g"][0][0] == (0.0 if i % 2 == 0 else -0.2)
        assert d["a_rich"] == (i % 2 == 0 and (i // 2) % 2 == 0)
    assert m == inputs.batch_members()  # seeded
    # both droplet kinds occur among the symmetric members
    assert {d["a_rich"] for d in m[0::2]} == {True, False}

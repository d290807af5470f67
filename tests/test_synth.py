"""The seeded input generator: SplitMix64 outputs, ranges, exactness."""

import numpy as np

import synth


def test_mix64_matches_published_splitmix64_sequence():
    # splitmix64 seeded with 0 returns mix64(k * gamma) for k = 1, 2, 3
    # (Vigna's reference splitmix64.c); its first three outputs are these.
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        z = synth.mix64(np.array([g, g * np.uint64(2), g * np.uint64(3)], dtype=np.uint64))
    assert [int(x) for x in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_coefficients_are_exact_symmetric_fp32():
    c = synth.coef_table(8, 7, 6, 33)
    assert c.dtype == np.float32 and c.shape == (8, 7, 6, 33)
    assert np.all(np.abs(c) < 1)
    k = (c.astype(np.float64) * 2**24 + 2**24 - 1) / 2
    assert np.all(k == np.round(k))  # (2k+1-2^24)/2^24 exactly
    assert abs(c.mean()) < 0.02 and abs(c.astype(np.float64).var() - 1 / 3) < 0.01


def test_coefficient_subsets_match_full_table():
    full = synth.coef_table(5, 4, 3, 40, stream=3)
    cols = [0, 7, 39, 12]
    sub = synth.coef_table(5, 4, 3, 40, stream=3, splines=cols)
    np.testing.assert_array_equal(sub, full[..., cols])
    chunked = synth.coef_table(5, 4, 3, 40, stream=3, chunk=64)
    np.testing.assert_array_equal(chunked, full)


def test_positions_uniform_and_batches_differ():
    p0 = synth.positions(4096, batch=0)
    p1 = synth.positions(4096, batch=1)
    assert p0.shape == (3, 4096) and p0.dtype == np.float64
    assert p0.min() >= 0 and p0.max() < 1
    assert not np.array_equal(p0, p1)
    assert abs(p0.mean() - 0.5) < 0.02
    np.testing.assert_array_equal(p0, synth.positions(4096, batch=0))
    pb = synth.positions(100, box=(2.0, 3.0, 0.5))
    np.testing.assert_array_equal(pb[1], synth.positions(100)[1] * 3.0)


def test_torch_generator_matches_numpy_on_cpu():
    torch = __import__("pytest").importorskip("torch")
    a = synth.coef_table(6, 5, 7, 45, stream=6)
    b = synth.coef_table_torch(torch, 6, 5, 7, 45, device="cpu", stream=6, chunk=777)
    np.testing.assert_array_equal(a, b.numpy())

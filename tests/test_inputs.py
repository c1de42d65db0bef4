"""The seeded input generators shared by the oracle and the GPU path (CPU only)."""
import numpy as np

from henry_inputs import draw_theta, halton, philox4x32_10, qmc_theta


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 published with the generator (Salmon et al.,
    SC'11, Random123 distribution): counter, key -> output."""
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for ctr, key, want in kat:
        got = philox4x32_10(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(v) for v in got] == want


def test_theta_distributions_and_coupling():
    th = draw_theta(7, 20000)
    assert th.shape == (20000, 13)
    u = th[:, [0, 1, 2, 3, 12]]
    assert u.min() >= -1.0 and u.max() <= 1.0
    assert abs(u.mean()) < 0.02 and abs(u.var() - 1.0 / 3.0) < 0.01
    z = th[:, 4:12]
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    # counter-based: a sub-range is the same rows; levels and seeds are independent streams
    assert np.array_equal(draw_theta(7, 5, first_sample=100), th[100:105])
    assert not np.array_equal(draw_theta(7, 5, level=1), th[:5])
    assert not np.array_equal(draw_theta(8, 5), th[:5])


def test_halton_radical_inverses():
    """Radical inverses by hand: base 2 -> 1/2, 1/4, 3/4, 1/8, 5/8; base 3 -> 1/3, 2/3, 1/9,
    4/9, 7/9; base 5 -> 1/5, 2/5, 3/5, 4/5, 1/25."""
    h = halton(5)
    np.testing.assert_allclose(h[:, 0], [1 / 2, 1 / 4, 3 / 4, 1 / 8, 5 / 8], rtol=0, atol=1e-15)
    np.testing.assert_allclose(h[:, 1], [1 / 3, 2 / 3, 1 / 9, 4 / 9, 7 / 9], rtol=0, atol=1e-15)
    np.testing.assert_allclose(h[:, 2], [1 / 5, 2 / 5, 3 / 5, 4 / 5, 1 / 25], rtol=0, atol=1e-15)
    # points 0 .. b^k - 1 of base b are the b^k-point stratification {j / b^k}
    for b, k in ((2, 9), (3, 5), (5, 3)):
        d = (2, 3, 5).index(b)
        v = np.sort(halton(b ** k, start=0)[:, d])
        np.testing.assert_allclose(v, np.arange(b ** k) / b ** k, atol=1e-15)


def test_qmc_theta_layout():
    th = qmc_theta(600)
    assert th.shape == (600, 13)
    assert np.all(th[:, 2:12] == 0.0)
    np.testing.assert_allclose(th[:3, 0], [0.0, -0.5, 0.5])
    np.testing.assert_allclose(th[:3, 1], [-1 / 3, 1 / 3, -7 / 9])
    np.testing.assert_allclose(th[:3, 12], [-0.6, -0.2, 0.2])
    # low discrepancy: the means of the 600 points are within 1e-2 of 0
    assert np.abs(th[:, [0, 1, 12]].mean(axis=0)).max() < 1e-2

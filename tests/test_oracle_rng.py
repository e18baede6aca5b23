"""Pins for the counter-based probe generator of the oracle."""
import numpy as np

from oracle import rng


def test_splitmix64_published_stream_seed0():
    # First outputs of a SplitMix64 stream seeded with 0 (Steele, Lea & Flood
    # 2014; the widely reproduced reference values).
    assert rng.splitmix64_stream(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                            0x06C45D188009454F]


def test_splitmix64_published_stream_seed1234567():
    # Reference outputs of the public-domain splitmix64.c test vector.
    assert rng.splitmix64_stream(1234567, 5) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_rademacher_values_and_balance():
    e = rng.rademacher(7, rng.TAG_SLQ, 20000, 8)
    assert set(np.unique(e)) == {-1.0, 1.0}
    assert abs(e.mean()) < 5.0 / np.sqrt(e.size)
    # columns are distinct streams
    assert np.abs(e[:, 0] @ e[:, 1]) < 5.0 * np.sqrt(20000)


def test_rademacher_column_offset():
    a = rng.rademacher(3, rng.TAG_SLQ, 50, 10)
    b = rng.rademacher(3, rng.TAG_SLQ, 50, 4, col0=6)
    assert np.array_equal(a[:, 6:], b)


def test_gaussian_moments():
    g = rng.gaussian(11, rng.TAG_PRED_Z1, 200000, 2)
    x = g.ravel()
    assert abs(x.mean()) < 5.0 / np.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / x.size)
    # fourth moment of a standard normal is 3
    assert abs(np.mean(x ** 4) - 3.0) < 0.05
    # the two tags of Box-Muller are independent streams
    assert abs(np.corrcoef(g[:, 0], g[:, 1])[0, 1]) < 0.01

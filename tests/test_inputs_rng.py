"""Pins of the counter-based Gaussian generator that draws the test tensor of
Alg. 2 (its first step, randn) in the input module: Philox4x32-10 against the
known-answer vectors published with the generator (Salmon, Moraes, Dror and
Shaw, SC'11, Random123 distribution), the Box-Muller transform's logarithm,
sine, cosine and square root against numpy's, and the law of the stream."""
import numpy as np

from paper_2504_04989_amd import inputs


def test_philox4x32_10_known_answers():
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = inputs.philox4x32_10(np.array([ctr], dtype=np.uint64), key)[0]
        assert [int(x) for x in got] == list(want)


def test_transform_pieces_match_numpy():
    u = np.concatenate([np.linspace(2.0 ** -53, 1 - 2.0 ** -53, 200001), [0.5, 0.25, 0.75, 2.0 ** -52]])
    lg = inputs._log_unit(u)
    assert np.max(np.abs(lg - np.log(u)) / np.maximum(np.abs(np.log(u)), 1e-300)) < 1e-15
    c, s = inputs._sincos_2pi(u)
    assert np.max(np.abs(c - np.cos(2 * np.pi * u))) < 2e-15
    assert np.max(np.abs(s - np.sin(2 * np.pi * u))) < 2e-15
    x = np.concatenate([np.linspace(1e-16, 80.0, 100001), [1.0, 4.0, 2.0]])
    assert np.max(np.abs(inputs._sqrt_newton(x) - np.sqrt(x)) / np.sqrt(x)) <= 2.3e-16


def test_stream_is_standard_normal():
    z = inputs.omega_counter(2_000_000, 12345)
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(np.mean(z ** 3)) < 5 * np.sqrt(15 / n)
    assert abs(np.mean(z ** 4) - 3) < 5 * np.sqrt(96 / n)
    # P(|z| > 3) of the standard normal is 0.0026998
    p = np.mean(np.abs(z) > 3)
    assert abs(p - 0.0026998) < 5 * np.sqrt(0.0027 / n)
    # even and odd elements (cos and sin of one pair) are uncorrelated
    assert abs(np.mean(z[0::2] * z[1::2])) < 5 / np.sqrt(n / 2)


def test_stream_layout_and_seed_independence():
    a = inputs.omega(6, 4, 5, 3)
    assert np.array_equal(a.ravel(), inputs.omega_counter(120, 3))
    b = inputs.omega(6, 4, 5, 4)
    assert not np.allclose(a, b)
    assert np.array_equal(inputs.omega_counter(7, 9), inputs.omega_counter(8, 9)[:7])

"""Pins of the oracle's power spectrum (the discrete Fourier transform that
extracts the shedding frequency, Sec. 4.2), no GPU: agreement with
numpy.fft.rfft (a library routine for the same definition), the closed form
of a pure tone, Parseval's identity and invariance under circular shifts."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n", [1, 2, 7, 64, 1000, 1001])
def test_matches_numpy_fft(n):
    x = np.random.default_rng(n).standard_normal(n)
    p = oracle.dft_power(x)
    want = np.abs(np.fft.rfft(x)) ** 2
    assert p.shape == want.shape
    assert np.abs(p - want).max() <= 1e-12 * (np.abs(x).sum() ** 2)


@pytest.mark.parametrize("n,m", [(64, 5), (1000, 37), (999, 1), (4096, 2048)])
def test_pure_tone(n, m):
    a, phi = 0.3, 0.7
    j = np.arange(n)
    x = a * np.cos(2 * np.pi * m * j / n + phi)
    p = oracle.dft_power(x)
    amp = (n * a / 2) ** 2 * (4 if 2 * m == n else 1) * (np.cos(phi) ** 2 if 2 * m == n else 1)
    assert abs(p[m] - amp) <= 1e-10 * amp
    others = np.delete(p, m)
    assert others.max() <= 1e-16 * amp
    assert int(np.argmax(p[1:])) + 1 == m


def test_parseval_and_shift():
    n = 513
    x = np.random.default_rng(7).uniform(-1, 1, n) + 0.2
    p = oracle.dft_power(x)
    full = p[0] + 2 * p[1:].sum()          # n odd: bins 1..n//2 appear twice
    assert abs(full - n * np.dot(x, x)) <= 1e-12 * n * np.dot(x, x)
    q = oracle.dft_power(np.roll(x, 123))
    assert np.abs(p - q).max() <= 1e-12 * p.max()


def test_single_bin_equals_spectrum():
    x = np.random.default_rng(9).standard_normal(301)
    p = oracle.dft_power(x)
    bins = [0, 1, 17, 150]
    assert np.array_equal(oracle.dft_power_at(x, bins), p[bins])

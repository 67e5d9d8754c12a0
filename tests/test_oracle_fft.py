"""Pins for the oracle FFT: brute-force DFT, Parseval, on-bin tones."""
import numpy as np
import pytest

from oracle.fft import dft_bruteforce, factorize, fft, is_7smooth, next_7smooth


def _smooth_sizes(limit):
    return [n for n in range(1, limit + 1) if is_7smooth(n)]


@pytest.mark.parametrize("n", _smooth_sizes(64) + [96, 105, 210, 343, 384, 625, 1000, 1029, 2187, 4096])
def test_fft_matches_bruteforce(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = fft(x)
    ref = dft_bruteforce(x)
    err = np.max(np.abs(X - ref)) / max(np.max(np.abs(ref)), 1e-300)
    assert err <= 1e-12 * max(1.0, np.log2(n))


def test_parseval_and_inverse():
    rng = np.random.default_rng(7)
    n = 2 * 3 * 5 * 7 * 8
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = fft(x)
    assert abs(np.sum(np.abs(X) ** 2) - n * np.sum(np.abs(x) ** 2)) < 1e-9 * n * np.sum(np.abs(x) ** 2)
    # inverse through conjugation: conj(fft(conj(X))) = N x
    back = np.conj(fft(np.conj(X)))
    assert np.max(np.abs(back - n * x)) < 1e-9 * n


def test_on_bin_tone_is_delta():
    n = 360
    k0 = 17
    x = np.exp(2j * np.pi * k0 * np.arange(n) / n)
    X = fft(x)
    expect = np.zeros(n, complex)
    expect[k0] = n
    assert np.max(np.abs(X - expect)) < 1e-9


def test_non_smooth_rejected_and_next_smooth():
    with pytest.raises(ValueError):
        factorize(11 * 4)
    assert next_7smooth(2 * 172800) == 345600
    assert next_7smooth(1021) == 1024
    assert next_7smooth(11) == 12

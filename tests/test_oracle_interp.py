"""Pins for the oracle interpolation kernels: identity at integer positions,
exact recovery of periodic band-limited tones by the full Dirichlet kernel,
closed-form Lanczos values, and the band-edge power loss of truncated kernels
(paper Sec. V.B reports up to ~30 % near the band edge)."""
import math

import numpy as np
import pytest

from oracle.interp import (KERNEL_DIRICHLET, KERNEL_LANCZOS, dirichlet_weight,
                           interpolate, interpolate_full_dirichlet, lanczos_weight)


@pytest.mark.parametrize("kernel,W", [(KERNEL_LANCZOS, 8), (KERNEL_DIRICHLET, 16), (KERNEL_LANCZOS, 4)])
def test_integer_positions_are_identity(kernel, W):
    rng = np.random.default_rng(1)
    n = 200
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    u = np.arange(n, dtype=float)
    out = interpolate(z, u, kernel, W)
    assert np.max(np.abs(out - z)) < 1e-12


@pytest.mark.parametrize("n", [64, 65, 128, 255, 1024])
def test_full_dirichlet_recovers_periodic_tones(n):
    rng = np.random.default_rng(n)
    t = np.arange(n)
    ks = rng.integers(-(n // 2) + 1, n // 2, 3)
    amps = rng.standard_normal(3) + 1j * rng.standard_normal(3)

    def tone(x):
        return sum(a * np.exp(2j * np.pi * k * x / n) for a, k in zip(amps, ks))

    u = rng.uniform(0, n - 1, 40)
    if n > 512:
        u = u[:10]
    out = interpolate_full_dirichlet(tone(t), u)
    assert np.max(np.abs(out - tone(u))) < 1e-11


def test_lanczos_closed_form_values():
    W = 8
    for x in (0.5, 1.25, -2.5, 3.9):
        sx = math.sin(math.pi * x) / (math.pi * x)
        sw = math.sin(2 * math.pi * x / W) / (2 * math.pi * x / W)
        assert abs(lanczos_weight(x, W) - sx * sw) < 1e-15
    assert lanczos_weight(0.0, W) == 1.0
    assert lanczos_weight(4.0, W) == 0.0 and lanczos_weight(-4.5, W) == 0.0


def test_dirichlet_close_to_sinc_at_large_n():
    x = np.array([0.3, 1.7, -5.5, 7.9])
    n = 3456000
    sinc = np.sinc(x)
    assert np.max(np.abs(dirichlet_weight(x, n) - sinc)) < 1e-11
    assert abs(dirichlet_weight(0.0, n) - 1.0) == 0.0


def _tone_gain(kernel, W, frac_band, n=4096, m=2000, seed=0):
    """Power gain |interp|^2/|exact|^2 for a tone at frac_band * B (B = 1/dt)."""
    rng = np.random.default_rng(seed)
    t = np.arange(n)
    z = np.exp(2j * np.pi * frac_band * t)
    u = rng.uniform(64, n - 64, m)
    out = interpolate(z, u, kernel, W)
    return np.mean(np.abs(out) ** 2)


def test_band_edge_loss_table():
    """Truncated kernels pass the centre of the band and lose power towards
    its edges (paper Sec. V.B); the windowed kernel is flat in the central
    half, the truncated (rectangular-window) Dirichlet kernel ripples by a
    few per cent there, and every kernel loses at least 10 % near B/2."""
    lan8 = [_tone_gain(KERNEL_LANCZOS, 8, f) for f in (0.05, 0.1, 0.2)]
    assert max(abs(g - 1) for g in lan8) < 1e-2
    lan16 = [_tone_gain(KERNEL_LANCZOS, 16, f) for f in (0.05, 0.1, 0.2, 0.25)]
    assert max(abs(g - 1) for g in lan16) < 3e-3
    dir16 = [_tone_gain(KERNEL_DIRICHLET, 16, f) for f in (0.05, 0.1, 0.2, 0.25)]
    assert max(abs(g - 1) for g in dir16) < 8e-2
    for kernel, W in ((KERNEL_LANCZOS, 8), (KERNEL_DIRICHLET, 16), (KERNEL_LANCZOS, 16)):
        assert _tone_gain(kernel, W, 0.49) < 0.9
    # a wider window loses less at 0.3 B
    assert abs(_tone_gain(KERNEL_LANCZOS, 16, 0.3) - 1) < abs(_tone_gain(KERNEL_LANCZOS, 4, 0.3) - 1)

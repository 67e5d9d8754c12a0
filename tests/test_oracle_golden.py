"""Values the paper prints, stored in tests/golden/paper_values.json with
their citations, checked against the oracle."""
import json
import os

import numpy as np

from oracle import fstat as of
from oracle.ephemeris import velocity_over_c
from oracle.interp import KERNEL_LANCZOS
from paper_0912_4255_amd.synth import DET_H, Ephemeris, Segment

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_heterodyne_worked_example():
    """Analytic tones sampled at 1 kHz are heterodyned at 995 Hz
    (x_h = x exp(-2 pi i f_h t)) and decimated by 100 (the tones are exact
    in the 10 Hz band, so no filter is needed).  The paper's points (995 Hz ->
    DC, 990 -> -5, 1000 -> +5) land on DC and the Nyquist bin; interior tones
    following the same rule f -> f - f_h pin the sign."""
    g = GOLD["heterodyne_example"]
    fs, D, fh = g["original_rate_hz"], g["decimation"], g["f_het_hz"]
    n_out = 2000
    t = np.arange(n_out * D) / fs
    dt = D / fs
    assert abs(1.0 / dt - g["band_hz"]) < 1e-12
    points = [tuple(p) for p in g["maps_to_hz"]] + [(992.0, -3.0), (998.5, 3.5), (995.25, 0.25)]
    seg = Segment(n=n_out, dt=dt, t_start=0.0, f_het=fh)
    eph0 = Ephemeris(au_c=0.0, re_c=0.0)
    for f_in, f_out in points:
        x = np.exp(2j * np.pi * f_in * t)
        xh = (x * np.exp(-2j * np.pi * fh * t))[::D]
        rs = of.resample(xh, np.zeros((0, 2), np.int64), seg, 0.3, 0.2, eph0, DET_H,
                         KERNEL_LANCZOS, 8)
        rs["a"] = np.ones(n_out)
        rs["b"] = np.linspace(-1, 1, n_out)
        _, fa, _ = of.fstat_spectrum([rs], [DET_H], 0.0, 2 * n_out)
        s = int(of.signed_bin(int(np.argmax(np.abs(fa))), 2 * n_out))
        got = s / (2 * n_out * dt)
        if abs(f_out) == g["band_hz"] / 2:     # +-B/2 is one bin, labelled -B/2
            assert abs(got + g["band_hz"] / 2) < 1e-9
        else:
            assert abs(got - f_out) < 1e-9


def test_doppler_order_of_magnitude():
    g = GOLD["doppler"]
    tau = np.linspace(0, 3.2e7, 4001)
    v = np.linalg.norm(velocity_over_c(tau, Ephemeris(), DET_H), axis=-1)
    assert 0.5 * g["order_of_magnitude"] < v.max() < 2 * g["order_of_magnitude"]

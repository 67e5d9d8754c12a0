"""Pins of the time-domain front end of the oracle (paper Sec. III.A.1).

* no filter and no downsampling (L = 1, D = 1): the product with
  exp(-2 pi i f_h t), exactly;
* an in-band tone of the real series comes out as its positive-frequency
  half, heterodyned to f0 - f_h, with unit gain (the filter's sum) and the
  phase of output sample j at raw sample j D;
* a tone beyond the new Nyquist frequency (it would alias into the band) is
  suppressed to the filter's stop band;
* the paper's worked example: f_h = 995 Hz and D = 100 on a 1 kHz series
  (10 Hz output rate) keeps tones inside the flat part of the band (992 and
  998 Hz) and removes one at 1012 Hz that would alias onto -3 Hz."""
import numpy as np

from oracle import heterodyne as oh


def test_no_filter_is_the_heterodyne():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(500)
    dt, fh = 1.0 / 64.0, 10.3
    got = oh.heterodyne_decimate(x, dt, fh, D=1, K=0, beta=8.0, n_out=500)
    assert np.allclose(got, x * np.exp(-2j * np.pi * fh * np.arange(500) * dt), rtol=0, atol=1e-14)


def test_in_band_tone_unit_gain_and_phase():
    dt, D, K = 1.0 / 256.0, 32, 12
    fh = 100.0
    B = 1.0 / (D * dt)                                   # 8 Hz
    n = 256 * 120
    t = np.arange(n) * dt
    out_n = n // D
    tj = np.arange(out_n) * D * dt
    for f0, phi in ((fh + 0.31 * B, 0.4), (fh - 0.22 * B, 2.0), (fh, -1.0)):
        x = 3.0 * np.cos(2 * np.pi * f0 * t + phi)
        got = oh.heterodyne_decimate(x, dt, fh, D, K, 8.0, out_n)
        exp = 1.5 * np.exp(1j * (2 * np.pi * f0 * tj + phi)) * np.exp(-2j * np.pi * fh * tj)
        core = slice(2 * K, out_n - 2 * K)                  # away from the transients
        assert np.max(np.abs(got[core] - exp[core])) < 1e-3 * 1.5, f0


def test_tone_beyond_the_new_nyquist_frequency_is_suppressed():
    dt, D, K = 1.0 / 256.0, 32, 12
    fh = 100.0
    B = 1.0 / (D * dt)
    n = 256 * 60
    t = np.arange(n) * dt
    x = np.cos(2 * np.pi * (fh + 0.8 * B) * t)          # aliases to -0.2 B after downsampling
    got = oh.heterodyne_decimate(x, dt, fh, D, K, 8.0, n // D)
    assert np.max(np.abs(got[2 * K:-2 * K])) < 1e-3


def test_worked_example_990_to_1000_hz():
    dt, D = 1.0 / 1000.0, 100                            # 1 kHz raw, 10 Hz out
    fh = 995.0
    n = 1000 * 40
    t = np.arange(n) * dt
    keep = np.cos(2 * np.pi * 992.0 * t) + np.cos(2 * np.pi * 998.0 * t)
    drop = np.cos(2 * np.pi * 1012.0 * t)
    out_n = n // D
    tj = np.arange(out_n) * D * dt
    got = oh.heterodyne_decimate(keep + drop, dt, fh, D, 12, 8.0, out_n)
    exp = 0.5 * (np.exp(2j * np.pi * (992.0 - fh) * tj) + np.exp(2j * np.pi * (998.0 - fh) * tj))
    core = slice(24, out_n - 24)
    assert np.max(np.abs(got[core] - exp[core])) < 2e-3


def test_sampled_evaluation_equals_the_full_one():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(4000)
    full = oh.heterodyne_decimate(x, 1.0 / 128.0, 20.0, 16, 6, 7.0, 250)
    js = [0, 1, 77, 248, 249]
    assert np.allclose(oh.heterodyne_decimate_at(x, 1.0 / 128.0, 20.0, 16, 6, 7.0, js), full[js], rtol=0, atol=1e-12)

"""Pins of the SFT front end of the oracle (paper Sec. III.B).

* chunking and the running median against brute force and closed forms;
* the merge with the exact finite-N kernel and every term equals the DFT of
  the concatenated data (eqs. e1, dft1-dft3), for the chunk as it is and
  zero-padded to a 7-smooth number of SFTs;
* the large-N kernel of eq. e75 approaches the exact one as 1/N;
* an on-bin tone goes through the whole front end exactly (relabelling,
  inverse transform, eq. hetStartCorr across a gap, stitching);
* white noise comes out with unit power after the normalisation of eq.
  dimlessSFTs1.
SFTs are made here from raw series with numpy's FFT (test side only)."""
import numpy as np
import pytest

from oracle import sft as osft
from oracle.fft import next_7smooth


def make_sfts(x, N, starts, k_lo, K):
    """SFT bands (eq. e25) of the raw stretches x[s:s+N]."""
    return np.stack([np.fft.fft(x[s:s + N])[k_lo:k_lo + K] for s in starts])


def test_chunks_by_start_time():
    t = [0.0, 10.0, 20.0, 40.0, 50.0, 70.0]
    assert osft.chunks(t, 10.0) == [(0, 3), (3, 2), (5, 1)]
    assert osft.chunks([5.0], 10.0) == [(0, 1)]


def test_running_median_ramp_and_clamped_edges():
    K, w = 40, 7
    X = np.arange(K, dtype=np.float64)               # |X|^2 = k^2, increasing
    m = osft.running_median_power(X[None, :], w)[0]
    h = w // 2
    exp = np.clip(np.arange(K), h, K - 1 - h)        # window clamped inside the band
    assert np.array_equal(m, (exp ** 2).astype(np.float64))


def test_running_median_is_the_middle_order_statistic():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 25)) + 1j * rng.standard_normal((3, 25))
    w = 9
    m = osft.running_median_power(X, w)
    p = np.abs(X) ** 2
    for a in range(3):
        for k in range(25):
            lo = min(max(k - w // 2, 0), 25 - w)
            vals = [float(v) for v in p[a, lo:lo + w]]
            less = [v for v in vals if sum(u < v for u in vals) <= w // 2 and sum(u > v for u in vals) <= w // 2]
            assert m[a, k] in less


def test_normalised_noise_has_unit_power():
    rng = np.random.default_rng(2)
    P0 = 37.0
    X = np.sqrt(P0 / 2) * (rng.standard_normal((40, 2000)) + 1j * rng.standard_normal((40, 2000)))
    Xh = osft.normalise(X, 101)
    # median of Exp(P0) is P0 ln 2; the window estimate is unbiased to a few 1e-3
    assert abs(np.mean(np.abs(Xh) ** 2) - 1.0) < 0.02


@pytest.mark.parametrize("M,Mp", [(4, 4), (5, 6)])
def test_merge_with_exact_kernel_equals_long_dft(M, Mp):
    """Every term and the finite-N kernel: eq. dft2 is an identity, so the
    merge is the DFT of the chunk (zero-padded to Mp SFTs)."""
    rng = np.random.default_rng(3)
    N = 24
    x = rng.standard_normal(M * N) + 1j * rng.standard_normal(M * N)
    X = make_sfts(x, N, [a * N for a in range(M)], 0, N)
    b = np.arange(N * Mp)
    got = osft.merge_chunk(X, 0, Mp, b, dk=N, kernel=lambda bb, k, MM: osft.dirichlet_exact(bb, k, MM, N))
    ref = np.fft.fft(np.concatenate([x, np.zeros((Mp - M) * N)]))
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_large_n_kernel_approaches_exact_as_one_over_n():
    """Eq. e75 drops terms of order y/N: with the same truncation, the merge
    with the large-N kernel differs from the exact-kernel merge by ~1/N."""
    rng = np.random.default_rng(4)
    errs = []
    for N in (64, 256):
        M = 3
        x = rng.standard_normal(M * N) + 1j * rng.standard_normal(M * N)
        X = make_sfts(x, N, [a * N for a in range(M)], 0, N)
        b = np.arange(5 * M, N * M - 5 * M)
        a = osft.merge_chunk(X, 0, M, b, dk=4)
        e = osft.merge_chunk(X, 0, M, b, dk=4, kernel=lambda bb, k, MM: osft.dirichlet_exact(bb, k, MM, N))
        errs.append(np.max(np.abs(a - e)) / np.max(np.abs(e)))
    assert errs[1] < errs[0] / 3.0


def test_on_bin_tone_through_the_front_end():
    """A tone on an SFT bin, two chunks of 3 and 4 SFTs around one missing SFT:
    each SFT holds one nonzero in-band bin, the merge puts it on one long bin
    (all other bins cancel exactly, whatever the kernel), and the output is
    the heterodyned tone N / sqrt(B T_sft) (A/2) e^{i(2 pi f0 t + phi)} e^{-2 pi i f_h (t - t_s)}
    on both chunks, with the phase carried across the gap by eq. hetStartCorr.
    The analysis starts one output sample before the data, so that
    f_h (t_c - t_s) is not a whole number of cycles and the correction (and
    its sign) matters."""
    N, dt_raw = 256, 1.0 / 64.0
    T_sft = N * dt_raw                                  # 4 s, bins of 0.25 Hz
    slots = [0, 1, 2, 4, 5, 6, 7]                       # slot 3 missing
    f_het, band = 10.25, 2.0                            # f_h T_sft = 41, B T_sft = 8
    t_s = -1.0 / band
    k0 = 42                                             # f0 = 10.5 Hz
    f0, A, phi = k0 / T_sft, 3.0, 0.7
    t = np.arange(8 * N) * dt_raw                       # raw data from t = 0
    x = 0.5 * A * np.exp(1j * (2 * np.pi * f0 * t + phi))
    k_lo, K = 30, 24
    X = make_sfts(x, N, [s * N for s in slots], k_lo, K)
    t_sft = np.array([s * T_sft for s in slots])
    n_out = int(8 * T_sft * band) + 1
    got, gaps = osft.heterodyne_from_sfts(X, t_sft, T_sft, k_lo, t_s, f_het, band, n_out, dk=8,
                                          band_taper=0.25, edge_taper_s=0.0, normalise_sfts=False)
    tj = t_s + np.arange(n_out) / band
    exp = (N / np.sqrt(band * T_sft)) * 0.5 * A * np.exp(1j * (2 * np.pi * f0 * tj + phi)) \
        * np.exp(-2j * np.pi * f_het * (tj - t_s))
    gap = (1 + int(3 * T_sft * band), 1 + int(4 * T_sft * band))
    exp[0] = 0
    exp[gap[0]:gap[1]] = 0
    assert np.array_equal(gaps, np.array([(0, 1), gap]))
    assert np.max(np.abs(got - exp)) <= 1e-9 * np.max(np.abs(exp))


def test_padded_chunk_equals_band_limited_padded_data():
    """A chunk of 5 SFTs (not 7-smooth) is transformed on the grid of 6: with
    the exact kernel and every term, its series is the band-limited
    interpolation of the zero-padded chunk, computed here from the raw data."""
    rng = np.random.default_rng(5)
    N, M = 32, 5
    Mp = next_7smooth(M)
    x = rng.standard_normal(M * N) + 1j * rng.standard_normal(M * N)
    X = make_sfts(x, N, [a * N for a in range(M)], 0, N)
    band_bins, f_het_bins = 8, 10
    z, mp = osft.chunk_series(X, 0, band_bins, f_het_bins, dk=N, band_taper=0.0,
                              kernel=lambda bb, k, MM: osft.dirichlet_exact(bb, k, MM, N))
    assert mp == Mp
    n = band_bins * Mp
    F = np.fft.fft(np.concatenate([x, np.zeros((Mp - M) * N)]))
    q = np.arange(n) - n // 2
    Y = F[f_het_bins * Mp + q]
    j = np.arange(band_bins * M)
    ref = (np.exp(2j * np.pi * np.outer(j, q) / n) @ Y) / np.sqrt(n * M)
    assert np.max(np.abs(z - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_white_noise_comes_out_with_unit_power():
    """Normalised SFTs of white noise: E|x_h|^2 = mean of the squared band
    window (the scale reading), within the statistics of the sample."""
    rng = np.random.default_rng(6)
    N, dt_raw = 512, 1.0 / 64.0
    T_sft = N * dt_raw
    M = 8
    x = rng.standard_normal(M * N)                      # real raw noise
    f_het, band = 12.0, 4.0
    k_lo = int((f_het - band / 2) * T_sft) - 60
    K = int(band * T_sft) + 120
    X = make_sfts(x, N, [a * N for a in range(M)], k_lo, K)
    n_out = int(M * T_sft * band)
    r = 0.1
    z, gaps = osft.heterodyne_from_sfts(X, np.arange(M) * T_sft, T_sft, k_lo, 0.0, f_het, band, n_out,
                                        dk=8, median_window=51, band_taper=r, normalise_sfts=True)
    assert gaps.shape == (0, 2)
    w2 = np.mean(osft.tukey(int(band * T_sft) * M, r) ** 2)
    p = np.mean(np.abs(z[n_out // 8: -n_out // 8]) ** 2)
    assert abs(p / w2 - 1.0) < 0.08

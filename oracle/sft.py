"""From short Fourier transforms to the heterodyned, downsampled series
(oracle, FP64): the frequency-domain front end of paper Sec. III.B.

TEST INFRASTRUCTURE, like the rest of this package.

The steps, in the order of the summary at the end of Sec. III.B:

1. the input is a set of SFTs X_{alpha,k} = sum_j x_{alpha,j} e^{-2 pi i j k / N}
   (eq. e25) of consecutive stretches of N raw samples, of which a band of
   bins k_lo .. k_lo + K - 1 is kept;
2. normalisation (eq. dimlessSFTs1): X^_{alpha,k} = X_{alpha,k} / sqrt(S_{alpha,k})
   with S from a running median of |X|^2 over frequency;
3. contiguous SFTs (start times exactly T_sft apart) form chunks;
4. each chunk of M SFTs becomes one long-baseline transform (eqs. dft3, e9,
   e91): X_b = sum_alpha e^{-2 pi i b alpha / M} sum_{k = k*-dk}^{k*+dk} X^_{alpha,k} P_{b,k},
   k* = floor(b / M), with the large-N Dirichlet kernel of eq. e75,
   P_{b,k} = sin(y)/y - i (1 - cos y)/y, y = 2 pi (b/M - k);
5. the band around f_h is relabelled so that f_h is DC (Sec. III.B,
   "Heterodyning"), windowed with a Tukey window over frequency ("Downsampling
   and low-pass filtering") and inverse transformed: the chunk's samples at
   dt = 1/B from its own start t_c;
6. each chunk is moved to the common heterodyne reference t_s by the factor
   of eq. hetStartCorr, tapered at its edges with a Tukey window in time and
   written into the output series; gaps stay zero ("Gaps in the data").

Readings (where the paper leaves a choice; each is listed in the design
notes):

* Running median: window of w bins (odd), clamped inside the stored band at
  its edges so that every estimate uses w values; the median of |X|^2 is
  turned into the mean power by dividing by ln 2 (|X|^2 of Gaussian noise is
  exponentially distributed), S = median / ln 2, so normalised noise has
  E|X^|^2 = 1.
* Eqs. e9/e91 print the kernel as P_{alpha,k}; the derivation (eqs. dft2-dft3)
  gives P_{b,k}, which is used.  P = 1 at y = 0 (its limit).
* Sign of the heterodyne: as in the time-domain path, x_h = x e^{-2 pi i f_h (t - t_s)}.
  Relabelling bin f_h of a chunk as DC gives x e^{-2 pi i f_h (t - t_c)}, so the
  correction is e^{-2 pi i f_h (t_c - t_s)} (eq. hetStartCorr prints the
  opposite sign, matching its opposite heterodyne sign).
* f_h and the band B are whole numbers of SFT bins (f_h T_sft and B T_sft
  integers, B T_sft even), so that f_h is a bin of every chunk and the chunk's
  series starts on the output grid.
* Chunk length: the inverse transform has n = B T_sft M' points with M' the
  smallest 7-smooth number >= M (zero SFTs appended: the merge then runs on
  the M' grid); the first B T_sft M samples are the chunk.  With M 7-smooth
  this is the paper's transform as written.
* Scale: the inverse transform is divided by sqrt(n M), so that normalised
  white noise gives E|x_h|^2 = mean of the squared band window (1 for a
  rectangular band), the unit-variance convention of the time-domain path.
* Windows: a Tukey window over the band with a cosine taper over a fraction
  r of the band (r/2 at each edge), and a Tukey taper in time of tau seconds
  at each chunk edge (nothing when tau = 0).
"""
import numpy as np

from .fft import fft, next_7smooth


def running_median_power(X, w):
    """Running median of |X|^2 along the last axis over w bins (w odd),
    window clamped inside the band, FP64.  Returns an array like |X|^2."""
    p = np.abs(np.asarray(X, dtype=np.complex128)) ** 2
    K = p.shape[-1]
    if w < 1 or w % 2 == 0 or w > K:
        raise ValueError("window must be odd and at most the band")
    h = w // 2
    out = np.empty_like(p)
    for k in range(K):
        lo = min(max(k - h, 0), K - w)
        win = np.sort(p[..., lo:lo + w], axis=-1)
        out[..., k] = win[..., h]
    return out


def normalise(X, w):
    """Eq. dimlessSFTs1: X / sqrt(S), S = running median of |X|^2 / ln 2."""
    S = running_median_power(X, w) / np.log(2.0)
    return np.asarray(X, dtype=np.complex128) / np.sqrt(S)


def chunks(t_sft, T_sft):
    """Contiguous runs of SFTs: (first index, count) with start times exactly
    T_sft apart (step 3 of the summary)."""
    t = np.asarray(t_sft, dtype=np.float64)
    out = []
    a0 = 0
    for a in range(1, len(t) + 1):
        if a == len(t) or t[a] - t[a - 1] != T_sft:
            out.append((a0, a - a0))
            a0 = a
    return out


def dirichlet_large_n(b, k, M):
    """P_{b,k} of eq. e75 with y = 2 pi (b/M - k): sin(y)/y - i (1 - cos y)/y,
    1 at y = 0."""
    y = 2.0 * np.pi * (np.asarray(b, dtype=np.float64) / M - k)
    small = np.abs(y) < 1e-300
    ys = np.where(small, 1.0, y)
    P = np.sin(ys) / ys - 1j * (1.0 - np.cos(ys)) / ys
    return np.where(small, 1.0 + 0j, P)


def dirichlet_exact(b, k, M, N):
    """The exact finite sum (1/N) sum_{j<N} e^{-i y j / N} of eq. dft2 (before
    the large-N step), for the pins."""
    y = 2.0 * np.pi * (np.asarray(b, dtype=np.float64) / M - k)
    j = np.arange(N)
    return np.exp(-1j * np.multiply.outer(y, j) / N).sum(axis=-1) / N


def merge_chunk(Xh, k_lo, M_grid, b_values, dk, kernel=None):
    """Eq. e9/e91 for one chunk: X_b for the given long-baseline bins b.

    Xh: [M][K] normalised SFT bands (bins k_lo .. k_lo + K - 1) of the chunk's
    M SFTs, in time order.  M_grid: the M of the long transform (M' >= M;
    SFTs M .. M'-1 are zero).  Terms outside the stored band are absent.
    kernel(b, k, M): P_{b,k}; the large-N kernel by default."""
    kernel = kernel or dirichlet_large_n
    Xh = np.asarray(Xh, dtype=np.complex128)
    M, K = Xh.shape
    out = np.zeros(len(b_values), dtype=np.complex128)
    for i, b in enumerate(b_values):
        ks = b // M_grid
        k = np.arange(ks - dk, ks + dk + 1)
        ok = (k >= k_lo) & (k < k_lo + K)
        k = k[ok]
        P = kernel(b, k, M_grid)
        inner = Xh[:, k - k_lo] @ P                       # sum over k, per SFT
        alpha = np.arange(M)
        out[i] = np.sum(np.exp(-2j * np.pi * b * alpha / M_grid) * inner)
    return out


def tukey(n, r):
    """Tukey window of n points with a cosine taper over a fraction r."""
    x = (np.arange(n) + 0.5) / n
    w = np.ones(n)
    if r > 0:
        e = r / 2.0
        lo = x < e
        hi = x > 1.0 - e
        w[lo] = 0.5 * (1.0 - np.cos(np.pi * x[lo] / e))
        w[hi] = 0.5 * (1.0 - np.cos(np.pi * (1.0 - x[hi]) / e))
    return w


def chunk_series(Xh, k_lo, band_bins, f_het_bins, dk, band_taper, kernel=None):
    """Steps 4-5 for one chunk of M SFTs: the chunk's heterodyned series at
    dt = 1/B from its start, B T_sft M samples.

    band_bins: SFT bins in the output band (B T_sft, even); f_het_bins:
    f_h T_sft (integer).  Returns (series, M')."""
    M = Xh.shape[0]
    Mp = next_7smooth(M)
    n = band_bins * Mp
    q = np.arange(n) - n // 2                              # relabelled bins, ascending
    b = f_het_bins * Mp + q
    Xb = merge_chunk(Xh, k_lo, Mp, b, dk, kernel)
    Y = tukey(n, band_taper) * Xb
    # natural DFT order: relabelled bin q at index q mod n
    Yn = np.empty(n, dtype=np.complex128)
    Yn[q % n] = Y
    z = np.conj(fft(np.conj(Yn))) / np.sqrt(n * M)         # sum_q Y_q e^{+2 pi i q j / n}
    return z[:band_bins * M], Mp


def time_taper(n, n_edge):
    """Tukey taper in time: cosine rise over n_edge samples at each end."""
    w = np.ones(n)
    if n_edge > 0:
        e = min(n_edge, n // 2)
        x = (np.arange(e) + 0.5) / e
        r = 0.5 * (1.0 - np.cos(np.pi * x))
        w[:e] = r
        w[n - e:] = r[::-1]
    return w


def heterodyne_from_sfts(X, t_sft, T_sft, k_lo, t_start, f_het, band, n_out, dk=8, median_window=101,
                         band_taper=0.05, edge_taper_s=0.0, normalise_sfts=True, kernel=None):
    """The whole front end (steps 1-6): complex series x_h[n_out] at
    t_s + j / B and the gaps as half-open sample ranges.

    X: [n_sft][K] SFT bands (complex), t_sft: start times (s), T_sft: SFT
    length (s), k_lo: first stored bin, f_het: heterodyne frequency (Hz),
    band: B (Hz)."""
    X = np.asarray(X, dtype=np.complex128)
    sft_bins = int(round(band * T_sft))
    f_het_bins = int(round(f_het * T_sft))
    if abs(sft_bins - band * T_sft) > 1e-9 or sft_bins % 2 or abs(f_het_bins - f_het * T_sft) > 1e-9:
        raise ValueError("B T_sft must be an even integer and f_h T_sft an integer")
    Xh = normalise(X, median_window) if normalise_sfts else X
    dt = 1.0 / band
    x = np.zeros(n_out, dtype=np.complex128)
    covered = np.zeros(n_out, dtype=bool)
    n_edge = int(round(edge_taper_s / dt))
    for a0, M in chunks(t_sft, T_sft):
        z, _ = chunk_series(Xh[a0:a0 + M], k_lo, sft_bins, f_het_bins, dk, band_taper, kernel)
        t_c = float(t_sft[a0])
        z = z * np.exp(-2j * np.pi * f_het * (t_c - t_start))    # eq. hetStartCorr (sign per the reading)
        z = z * time_taper(len(z), n_edge)
        j0 = int(round((t_c - t_start) / dt))
        lo, hi = max(j0, 0), min(j0 + len(z), n_out)
        if lo < hi:
            x[lo:hi] = z[lo - j0:hi - j0]
            covered[lo:hi] = True
    gaps = []
    j = 0
    while j < n_out:
        if not covered[j]:
            e = j
            while e < n_out and not covered[e]:
                e += 1
            gaps.append((j, e))
            j = e
        else:
            j += 1
    return x, np.array(gaps, dtype=np.int64).reshape(-1, 2)

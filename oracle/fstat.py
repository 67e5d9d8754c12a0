"""Resampling, demodulation and the F-statistic (oracle, FP64).

Follows the seven-step procedure of paper Sec. III.A.2 in the paper's order:

1. start from the heterodyned, downsampled series x_h(t^k) (regular detector
   grid t^k = k dt from the segment start);
2. heterodyne correction on the detector grid, z = x_h exp(-2 pi i f_h t_m)
   (eqs. absorb, Fa3; sign per the heterodyne reading below);
3. detector times T^k of the regular SSB grid (eq. eq21, ``oracle.timing``);
4. interpolate z at T^k (``oracle.interp``);
5. a(t_b^k), b(t_b^k): evaluated analytically at T^k, which is the value the
   paper's "similar procedure" (interpolation of a and b) approximates;
6. F_a, F_b of eqs. eq19/eq20 with one FFT each after zero padding;
7. 2F from eq. eq6 with A, B, C, D of eqs. eq9/eq10.

Readings where the paper is silent or inconsistent (each is listed in the
design notes):

* Heterodyne sign: the worked example of Sec. III.A.1 (995 Hz moved to DC)
  and the bin relabelling of Sec. III.B need x_h = x exp(-2 pi i f_h t); eq.
  eq15 prints the opposite sign.  With this sign the correction is
  z = x_h exp(-2 pi i f_h t_m) and bin s sits at f_h + s df.
* Spindown phase sign: eqs. eq12/eq13/eq19/eq20 print exp(+i Phi_s), but
  eq. eq5 inserted into eqs. eq7/eq8 gives exp(-i Phi); exp(-i Phi_s) is used.
* Spindown phase (eq. eq4pt1): Phi_s = 2 pi sum_j f^(j) (T^{j+1}/(j+1)! + t_m T^j/j!)
  at T^k with t_m,k = t_b^k - T^k (eq. phi-s-explain); s = 1 by default, up to 3
  when a template carries (fdot, f^(2), f^(3)).
* dt_b/dt is taken as 1 (the paper drops the ~1e-4 Doppler Jacobian, eqs.
  eq11b/eq11c).
* Gaps: the input is zero-filled; A, B, C are sums over the SSB grid with the
  nearest-sample mask m~_k = m[floor(u_k + 1/2)] (0 outside the segment), so
  the noise mean of 2F stays 4 with gaps.
* Units: complex noise with E|n|^2 = sigma^2 per sample, S_h = 2 dt sigma^2;
  the T0 and dt factors of eqs. eq6/eq10 cancel and
  2F = (2/sigma^2) (B'|f_a|^2 + A'|f_b|^2 - 2 C' Re(f_a f_b^*)) / D'
  with the unnormalised sums f_a = sum_k a_k z~_k e^{-i Phi_s,k} e^{-2 pi i s k / N_fft}
  and A' = sum_k m~_k a_k^2 (and B', C' likewise).
* Several detectors (the paper is single-detector; cf. the whitened form of
  eq. LALDemodFstat): the integrands and A', B', C' are noise-weighted sums
  over detectors with weights 1/sigma_X^2, one FFT pair per template, and
  2F = 2 (B'|f_a|^2 + A'|f_b|^2 - 2 C' Re(f_a f_b^*)) / D'.
* Output bins: FFT index k holds signed bin s = k for k < N_fft/2 and
  k - N_fft otherwise (Sec. V.A); reported bands are ascending in s.
"""
import numpy as np

from .antenna import beam_ab
from .ephemeris import roemer_delay
from .fft import fft, next_7smooth
from .interp import interpolate
from .timing import invert_ssb_times

NFFT_TWICE = 0
NFFT_SMOOTH7 = 1
NFFT_SMOOTH7_256 = 2


def fft_length(n, policy):
    """Zero-padded length of step 5 (Sec. III.A.2): twice the series, the
    smallest even 7-smooth length >= 2n, or the smallest 7-smooth multiple
    of 256 that is >= 2n.  Even, so that a band reaching the Nyquist edges
    f_het +- 1/(2 dt) starts and ends on bins; an even 7-smooth m >= 2n is
    2j with j 7-smooth and j >= n, and a 7-smooth multiple of 256 is 256j
    with j 7-smooth and 256j >= 2n."""
    if policy == NFFT_TWICE:
        return 2 * n
    if policy == NFFT_SMOOTH7:
        return 2 * next_7smooth(n)
    if policy == NFFT_SMOOTH7_256:
        return 256 * next_7smooth(-(-2 * n // 256))
    raise ValueError("unknown FFT length policy")


def sample_mask(n, gaps):
    """m[j] = 0 inside the half-open gap ranges, 1 elsewhere."""
    m = np.ones(n, dtype=np.float64)
    for s, e in np.asarray(gaps, dtype=np.int64).reshape(-1, 2):
        m[s:e] = 0.0
    return m


def heterodyne_correction(x_h, seg, alpha, delta, eph, det, binary=None):
    """Step 2: z(t^k) = x_h(t^k) exp(-2 pi i f_h t_m(t^k)) on the detector grid
    (t_m replaced by the total delay d with a binary orbit)."""
    t = np.arange(seg.n, dtype=np.float64) * seg.dt
    tm = roemer_delay(seg.t_start + t, alpha, delta, eph, det)
    if binary is not None:
        from .binary import binary_delay, emission_time
        tm = tm - binary_delay(emission_time(seg.t_start + t + tm, binary), binary)
    return np.asarray(x_h, dtype=np.complex128) * np.exp(-2j * np.pi * seg.f_het * tm)


def resample(x_h, gaps, seg, alpha, delta, eph, det, kernel, W, binary=None):
    """Steps 2-5 for one detector and one sky position.

    Returns a dict with the detector times T^k, t_m,k, u_k = T^k/dt, the
    resampled series z~_k, the beam patterns a_k, b_k at T^k and the SSB
    mask m~_k."""
    z = heterodyne_correction(x_h, seg, alpha, delta, eph, det, binary)
    T, tm = invert_ssb_times(seg, alpha, delta, eph, det, binary=binary)
    u = T / seg.dt
    zt = interpolate(z, u, kernel, W)
    a, b = beam_ab(seg.t_start + T, alpha, delta, eph, det)
    m = sample_mask(seg.n, gaps)
    near = np.floor(u + 0.5).astype(np.int64)
    inside = (near >= 0) & (near < seg.n)
    m_ssb = np.where(inside, m[np.clip(near, 0, seg.n - 1)], 0.0)
    return {"T": T, "tm": tm, "u": u, "z": zt, "a": a, "b": b, "mask": m_ssb}


def antenna_sums(rs_list, dets):
    """Noise-weighted A', B', C' (eqs. eq9/eq10 as sums over the masked SSB grid)."""
    A = B = C = 0.0
    for rs, det in zip(rs_list, dets):
        w = 1.0 / det.sigma2
        A += w * np.sum(rs["mask"] * rs["a"] ** 2)
        B += w * np.sum(rs["mask"] * rs["b"] ** 2)
        C += w * np.sum(rs["mask"] * rs["a"] * rs["b"])
    return A, B, C


def spindown_phase(T, tm, fdot):
    """Phi_s,k of eq. eq4pt1 at T_k with t_m,k:
    2 pi sum_{j=1..s} f^(j) (T^{j+1} / (j+1)! + t_m T^j / j!).
    fdot is f^(1) (s = 1) or the sequence (f^(1), ..., f^(s))."""
    spins = np.atleast_1d(np.asarray(fdot, dtype=np.float64))
    cycles = 0.0
    Tj = T                        # T^j
    fact = 1.0                    # j!
    for j, fj in enumerate(spins, start=1):
        fact_next = fact * (j + 1)
        cycles = cycles + fj * (Tj * T / fact_next + tm * Tj / fact)
        Tj = Tj * T
        fact = fact_next
    return 2.0 * np.pi * cycles


def integrands(rs_list, dets, fdot):
    """y^a_k, y^b_k: the summands of eqs. eq19/eq20 before the Fourier kernel,
    noise-weighted over detectors."""
    ya = 0.0
    yb = 0.0
    for rs, det in zip(rs_list, dets):
        w = 1.0 / det.sigma2
        e = np.exp(-1j * spindown_phase(rs["T"], rs["tm"], fdot))
        ya = ya + w * rs["a"] * rs["z"] * e
        yb = yb + w * rs["b"] * rs["z"] * e
    return ya, yb


def twoF_from(fa, fb, A, B, C):
    """2F = 2 (B|fa|^2 + A|fb|^2 - 2 C Re(fa fb^*)) / D, D = AB - C^2 (eq. eq6)."""
    D = A * B - C * C
    return 2.0 * (B * np.abs(fa) ** 2 + A * np.abs(fb) ** 2
                  - 2.0 * C * np.real(fa * np.conj(fb))) / D


def signed_bin(k, n_fft):
    k = np.asarray(k)
    return np.where(k < n_fft / 2.0, k, k - n_fft)


def band_indices(n_fft, s_lo, n_out):
    """FFT indices of the ascending band s = s_lo .. s_lo + n_out - 1."""
    s = s_lo + np.arange(n_out)
    if n_out > 0 and (s[0] < -(n_fft // 2) or s[-1] > (n_fft + 1) // 2 - 1):
        raise ValueError("band outside the data band")
    return np.mod(s, n_fft)


def fstat_spectrum(rs_list, dets, fdot, n_fft):
    """Steps 6-7: 2F at every FFT index (FFT order), plus f_a, f_b."""
    A, B, C = antenna_sums(rs_list, dets)
    ya, yb = integrands(rs_list, dets, fdot)
    n = ya.shape[0]
    pa = np.zeros(n_fft, dtype=np.complex128)
    pb = np.zeros(n_fft, dtype=np.complex128)
    pa[:n] = ya
    pb[:n] = yb
    fa = fft(pa)
    fb = fft(pb)
    return twoF_from(fa, fb, A, B, C), fa, fb


def fstat_band(rs_list, dets, fdot, n_fft, s_lo, n_out):
    """2F over the ascending band of signed bins [s_lo, s_lo + n_out)."""
    F, _, _ = fstat_spectrum(rs_list, dets, fdot, n_fft)
    return F[band_indices(n_fft, s_lo, n_out)]


def fstat_bins(rs_list, dets, fdot, n_fft, signed_bins):
    """2F at selected signed bins by direct O(N) sums (each equals the FFT bin
    of the zero-padded integrands)."""
    A, B, C = antenna_sums(rs_list, dets)
    ya, yb = integrands(rs_list, dets, fdot)
    k = np.arange(ya.shape[0], dtype=np.float64)
    out = np.empty(len(signed_bins))
    for i, s in enumerate(signed_bins):
        e = np.exp(-2j * np.pi * np.mod(s * k, n_fft) / n_fft)
        out[i] = twoF_from(np.sum(ya * e), np.sum(yb * e), A, B, C)
    return out


def fstat_point(rs_list, dets, seg, f, fdot):
    """2F at a continuous frequency f: f_a(f) = sum_k y^a_k exp(-2 pi i (f - f_h) k dt).
    At f = f_h + s / (N_fft dt) this is FFT bin s."""
    A, B, C = antenna_sums(rs_list, dets)
    ya, yb = integrands(rs_list, dets, fdot)
    tb = np.arange(ya.shape[0], dtype=np.float64) * seg.dt
    e = np.exp(-2j * np.pi * (f - seg.f_het) * tb)
    return twoF_from(np.sum(ya * e), np.sum(yb * e), A, B, C)


def resample_all(xs, gaps_list, seg, alpha, delta, eph, dets, kernel, W, binary=None):
    return [resample(x, g, seg, alpha, delta, eph, d, kernel, W, binary=binary)
            for x, g, d in zip(xs, gaps_list, dets)]


def fstat_definition(xs, gaps_list, seg, freqs, fdot, alpha, delta, eph, dets):
    """Definition mode (eqs. eq7/eq8 as sums over the detector grid, no
    resampling): f_a(f) = sum_j m_j a(t_j) x_h[j] exp(-i[2 pi (f - f_h) t_j
    + 2 pi f t_m(t_j) + Phi_s(t_j)]) with Phi_s(t) = 2 pi fdot (t^2/2 + t_m t),
    A' = sum_j m_j a(t_j)^2, noise-weighted over detectors; 2F as eq. eq6."""
    freqs = np.atleast_1d(np.asarray(freqs, dtype=np.float64))
    t = np.arange(seg.n, dtype=np.float64) * seg.dt
    fa = np.zeros(len(freqs), dtype=np.complex128)
    fb = np.zeros(len(freqs), dtype=np.complex128)
    A = B = C = 0.0
    for x, g, det in zip(xs, gaps_list, dets):
        w = 1.0 / det.sigma2
        tau = seg.t_start + t
        tm = roemer_delay(tau, alpha, delta, eph, det)
        a, b = beam_ab(tau, alpha, delta, eph, det)
        m = sample_mask(seg.n, g)
        A += w * np.sum(m * a * a)
        B += w * np.sum(m * b * b)
        C += w * np.sum(m * a * b)
        phis = 2.0 * np.pi * fdot * (t * t / 2.0 + tm * t)
        xm = m * np.asarray(x, dtype=np.complex128)
        for i, f in enumerate(freqs):
            ph = 2.0 * np.pi * (f - seg.f_het) * t + 2.0 * np.pi * f * tm + phis
            e = np.exp(-1j * ph)
            fa[i] += w * np.sum(a * xm * e)
            fb[i] += w * np.sum(b * xm * e)
    return twoF_from(fa, fb, A, B, C)

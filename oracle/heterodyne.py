"""Time-domain front end (oracle, FP64): heterodyning, low-pass filtering
and downsampling of a real high-rate series, paper Sec. III.A.1
("Heterodyning, low-pass filtering, and downsampling", eqs. eq14-eq16).

TEST INFRASTRUCTURE, like the rest of this package.

The steps, in the paper's order, for raw samples x[m] at t_m = t_s + m dt_r:
1. heterodyne: x[m] exp(-2 pi i f_h (t_m - t_s)) (the sign of the worked
   example, as in the rest of this package: f_h moves to DC);
2. low-pass filter at the new Nyquist frequency B/2 = 1 / (2 D dt_r) (eq. eq16);
3. keep every D-th sample: x_h[j] at t_s + j D dt_r.

Readings (the paper leaves the filter open; listed in the design notes):
* filter: a Kaiser-windowed sinc of L = 2 K D + 1 taps centred on tap
  c = K D, cutoff B/2, window parameter beta, normalised to unit gain at DC;
  the passband is therefore flat only well inside +-B/2 and the edges are
  attenuated, as for any finite filter that cuts at the new Nyquist
  frequency;
* raw samples outside the series are zero (the filter's start and end
  transients are kept, not trimmed);
* output sample j is centred on raw sample j D.
"""
import numpy as np


def kaiser_lowpass(D, K, beta):
    """Taps h[0..L-1], L = 2 K D + 1: sinc at cutoff 1/(2D) cycles per raw
    sample times a Kaiser window, sum 1."""
    L = 2 * K * D + 1
    c = K * D
    n = np.arange(L) - c
    h = np.sinc(n / D) / D
    w = np.i0(beta * np.sqrt(1.0 - (n / c) ** 2)) / np.i0(beta) if c > 0 else np.ones(1)
    h = h * w
    return h / np.sum(h)


def heterodyne_decimate(x, dt_r, f_het, D, K, beta, n_out):
    """Steps 1-3: complex x_h[n_out] from real x (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    h = kaiser_lowpass(D, K, beta)
    L = len(h)
    c = K * D
    m_all = np.arange(len(x))
    xh = x * np.exp(-2j * np.pi * f_het * (m_all * dt_r))            # step 1
    out = np.zeros(n_out, dtype=np.complex128)
    for j in range(n_out):                                            # steps 2-3
        m = j * D + c - np.arange(L)
        ok = (m >= 0) & (m < len(x))
        out[j] = np.sum(h[ok] * xh[m[ok]])
    return out


def heterodyne_decimate_at(x, dt_r, f_het, D, K, beta, js):
    """Steps 1-3 at the output samples js only (for sampled checks of long
    series); the same arithmetic as heterodyne_decimate."""
    x = np.asarray(x)
    h = kaiser_lowpass(D, K, beta)
    L = len(h)
    c = K * D
    out = np.zeros(len(js), dtype=np.complex128)
    for o, j in enumerate(js):
        m = j * D + c - np.arange(L)
        ok = (m >= 0) & (m < len(x))
        mm = m[ok]
        out[o] = np.sum(h[ok] * x[mm].astype(np.float64) * np.exp(-2j * np.pi * f_het * (mm * dt_r)))
    return out

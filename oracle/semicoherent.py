"""Semi-coherent combination of per-segment F-statistics (oracle, FP64).

TEST INFRASTRUCTURE, like the rest of this package.

The paper computes a coherent 2F per segment and points to hierarchical
schemes that combine segments (Sec. I).  The combination built here is the
plain sum of per-segment 2F values along each template's frequency track
("StackSlide"): a template is (sky, f0, fdot) with f0 the frequency at a
reference time t_ref; segment i, whose phase reference is its own start
t_s,i (Sec. III.A.1, reading 9), sees the frequency
    f_i = f0 + fdot (t_s,i - t_ref)
and contributes its 2F at the nearest bin of its own grid,
    s_i = floor((f_i - f_het,i) / df_i + 1/2),
when that bin lies in the segment's reported band (nothing otherwise).
On the common grid f0_j = f_lo + j df_c, j < n_c:
    S(sky, fdot, j) = sum_i 2F_i(sky, fdot, s_i(j)).
Readings (listed in the design notes): the sum is unweighted; the nearest
bin is taken with halves rounded up, in FP64; a bin outside a segment's band
adds nothing.

At spindown order s a template is (sky, f0, f^(1), ..., f^(s)), all at t_ref.
The frequency's Taylor series (eq. eq4) moves it to the segment start,
    f_i = f0 + sum_k f^(k) D^k / k!,   D = t_s,i - t_ref,
and the segment demodulates with the spindowns moved there,
    f^(j)(t_s,i) = sum_{k >= j} f^(k) D^(k-j) / (k-j)!.
"""
import math

import numpy as np


def nearest_bin(f, f_het, df):
    """Signed bin of frequency f on the grid f_het + s df, halves up (FP64)."""
    return int(math.floor((f - f_het) / df + 0.5))


def translate_spindowns(spins, D):
    """(f^(1), ..., f^(s)) at t moved to t + D: f^(j)(t + D) =
    sum_{k >= j} f^(k) D^(k-j) / (k-j)!."""
    spins = np.atleast_1d(np.asarray(spins, dtype=np.float64))
    out = np.zeros(len(spins))
    for j in range(len(spins)):
        for k in range(j, len(spins)):
            out[j] += spins[k] * D ** (k - j) / math.factorial(k - j)
    return out


def frequency_shift(spins, D):
    """f(t + D) - f(t) = sum_k f^(k) D^k / k!, each term a product of
    separately rounded factors and the terms added in order of k, so that the
    nearest-bin decision is taken on one well-defined FP64 number."""
    spins = np.atleast_1d(np.asarray(spins, dtype=np.float64))
    shift = float(spins[0]) * D
    if len(spins) > 1:
        shift = shift + float(spins[1]) * ((D * D) * 0.5)
    if len(spins) > 2:
        shift = shift + float(spins[2]) * (((D * D) * D) * (1.0 / 6.0))
    return shift


def accumulate_segment(S, maps, s_lo, n_out, f_het, df, t_seg, fdots, t_ref, f_lo, df_c):
    """Add one segment's 2F maps to S (in place).

    S: [n_sky][n_fdot][n_c]; maps: [n_sky][n_fdot][n_out] with bin s_lo + i
    at index i, made with the spindowns moved to t_seg; fdots: [n_fdot]
    (order 1) or [n_fdot][s], at t_ref."""
    n_sky, n_fdot, n_c = S.shape
    for f in range(n_fdot):
        shift = frequency_shift(fdots[f], t_seg - t_ref)
        for j in range(n_c):
            s = nearest_bin(f_lo + j * df_c + shift, f_het, df)
            i = s - s_lo
            if 0 <= i < n_out:
                S[:, f, j] += maps[:, f, i]
    return S

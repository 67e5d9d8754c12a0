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
"""
import math

import numpy as np


def nearest_bin(f, f_het, df):
    """Signed bin of frequency f on the grid f_het + s df, halves up (FP64)."""
    return int(math.floor((f - f_het) / df + 0.5))


def accumulate_segment(S, maps, s_lo, n_out, f_het, df, t_seg, fdots, t_ref, f_lo, df_c):
    """Add one segment's 2F maps to S (in place).

    S: [n_sky][n_fdot][n_c]; maps: [n_sky][n_fdot][n_out] with bin s_lo + i
    at index i; fdots: [n_fdot]."""
    n_sky, n_fdot, n_c = S.shape
    for f in range(n_fdot):
        shift = fdots[f] * (t_seg - t_ref)
        for j in range(n_c):
            s = nearest_bin(f_lo + j * df_c + shift, f_het, df)
            i = s - s_lo
            if 0 <= i < n_out:
                S[:, f, j] += maps[:, f, i]
    return S

"""SSB sample grid and its inversion to detector time (oracle, FP64).

Paper Sec. III.A.2, eq. eq21: t_b^k = t^k + t_m(t^k).  The method needs the
inverse: detector times T^k whose barycentric times are regularly spaced.
Readings (the paper states neither the grid nor the inversion method):

* the SSB grid is t_b^k = k dt, k = 0..N-1, measured from the segment start,
  with the same spacing and length as the detector series;
* T^k is found by the fixed-point iteration T <- t_b^k - t_m(T) started at
  T = t_b^k.  Its contraction factor is |dt_m/dt| <= ~1e-4, so a handful of
  iterations reach FP64 resolution; iteration stops when the update is below
  1e-12 s or after 12 iterations.
* t_m,k = t_b^k - T^k (eq. phi-s-explain reads the Roemer term off the
  inverted times the same way).
"""
import numpy as np

from .ephemeris import roemer_delay


def ssb_grid(seg):
    """t_b^k = k dt (segment-relative seconds)."""
    return np.arange(seg.n, dtype=np.float64) * seg.dt


def invert_ssb_times(seg, alpha, delta, eph, det, tol=1e-12, max_iter=12, binary=None):
    """Return (T, t_m_at_T): detector times T^k with T^k + t_m(T^k) = k dt,
    and t_m,k = t_b^k - T^k.  With a binary orbit (oracle.binary) the grid is
    regular in emission time and the target is k dt + R(t_s + k dt); the
    second value is then the total delay d at T^k."""
    tb = ssb_grid(seg)
    target = tb
    if binary is not None:
        from .binary import binary_delay
        target = tb + binary_delay(seg.t_start + tb, binary)
    T = target.copy()
    for _ in range(max_iter):
        T_new = target - roemer_delay(seg.t_start + T, alpha, delta, eph, det)
        step = np.max(np.abs(T_new - T)) if T.size else 0.0
        T = T_new
        if step <= tol:
            break
    return T, tb - T

"""Binary-orbit timing of the source (oracle, FP64).

TEST INFRASTRUCTURE, like the rest of this package.

The paper names searches over binary systems as a use of the method's
savings (Sec. VI) without giving the timing model; the one built here (listed
in the design notes) is the circular-orbit Roemer delay of the source,
    R(tau_e) = a_p sin(2 pi (tau_e - t_asc) / P_b),
with tau_e the emission time, a_p the projected semi-major axis in
light-seconds and t_asc the time of the ascending node: a wavefront emitted
at tau_e reaches the SSB at tau_SSB = tau_e + R(tau_e).  With the detector's
Roemer delay t_m (eq. eq4pt2), tau_SSB = tau + t_m(tau) for detector time
tau, and the total delay from emission to detection is
    d(tau) = t_m(tau) - R(tau_e(tau)),   tau_e + R(tau_e) = tau + t_m(tau).
The resampled grid is regular in emission time, tau_e^k = t_s + k dt, so the
inversion (eq. eq21) targets tau_SSB^k = tau_e^k + R(tau_e^k); t_m is replaced
by d in the heterodyne correction (eqs. absorb, Fa3) and in the spindown
phase (eq. eq4pt1), and t_m,k = t_b^k - T^k becomes d at T^k.
"""
import numpy as np


def binary_delay(tau_e, b):
    """R(tau_e) = a_p sin(2 pi (tau_e - t_asc) / P_b), the angle reduced in
    cycles before it is formed."""
    cyc = (np.asarray(tau_e, dtype=np.float64) - b.t_asc) / b.p_orb
    return b.a_p * np.sin(2.0 * np.pi * (cyc - np.floor(cyc)))


def emission_time(tau_ssb, b, tol=1e-13, max_iter=30):
    """tau_e with tau_e + R(tau_e) = tau_ssb, by the fixed point
    tau_e <- tau_ssb - R(tau_e) (contraction a_p 2 pi / P_b)."""
    tau_ssb = np.asarray(tau_ssb, dtype=np.float64)
    te = tau_ssb.copy()
    for _ in range(max_iter):
        te_new = tau_ssb - binary_delay(te, b)
        step = np.max(np.abs(te_new - te)) if te.size else 0.0
        te = te_new
        if step <= tol:
            break
    return te

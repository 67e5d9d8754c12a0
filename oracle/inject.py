"""Signal generator for tests (oracle, FP64).

The strain of paper Sec. II, eq. eq1: h = F+ h+ + Fx hx with F+, Fx from eqs.
eq2/eq3 and the phase Psi of eq. eq4 (s up to 3).  The polarisation amplitudes
are the usual A+ = h0 (1 + cos^2 iota)/2, Ax = h0 cos iota (not stated in the
paper; the validity of 2F does not depend on it): h = F+ A+ cos Psi +
Fx Ax sin Psi.  The complex heterodyned series keeps the positive-frequency
half of h, (F+ A+ - i Fx Ax) e^{i Psi} / 2, times exp(-2 pi i f_h t) (the
heterodyne sign of Sec. III.A.1's worked example).

Psi - Phi0 = 2 pi f0 (t + t_m) + Phi_s(t),
Phi_s = 2 pi sum_j f^(j) (t^{j+1}/(j+1)! + t_m t^j/j!) for j = 1..3 (f^(1) = fdot,
f^(2), f^(3) of the injection; zero unless set), with t measured from the
segment start (Phi0 is the phase there).  With a binary orbit (oracle.binary)
t_m is replaced by the total delay d = t_m - R(tau_e).
"""
import numpy as np

from .antenna import beam_fplus_fcross
from .ephemeris import roemer_delay


def signal(seg, inj, eph, det):
    """Noise-free complex heterodyned signal at the detector grid (complex128)."""
    t = np.arange(seg.n, dtype=np.float64) * seg.dt
    tau = seg.t_start + t
    tm = roemer_delay(tau, inj.alpha, inj.delta, eph, det)
    if inj.binary is not None:                    # total delay d = t_m - R(tau_e)
        from .binary import binary_delay, emission_time
        tm = tm - binary_delay(emission_time(tau + tm, inj.binary), inj.binary)
    fp, fx = beam_fplus_fcross(tau, inj.alpha, inj.delta, inj.psi, eph, det)
    a_plus = inj.h0 * (1.0 + inj.cosi ** 2) / 2.0
    a_cross = inj.h0 * inj.cosi
    cycles = ((inj.f0 - seg.f_het) * t + inj.f0 * tm
              + inj.fdot * (t * t / 2.0 + tm * t)
              + inj.f2 * (t ** 3 / 6.0 + tm * t * t / 2.0)
              + inj.f3 * (t ** 4 / 24.0 + tm * t ** 3 / 6.0))
    phase = inj.phi0 + 2.0 * np.pi * cycles
    return 0.5 * (fp * a_plus - 1j * fx * a_cross) * np.exp(1j * phase)


def rho2_matched(A, B, C, inj, sigma2=1.0):
    """Closed-form noncentrality of 2F for a perfectly matched template:
    with p = A+ (c, s), q = Ax (s, -c), c = cos 2psi, s = sin 2psi and the Gram
    matrix G = [[A, C], [C, B]] of unweighted antenna sums,
    rho^2 = (p^T G p + q^T G q) / (2 sigma^2)."""
    c, s = np.cos(2 * inj.psi), np.sin(2 * inj.psi)
    ap = inj.h0 * (1.0 + inj.cosi ** 2) / 2.0
    ax = inj.h0 * inj.cosi
    G = np.array([[A, C], [C, B]])
    p = ap * np.array([c, s])
    q = ax * np.array([s, -c])
    return float(p @ G @ p + q @ G @ q) / (2.0 * sigma2)

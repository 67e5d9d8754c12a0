"""Pins of the binary-orbit timing in the oracle.

* a_p = 0 changes nothing;
* with the detector at the SSB (zero ephemeris radii, t_m = 0) the inverted
  times are T^k = k dt + R(t_s + k dt) exactly: R is evaluated at the
  emission time of the regular grid, with its sign;
* the emission-time fixed point solves tau_e + R(tau_e) = tau_SSB to a few
  FP64 ulp of the epoch;
* an injection from a binary source (a_p = 1.44 light-s, P_b = 68,023.7 s, a
  phase modulation of 2 pi f0 a_p ~ 900 rad) is recovered to the closed-form
  rho^2 with the matched orbit and lost without it."""
import dataclasses

import numpy as np

from oracle import binary as ob
from oracle import fstat as of
from oracle import timing as ot
from oracle.inject import rho2_matched, signal
from oracle.interp import KERNEL_LANCZOS
from paper_0912_4255_amd.synth import DET_H, Binary, Ephemeris, Injection, Segment

SEG = Segment(n=21600, dt=4.0, t_start=1.0e5, f_het=100.0)
NOGAP = np.zeros((0, 2), np.int64)
ORBIT = Binary(a_p=1.44, p_orb=68023.7, t_asc=2.3e4)


def test_zero_orbit_is_no_orbit():
    eph = Ephemeris()
    T0, tm0 = ot.invert_ssb_times(SEG, 1.2, 0.3, eph, DET_H)
    T1, tm1 = ot.invert_ssb_times(SEG, 1.2, 0.3, eph, DET_H, binary=Binary(0.0, 68023.7, 0.0))
    assert np.array_equal(T0, T1) and np.array_equal(tm0, tm1)


def test_detector_at_the_ssb_gives_the_closed_form():
    eph = dataclasses.replace(Ephemeris(), au_c=0.0, re_c=0.0)
    T, d = ot.invert_ssb_times(SEG, 1.2, 0.3, eph, DET_H, binary=ORBIT)
    tb = np.arange(SEG.n) * SEG.dt
    R = ORBIT.a_p * np.sin(2 * np.pi * (SEG.t_start + tb - ORBIT.t_asc) / ORBIT.p_orb)
    assert np.allclose(T, tb + R, rtol=0, atol=1e-9)
    assert np.allclose(d, -R, rtol=0, atol=1e-9)


def test_emission_time_fixed_point_residual():
    tau_ssb = SEG.t_start + np.linspace(0.0, 86400.0, 1001)
    te = ob.emission_time(tau_ssb, ORBIT)
    assert np.max(np.abs(te + ob.binary_delay(te, ORBIT) - tau_ssb)) < 5e-11   # a few ulp at 2e5 s


def test_binary_injection_needs_the_matched_orbit():
    eph = Ephemeris()
    s = 2500
    df = 1.0 / (2 * SEG.n * SEG.dt)
    inj = Injection(h0=1.0, cosi=0.3, psi=0.4, phi0=1.0, f0=SEG.f_het + s * df, fdot=-1e-10, alpha=1.2,
                    delta=0.3, binary=ORBIT)
    x = signal(SEG, inj, eph, DET_H)
    rs = of.resample(x, NOGAP, SEG, inj.alpha, inj.delta, eph, DET_H, KERNEL_LANCZOS, 8, binary=ORBIT)
    A, B, C = of.antenna_sums([rs], [DET_H])
    rho2 = rho2_matched(A, B, C, inj)
    F = of.fstat_bins([rs], [DET_H], inj.fdot, 2 * SEG.n, [s])[0]
    assert abs(F / rho2 - 1.0) < 0.03
    rs0 = of.resample(x, NOGAP, SEG, inj.alpha, inj.delta, eph, DET_H, KERNEL_LANCZOS, 8)
    F0 = of.fstat_spectrum([rs0], [DET_H], inj.fdot, 2 * SEG.n)[0].max()
    assert F0 / rho2 < 0.1

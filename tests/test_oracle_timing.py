"""Pins for the oracle ephemeris, Roemer delay and SSB inversion: closed-form
amplitudes, the Doppler magnitude of paper Sec. II (order 1e-4), finite
differences and the inversion residual."""
import math

import numpy as np

from oracle.ephemeris import (position_lightsec, roemer_delay, roemer_rate, sky_vector,
                              velocity_over_c)
from oracle.timing import invert_ssb_times
from paper_0912_4255_amd.synth import AU_M, C_MS, DET_H, DET_L, Ephemeris, Segment

EPH = Ephemeris()
YEAR = EPH.p_orb


def test_orbital_speed_is_order_1e4():
    tau = np.linspace(0, YEAR, 2001)
    eph0 = Ephemeris(re_c=0.0)
    v = np.linalg.norm(velocity_over_c(tau, eph0, DET_H), axis=-1)
    expect = (AU_M / C_MS) * 2 * math.pi / EPH.p_orb
    assert np.allclose(v, expect, rtol=1e-12, atol=0)
    assert 9.8e-5 < expect < 1.0e-4


def test_position_norms():
    tau = np.linspace(0, YEAR, 777)
    orb = position_lightsec(tau, Ephemeris(re_c=0.0), DET_H)
    rot = position_lightsec(tau, Ephemeris(au_c=0.0), DET_L)
    assert np.allclose(np.linalg.norm(orb, axis=-1), AU_M / C_MS, rtol=1e-14)
    assert np.allclose(np.linalg.norm(rot, axis=-1), 6.371e6 / C_MS, rtol=1e-14)


def test_ecliptic_pole_leaves_rotation_only():
    # Ecliptic north pole in equatorial coordinates: alpha = 270 deg, delta = 90 deg - eps.
    alpha, delta = 1.5 * math.pi, math.pi / 2 - EPH.eps
    tau = np.linspace(0, YEAR, 5001)
    tm = roemer_delay(tau, alpha, delta, EPH, DET_H)
    assert np.max(np.abs(tm)) <= EPH.re_c * (1 + 1e-12)


def test_ecliptic_plane_amplitude_is_au_over_c():
    # Vernal equinox direction lies in the ecliptic: amplitude AU/c over a year.
    tau = np.linspace(0, YEAR, 200001)
    tm = roemer_delay(tau, 0.0, 0.0, Ephemeris(re_c=0.0), DET_H)
    assert abs(np.max(tm) - AU_M / C_MS) < 1e-6
    assert abs(np.min(tm) + AU_M / C_MS) < 1e-6
    assert abs(AU_M / C_MS - 499.00478383615643) < 1e-9


def test_rate_matches_finite_difference():
    tau = np.array([0.0, 1234.5, 3.3e5, 1.7e7])
    for alpha, delta in [(1.2, 0.3), (4.0, -1.1)]:
        h = 1.0
        fd = (roemer_delay(tau + h, alpha, delta, EPH, DET_H)
              - roemer_delay(tau - h, alpha, delta, EPH, DET_H)) / (2 * h)
        an = roemer_rate(tau, alpha, delta, EPH, DET_H)
        assert np.max(np.abs(fd - an)) < 1e-12


def test_sky_vector_unit():
    for a, d in [(0.1, 0.2), (3.0, -1.2), (6.0, 1.5)]:
        assert abs(np.linalg.norm(sky_vector(a, d)) - 1.0) < 1e-15


def test_inversion_residual():
    seg = Segment(n=20000, dt=0.5, t_start=1.0e6, f_het=100.0)
    T, tm = invert_ssb_times(seg, 1.2, 0.3, EPH, DET_H)
    tb = np.arange(seg.n) * seg.dt
    resid = T + roemer_delay(seg.t_start + T, 1.2, 0.3, EPH, DET_H) - tb
    assert np.max(np.abs(resid)) < 1e-9
    assert np.allclose(tm, tb - T, atol=0, rtol=0)
    # T is increasing (1 + dt_m/dt > 0) and |t_m| bounded by AU/c + R_E/c
    assert np.all(np.diff(T) > 0)
    assert np.max(np.abs(tm)) < EPH.au_c + EPH.re_c

"""Analytic detector ephemeris and Roemer delay (oracle, FP64).

The paper leaves the ephemeris to LAL files; the reading used here is a
circular 1 AU orbit in the ecliptic (tilted by the obliquity about the x axis
of the equatorial frame), with the Sun at the SSB, plus a spherical Earth
rotating at the sidereal rate.  Coordinates are equatorial, lengths are in
light-seconds.

* Roemer delay t_m = n0 . r_d / c: paper Sec. II, eq. eq4pt2.
* Its rate dt_m/dt = n0 . v_d / c (the Doppler factor): eq. eq11c.
* n0(alpha, delta) is the unit vector to the source in the SSB frame
  (Sec. II, below eq. eq4).

Parity unpinned (conventions, not results): lambda0 and theta0 (angles at
the epoch), the spherical-Earth radius.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def revolution_angle(tau, period, phase0):
    """phase0 + 2 pi tau / period, computed as 2 pi times the fractional number
    of revolutions so that large tau keeps full FP64 precision."""
    rev = np.asarray(tau, dtype=np.float64) / period
    rev = rev - np.floor(rev)
    return phase0 + TWO_PI * rev


def orbital_longitude(tau, eph):
    return revolution_angle(tau, eph.p_orb, eph.lambda0)


def local_sidereal_angle(tau, eph, det):
    return revolution_angle(tau, eph.p_sid, eph.theta0) + det.lon


def sky_vector(alpha, delta):
    """n0 = (cos d cos a, cos d sin a, sin d)."""
    return np.array([np.cos(delta) * np.cos(alpha),
                     np.cos(delta) * np.sin(alpha),
                     np.sin(delta)])


def position_lightsec(tau, eph, det):
    """r_d(tau) / c, shape (..., 3): Earth's heliocentric position on the
    circular orbit plus the site's position on the rotating sphere."""
    lam = orbital_longitude(tau, eph)
    th = local_sidereal_angle(tau, eph, det)
    ce, se = np.cos(eph.eps), np.sin(eph.eps)
    cp, sp = np.cos(det.lat), np.sin(det.lat)
    orb = eph.au_c * np.stack([np.cos(lam), ce * np.sin(lam), se * np.sin(lam)], axis=-1)
    rot = eph.re_c * np.stack([cp * np.cos(th), cp * np.sin(th), sp * np.ones_like(th)], axis=-1)
    return orb + rot


def velocity_over_c(tau, eph, det):
    """v_d(tau) / c, shape (..., 3): the time derivative of position_lightsec."""
    lam = orbital_longitude(tau, eph)
    th = local_sidereal_angle(tau, eph, det)
    ce, se = np.cos(eph.eps), np.sin(eph.eps)
    cp = np.cos(det.lat)
    w_orb = TWO_PI / eph.p_orb
    w_sid = TWO_PI / eph.p_sid
    orb = eph.au_c * w_orb * np.stack([-np.sin(lam), ce * np.cos(lam), se * np.cos(lam)], axis=-1)
    rot = eph.re_c * w_sid * np.stack([-cp * np.sin(th), cp * np.cos(th), np.zeros_like(th)], axis=-1)
    return orb + rot


def roemer_delay(tau, alpha, delta, eph, det):
    """t_m(tau) = n0 . r_d / c in seconds (eq. eq4pt2)."""
    return position_lightsec(tau, eph, det) @ sky_vector(alpha, delta)


def roemer_rate(tau, alpha, delta, eph, det):
    """dt_m/dt = n0 . v_d / c (eq. eq11c)."""
    return velocity_over_c(tau, eph, det) @ sky_vector(alpha, delta)

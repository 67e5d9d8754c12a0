"""Beam-pattern functions a(t), b(t) (oracle, FP64).

Paper Sec. II, eqs. eq2 and eq3: F+ = sin(zeta)[a cos 2psi + b sin 2psi],
Fx = sin(zeta)[b cos 2psi - a sin 2psi], with a and b depending on time, the
site and the source but not on psi.  The paper defers their formulas to
Jaranowski, Krolak & Schutz; here they are computed from their definition as
contractions of the detector tensor with the wave polarisation tensors:

* site frame at local sidereal angle theta and latitude phi:
  e_E = (-sin th, cos th, 0), e_N = (-sin phi cos th, -sin phi sin th, cos phi);
* arms u, v at azimuths gamma +- 45 deg (counter-clockwise from East), so
  zeta = 90 deg and sin(zeta) = 1; detector tensor d = (u u^T - v v^T) / 2;
* wave frame at psi = 0: p = (-sin a, cos a, 0),
  q = (-sin d cos a, -sin d sin a, cos d), e+ = p p^T - q q^T,
  ex = p q^T + q p^T;
* a = d : e+,  b = d : ex.

Rotating (p, q) by psi turns e+ into cos2psi e+ + sin2psi ex and ex into
-sin2psi e+ + cos2psi ex, which reproduces eqs. eq2/eq3 exactly.

Parity unpinned (convention): the bisector azimuth gamma.
"""
import numpy as np

from .ephemeris import local_sidereal_angle


def polarisation_tensors(alpha, delta):
    p = np.array([-np.sin(alpha), np.cos(alpha), 0.0])
    q = np.array([-np.sin(delta) * np.cos(alpha), -np.sin(delta) * np.sin(alpha), np.cos(delta)])
    e_plus = np.outer(p, p) - np.outer(q, q)
    e_cross = np.outer(p, q) + np.outer(q, p)
    return e_plus, e_cross


def arm_vectors(tau, eph, det):
    """Unit vectors u, v along the two arms, shape (..., 3) each."""
    th = local_sidereal_angle(tau, eph, det)
    sp, cp = np.sin(det.lat), np.cos(det.lat)
    zero = np.zeros_like(th)
    e_E = np.stack([-np.sin(th), np.cos(th), zero], axis=-1)
    e_N = np.stack([-sp * np.cos(th), -sp * np.sin(th), cp * np.ones_like(th)], axis=-1)
    gu = det.gamma + np.pi / 4
    gv = det.gamma - np.pi / 4
    u = np.cos(gu) * e_E + np.sin(gu) * e_N
    v = np.cos(gv) * e_E + np.sin(gv) * e_N
    return u, v


def beam_ab(tau, alpha, delta, eph, det):
    """(a, b) at times tau: the contractions d:e+ and d:ex, using
    (x x^T) : E = x^T E x for the two outer products in d."""
    u, v = arm_vectors(tau, eph, det)
    e_plus, e_cross = polarisation_tensors(alpha, delta)

    def contract(E):
        return 0.5 * (np.einsum("...i,ij,...j->...", u, E, u)
                      - np.einsum("...i,ij,...j->...", v, E, v))

    return contract(e_plus), contract(e_cross)


def beam_fplus_fcross(tau, alpha, delta, psi, eph, det):
    """F+ and Fx from eqs. eq2 and eq3 with sin(zeta) = 1."""
    a, b = beam_ab(tau, alpha, delta, eph, det)
    c2, s2 = np.cos(2 * psi), np.sin(2 * psi)
    return a * c2 + b * s2, b * c2 - a * s2

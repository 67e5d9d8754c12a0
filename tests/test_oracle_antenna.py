"""Pins for the oracle beam patterns: the textbook response of an L-shaped
detector in its own frame, psi invariance, zenith response."""
import math

import numpy as np

from oracle.antenna import arm_vectors, beam_ab, beam_fplus_fcross
from oracle.ephemeris import local_sidereal_angle, sky_vector
from paper_0912_4255_amd.synth import DET_H, DET_L, Ephemeris

EPH = Ephemeris()


def _zenith(tau, det):
    th = local_sidereal_angle(tau, EPH, det)
    cp, sp = math.cos(det.lat), math.sin(det.lat)
    return np.stack([cp * np.cos(th), cp * np.sin(th), sp * np.ones_like(th)], axis=-1)


def test_textbook_detector_frame_response():
    """F+^2 + Fx^2 = (1/4)(1 + cos^2 th)^2 cos^2 2ph + cos^2 th sin^2 2ph, with
    th the source's angle from zenith and ph its azimuth from arm u."""
    rng = np.random.default_rng(3)
    tau = rng.uniform(0, 3e7, 400)
    for det in (DET_H, DET_L):
        for _ in range(10):
            alpha, delta = rng.uniform(0, 2 * math.pi), math.asin(rng.uniform(-1, 1))
            n0 = sky_vector(alpha, delta)
            u, v = arm_vectors(tau, EPH, det)
            up = _zenith(tau, det)
            ct = up @ n0
            nx, ny = u @ n0, v @ n0
            rr = nx * nx + ny * ny
            c2, s2 = (nx * nx - ny * ny) / rr, 2 * nx * ny / rr
            expect = 0.25 * (1 + ct ** 2) ** 2 * c2 ** 2 + ct ** 2 * s2 ** 2
            a, b = beam_ab(tau, alpha, delta, EPH, det)
            assert np.max(np.abs(a * a + b * b - expect)) < 1e-12


def test_arms_orthonormal_and_horizontal():
    tau = np.linspace(0, 1e6, 50)
    u, v = arm_vectors(tau, EPH, DET_H)
    up = _zenith(tau, DET_H)
    assert np.allclose(np.sum(u * u, -1), 1) and np.allclose(np.sum(v * v, -1), 1)
    assert np.max(np.abs(np.sum(u * v, -1))) < 1e-15
    assert np.max(np.abs(np.sum(u * up, -1))) < 1e-15


def test_zenith_source_unit_response_and_psi_invariance():
    tau = np.array([12345.0])
    up = _zenith(tau, DET_H)[0]
    alpha = math.atan2(up[1], up[0])
    delta = math.asin(up[2])
    a, b = beam_ab(tau, alpha, delta, EPH, DET_H)
    assert abs(a[0] ** 2 + b[0] ** 2 - 1.0) < 1e-12
    tau = np.linspace(0, 86400, 100)
    ref = None
    for psi in (0.0, 0.3, 1.1, -0.7):
        fp, fx = beam_fplus_fcross(tau, 1.2, 0.3, psi, EPH, DET_H)
        s = fp * fp + fx * fx
        ref = s if ref is None else ref
        assert np.max(np.abs(s - ref)) < 1e-14

"""Finite-difference gradient of 2F at a continuous frequency (oracle, FP64).

A project addition (the paper has no gradients).  2F(theta), theta =
(f, f^(1), ..., f^(s), alpha, delta) with spindown order s (eq. eq4pt1 for
general s), is the resampling-chain statistic of ``oracle.fstat`` evaluated
at the continuous frequency f (``fstat_point``), with the series re-resampled
for every sky offset.  For a source in a circular binary orbit (the timing
model of ``oracle.binary``) theta ends with the orbit, (..., alpha, delta,
a_p, P_b, t_asc), and the series is re-resampled for every orbit offset too.  Derivatives are central differences with
Richardson extrapolation, D = (4 g(h/2) - g(h)) / 3, g(h) = (F(x+h) - F(x-h)) / (2h), with 2h taken as the
difference of the two rounded arguments.

Default steps: h_f = 1e-3 / T0 Hz, h_(j) = 1e-3 / T0^(j+1) Hz/s^j for
f^(j), h_alpha = h_delta = 1e-7 rad; for an orbit h_a = 1e-7 light-s,
h_P = 1e-3 s, h_asc = 1e-2 s.
"""
from collections import namedtuple

import numpy as np

from .fstat import fstat_point, resample_all


Orbit = namedtuple("Orbit", "a_p p_orb t_asc")


class PointProblem:
    """Fixed data for 2F(theta): series, gaps, segment, detectors, ephemeris,
    interpolation kernel; binary=True when theta ends with an orbit."""

    def __init__(self, xs, gaps_list, seg, dets, eph, kernel, W, binary=False):
        self.binary = binary
        self.xs = xs
        self.gaps = gaps_list
        self.seg = seg
        self.dets = dets
        self.eph = eph
        self.kernel = kernel
        self.W = W
        self._cache = {}

    def resampled(self, alpha, delta, orbit=None):
        key = (float(alpha), float(delta)) + (tuple(float(v) for v in orbit) if orbit is not None else ())
        if key not in self._cache:
            if len(self._cache) > 8:
                self._cache.clear()
            self._cache[key] = resample_all(self.xs, self.gaps, self.seg, alpha, delta,
                                            self.eph, self.dets, self.kernel, self.W,
                                            binary=Orbit(*key[2:]) if orbit is not None else None)
        return self._cache[key]

    def twoF(self, theta):
        th = np.asarray(theta, dtype=np.float64)
        ns = 5 if self.binary else 2
        f, spins, sky = float(th[0]), th[1:-ns], th[-ns:]
        orbit = sky[2:] if self.binary else None
        return fstat_point(self.resampled(sky[0], sky[1], orbit), self.dets, self.seg, f, spins)


def default_steps(seg, order=1, binary=False):
    T0 = seg.n * seg.dt
    return np.array([1e-3 / T0] + [1e-3 / T0 ** (j + 1) for j in range(1, order + 1)] + [1e-7, 1e-7]
                    + ([1e-7, 1e-3, 1e-2] if binary else []))


def central(fun, theta, i, h):
    """Central difference divided by the step actually represented in FP64
    (theta_i + h and theta_i - h are rounded; at f ~ 100 Hz the rounding is
    ~1e-6 of a 1e-8 Hz step)."""
    tp = np.array(theta, dtype=np.float64)
    tm = tp.copy()
    tp[i] += h
    tm[i] -= h
    return (fun(tp) - fun(tm)) / (tp[i] - tm[i])


def gradient(problem, theta, steps=None):
    """Richardson-extrapolated central differences of 2F w.r.t. every
    component of theta."""
    theta = np.asarray(theta, dtype=np.float64)
    if steps is None:
        steps = default_steps(problem.seg, len(theta) - (6 if problem.binary else 3), problem.binary)
    steps = np.asarray(steps)
    g = np.empty(len(theta))
    for i in range(len(theta)):
        g1 = central(problem.twoF, theta, i, steps[i])
        g2 = central(problem.twoF, theta, i, steps[i] / 2.0)
        g[i] = (4.0 * g2 - g1) / 3.0
    return g

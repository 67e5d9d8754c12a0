"""Finite-difference gradient of 2F at a continuous frequency (oracle, FP64).

A project addition (the paper has no gradients).  2F(theta), theta =
(f, f^(1), ..., f^(s), alpha, delta) with spindown order s = len(theta) - 3
(eq. eq4pt1 for general s), is the resampling-chain statistic of
``oracle.fstat`` evaluated at the continuous frequency f (``fstat_point``),
with the series re-resampled for every sky offset.  Derivatives are central differences with
Richardson extrapolation, D = (4 g(h/2) - g(h)) / 3, g(h) = (F(x+h) - F(x-h)) / (2h), with 2h taken as the
difference of the two rounded arguments.

Default steps: h_f = 1e-3 / T0 Hz, h_(j) = 1e-3 / T0^(j+1) Hz/s^j for
f^(j), h_alpha = h_delta = 1e-7 rad.
"""
import numpy as np

from .fstat import fstat_point, resample_all


class PointProblem:
    """Fixed data for 2F(theta): series, gaps, segment, detectors, ephemeris,
    interpolation kernel."""

    def __init__(self, xs, gaps_list, seg, dets, eph, kernel, W):
        self.xs = xs
        self.gaps = gaps_list
        self.seg = seg
        self.dets = dets
        self.eph = eph
        self.kernel = kernel
        self.W = W
        self._cache = {}

    def resampled(self, alpha, delta):
        key = (float(alpha), float(delta))
        if key not in self._cache:
            if len(self._cache) > 8:
                self._cache.clear()
            self._cache[key] = resample_all(self.xs, self.gaps, self.seg, alpha, delta,
                                            self.eph, self.dets, self.kernel, self.W)
        return self._cache[key]

    def twoF(self, theta):
        th = np.asarray(theta, dtype=np.float64)
        f, spins, alpha, delta = float(th[0]), th[1:-2], float(th[-2]), float(th[-1])
        return fstat_point(self.resampled(alpha, delta), self.dets, self.seg, f, spins)


def default_steps(seg, order=1):
    T0 = seg.n * seg.dt
    return np.array([1e-3 / T0] + [1e-3 / T0 ** (j + 1) for j in range(1, order + 1)] + [1e-7, 1e-7])


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
    steps = default_steps(problem.seg, len(theta) - 3) if steps is None else np.asarray(steps)
    g = np.empty(len(theta))
    for i in range(len(theta)):
        g1 = central(problem.twoF, theta, i, steps[i])
        g2 = central(problem.twoF, theta, i, steps[i] / 2.0)
        g[i] = (4.0 * g2 - g1) / 3.0
    return g

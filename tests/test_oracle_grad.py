"""Pins for the oracle's finite-difference gradient of 2F.

* in f and the spindowns f^(1..s) the resampled series is fixed, so the
  derivative has a closed form (the single-bin sum differentiated under the
  sum: d Phi_s / d f^(j) = 2 pi (T^(j+1)/(j+1)! + t_m T^j/j!)), derived here
  independently of the finite differences, at spindown orders 1, 2 and 3;
* in alpha and delta the series is re-resampled; the Richardson value must
  agree with plain central differences at two step sizes;
* at the noise-free peak of an on-bin matched injection of a stationary
  detector, d2F/df vanishes by symmetry.
"""
import numpy as np
import pytest

from oracle import fstat as of
from oracle import grad as og
from oracle.inject import signal
from oracle.interp import KERNEL_LANCZOS
from paper_0912_4255_amd.synth import DET_H, Ephemeris, Injection, Segment, gaussian_noise

EPH = Ephemeris()
SEG = Segment(n=21600, dt=4.0, t_start=0.0, f_het=100.0)
DF = 1.0 / (2 * SEG.n * SEG.dt)
NOGAP = np.zeros((0, 2), np.int64)


def _problem(seed=1, h0=0.5, eph=EPH):
    inj = Injection(h0=h0, cosi=0.2, psi=-0.3, phi0=2.0, f0=SEG.f_het + 3000.3 * DF,
                    fdot=-4e-10, alpha=2.1, delta=-0.4)
    x = gaussian_noise(np.random.default_rng(seed), SEG.n, 1.0) + signal(SEG, inj, eph, DET_H)
    return og.PointProblem([x], [NOGAP], SEG, [DET_H], eph, KERNEL_LANCZOS, 8), inj


def _analytic_f_spins(problem, theta):
    f, spins, alpha, delta = theta[0], theta[1:-2], theta[-2], theta[-1]
    rs = problem.resampled(alpha, delta)
    A, B, C = of.antenna_sums(rs, problem.dets)
    D = A * B - C * C
    ya, yb = of.integrands(rs, problem.dets, spins)
    t = np.arange(SEG.n) * SEG.dt
    e = np.exp(-2j * np.pi * (f - SEG.f_het) * t)
    T, tm = rs[0]["T"], rs[0]["tm"]
    # d/d f^(j) of the spindown phase, written out per order
    u = [T ** 2 / 2 + tm * T, T ** 3 / 6 + tm * T ** 2 / 2, T ** 4 / 24 + tm * T ** 3 / 6][:len(spins)]
    fa, fb = np.sum(ya * e), np.sum(yb * e)
    out = []
    for w in [-2j * np.pi * t] + [-2j * np.pi * uj for uj in u]:
        dfa, dfb = np.sum(w * ya * e), np.sum(w * yb * e)
        d = 2.0 * (2 * B * np.real(np.conj(fa) * dfa) + 2 * A * np.real(np.conj(fb) * dfb)
                   - 2 * C * np.real(dfa * np.conj(fb) + fa * np.conj(dfb))) / D
        out.append(d)
    return np.array(out)


@pytest.mark.parametrize("spins", [[3e-12], [3e-12, -2e-17], [3e-12, -2e-17, 5e-23]])
def test_fd_matches_closed_form_in_f_and_spindowns(spins):
    prob, inj = _problem()
    theta = np.array([inj.f0 + 0.2 * DF] + [inj.fdot + spins[0]] + spins[1:] + [inj.alpha, inj.delta])
    g = og.gradient(prob, theta)
    assert g.shape == theta.shape
    ref = _analytic_f_spins(prob, theta)
    assert np.max(np.abs(g[:1 + len(spins)] - ref) / np.abs(ref)) < 1e-6


@pytest.mark.parametrize("extra", [[], [4e-17]])
def test_richardson_consistent_in_sky(extra):
    prob, inj = _problem(seed=2)
    theta = np.array([inj.f0, inj.fdot] + extra + [inj.alpha + 2e-4, inj.delta - 1e-4])
    h = og.default_steps(SEG, 1 + len(extra))
    g = og.gradient(prob, theta)
    for i in (len(theta) - 2, len(theta) - 1):
        c1 = og.central(prob.twoF, theta, i, h[i])
        c2 = og.central(prob.twoF, theta, i, h[i] / 4)
        assert abs(c1 - g[i]) < 1e-4 * abs(g[i]) + 1e-3
        assert abs(c2 - g[i]) < 1e-4 * abs(g[i]) + 1e-3


def test_peak_has_zero_frequency_derivative():
    eph0 = Ephemeris(au_c=0.0, re_c=0.0)
    inj = Injection(h0=1.0, cosi=0.5, psi=0.1, phi0=0.3, f0=SEG.f_het + 2000 * DF,
                    fdot=0.0, alpha=1.0, delta=0.5)
    x = signal(SEG, inj, eph0, DET_H)
    prob = og.PointProblem([x], [NOGAP], SEG, [DET_H], eph0, KERNEL_LANCZOS, 8)
    theta = np.array([inj.f0, 0.0, inj.alpha, inj.delta])
    g = og.gradient(prob, theta)
    F = prob.twoF(theta)
    T0 = SEG.n * SEG.dt
    assert abs(g[0]) * (1.0 / T0) < 1e-6 * F


def test_binary_gradient_zero_orbit_and_consistency():
    """Binary theta (f, fdot, alpha, delta, a_p, P_b, t_asc): with a_p = 0 the
    orbit drops out, so 2F and the first four derivatives equal the isolated
    source's and the P_b, t_asc derivatives vanish exactly; on a real orbit
    each orbital derivative agrees with plain central differences at two
    step sizes."""
    x_prob, inj = _problem(seed=4)
    prob = og.PointProblem(x_prob.xs, x_prob.gaps, SEG, [DET_H], EPH, KERNEL_LANCZOS, 8, binary=True)
    th4 = np.array([inj.f0 + 0.1 * DF, inj.fdot, inj.alpha + 1e-4, inj.delta])
    g4 = og.gradient(x_prob, th4)
    th7 = np.concatenate([th4, [0.0, 40000.0, 9.0e3]])
    g7 = og.gradient(prob, th7)
    assert prob.twoF(th7) == x_prob.twoF(th4)
    assert np.allclose(g7[:4], g4, rtol=1e-9, atol=0)
    assert g7[5] == 0.0 and g7[6] == 0.0 and g7[4] != 0.0
    th = np.concatenate([th4, [0.8, 40000.0, 9.0e3]])
    h = og.default_steps(SEG, 1, binary=True)
    g = og.gradient(prob, th)
    for i in (4, 5, 6):
        c1 = og.central(prob.twoF, th, i, h[i])
        c2 = og.central(prob.twoF, th, i, h[i] / 4)
        assert abs(c1 - g[i]) < 1e-4 * abs(g[i]) + 1e-6, (i, c1, g[i])
        assert abs(c2 - g[i]) < 1e-4 * abs(g[i]) + 1e-6, (i, c2, g[i])

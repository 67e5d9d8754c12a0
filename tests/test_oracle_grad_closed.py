"""Closed-form pins of the oracle gradient's sky and orbit components.

The oracle differentiates 2F with respect to (alpha, delta) and the orbit
(a_p, P_b, t_asc) only by finite differences of the re-resampled chain.  Two
configurations reduce that chain far enough for a closed form, derived here
from the paper's formulas and not from the oracle's code:

* No Roemer delay (ephemeris with au_c = re_c = 0): t_m = 0, so T^k = k dt,
  the heterodyne correction is 1 and the interpolation sits on integer
  positions (the identity).  The sky then enters 2F only through the beam
  patterns a = d:e+ and b = d:ex (Sec. II, eqs. eq2, eq3), whose derivatives
  in alpha and delta follow from those of the wave-frame vectors p and q:
  da = 2 p^T d dp - 2 q^T d dq and db = 2 (dp^T d q + p^T d dq).  2F of
  eq. eq6 is then differentiated through f_a = sum a_k g_k, f_b likewise, and
  the antenna sums A', B', C' of eqs. eq9, eq10.

* The same detector and a source in a circular binary orbit, at a_p = 0.
  With S_k = sin(2 pi (t_s + k dt - t_asc) / P_b), the emission-grid target
  of the inversion moves T^k by S_k da_p; the total delay d = -R moves by
  -S da_p, so the heterodyne correction (eqs. absorb, Fa3) contributes
  2 pi i f_h S_k x_k; the interpolation contributes (S_k / dt) sum_m w'(m)
  x_(k-m) with the Lanczos derivative at integers w'(m) = (-1)^m / m
  sinc(2m/W); the spindown phase 2 pi fdot (T^2/2 + d T) is stationary at
  d = 0; the beam patterns move by their time derivative (sidereal rotation
  of the site frame) times S_k.  At a_p = 0 the derivatives in P_b and
  t_asc vanish exactly.

* The same orbit at a small a_p = e: the delay e S_k moves with P_b and
  t_asc through dS_k/dP_b and dS_k/dt_asc, so those derivatives are e times
  the zero-orbit derivative along these directions, up to O(e^2).

A swapped (alpha, delta), a dropped chain term or a wrong sign in any of
these fails the comparison.
"""
import numpy as np
import pytest

from oracle import grad as og
from oracle.inject import signal
from oracle.interp import KERNEL_LANCZOS
from paper_0912_4255_amd.synth import DET_H, Ephemeris, Injection, Segment, gaussian_noise

EPH0 = Ephemeris(au_c=0.0, re_c=0.0)
SEG = Segment(n=21600, dt=4.0, t_start=3.0e5, f_het=100.0)
DF = 1.0 / (2 * SEG.n * SEG.dt)
NOGAP = np.zeros((0, 2), np.int64)
W = 8


def _site_frame(tau, det, eph):
    """Arm unit vectors u, v and their derivatives in the local sidereal angle."""
    th = eph.theta0 + 2.0 * np.pi * np.mod(tau / eph.p_sid, 1.0) + det.lon
    sp, cp = np.sin(det.lat), np.cos(det.lat)
    s, c = np.sin(th), np.cos(th)
    z = np.zeros_like(th)
    eE = np.stack([-s, c, z], -1)
    eN = np.stack([-sp * c, -sp * s, cp + z], -1)
    deE = np.stack([-c, -s, z], -1)
    deN = np.stack([sp * s, -sp * c, z], -1)
    gu, gv = det.gamma + np.pi / 4, det.gamma - np.pi / 4
    u = np.cos(gu) * eE + np.sin(gu) * eN
    v = np.cos(gv) * eE + np.sin(gv) * eN
    du = np.cos(gu) * deE + np.sin(gu) * deN
    dv = np.cos(gv) * deE + np.sin(gv) * deN
    return u, v, du, dv


def _wave_frame(alpha, delta):
    """p, q and their derivatives in alpha and in delta."""
    sa, ca, sd, cd = np.sin(alpha), np.cos(alpha), np.sin(delta), np.cos(delta)
    p = np.array([-sa, ca, 0.0])
    q = np.array([-sd * ca, -sd * sa, cd])
    p_a = np.array([-ca, -sa, 0.0])
    q_a = np.array([sd * sa, -sd * ca, 0.0])
    p_d = np.zeros(3)
    q_d = np.array([-cd * ca, -cd * sa, -sd])
    return p, q, (p_a, q_a), (p_d, q_d)


def _beams(tau, alpha, delta, det, eph):
    """a, b, da/d(alpha, delta), db/d(alpha, delta), da/dtau, db/dtau."""
    u, v, du, dv = _site_frame(tau, det, eph)
    p, q, dA, dD = _wave_frame(alpha, delta)
    up, uq, vp, vq = u @ p, u @ q, v @ p, v @ q
    a = 0.5 * (up ** 2 - uq ** 2 - vp ** 2 + vq ** 2)
    b = up * uq - vp * vq
    da, db = [], []
    for dp, dq in (dA, dD):
        udp, udq, vdp, vdq = u @ dp, u @ dq, v @ dp, v @ dq
        # a = p^T d p - q^T d q, b = 2 p^T d q with d = (u u^T - v v^T)/2
        da.append(up * udp - vp * vdp - (uq * udq - vq * vdq))
        db.append(udp * uq - vdp * vq + up * udq - vp * vdq)
    w_sid = 2.0 * np.pi / eph.p_sid
    dup, duq, dvp, dvq = du @ p, du @ q, dv @ p, dv @ q
    a_t = w_sid * (up * dup - uq * duq - vp * dvp + vq * dvq)
    b_t = w_sid * (dup * uq + up * duq - dvp * vq - vp * dvq)
    return a, b, da, db, a_t, b_t


def _twoF_and_grad(fa, fb, A, B, C, dfa, dfb, dA, dB, dC):
    """2F = 2 (B|fa|^2 + A|fb|^2 - 2 C Re(fa fb*)) / D and its derivative
    along one direction (quotient rule)."""
    D = A * B - C * C
    N = B * abs(fa) ** 2 + A * abs(fb) ** 2 - 2 * C * np.real(fa * np.conj(fb))
    dN = (dB * abs(fa) ** 2 + 2 * B * np.real(np.conj(fa) * dfa) + dA * abs(fb) ** 2
          + 2 * A * np.real(np.conj(fb) * dfb)
          - 2 * dC * np.real(fa * np.conj(fb)) - 2 * C * np.real(dfa * np.conj(fb) + fa * np.conj(dfb)))
    dD = dA * B + A * dB - 2 * C * dC
    return 2 * N / D, 2 * (dN * D - N * dD) / D ** 2


def _data(seed):
    inj = Injection(h0=0.6, cosi=0.35, psi=0.25, phi0=0.7, f0=SEG.f_het + 2400.3 * DF,
                    fdot=-3e-10, alpha=0.9, delta=-0.45)
    x = gaussian_noise(np.random.default_rng(seed), SEG.n, 1.0) + signal(SEG, inj, EPH0, DET_H)
    return x, inj


def _phase_kernel(theta_f, fdot):
    t = np.arange(SEG.n) * SEG.dt
    # e^{-i Phi_s} with t_m = 0 (eq. eq4pt1) times the single-bin Fourier kernel
    return np.exp(-2j * np.pi * (fdot * t * t / 2.0 + (theta_f - SEG.f_het) * t))


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_sky_derivatives_match_closed_form_without_roemer_delay(seed):
    x, inj = _data(seed)
    prob = og.PointProblem([x], [NOGAP], SEG, [DET_H], EPH0, KERNEL_LANCZOS, W)
    theta = np.array([inj.f0 + 0.15 * DF, inj.fdot, inj.alpha + 0.02, inj.delta - 0.03])
    g = og.gradient(prob, theta)

    tau = SEG.t_start + np.arange(SEG.n) * SEG.dt
    a, b, da, db, _, _ = _beams(tau, theta[2], theta[3], DET_H, EPH0)
    gk = np.asarray(x, np.complex128) * _phase_kernel(theta[0], theta[1])
    fa, fb = np.sum(a * gk), np.sum(b * gk)
    A, B, C = np.sum(a * a), np.sum(b * b), np.sum(a * b)
    F, _ = _twoF_and_grad(fa, fb, A, B, C, 0, 0, 0, 0, 0)
    assert abs(prob.twoF(theta) - F) < 1e-9 * F
    for i, (dai, dbi) in enumerate(zip(da, db)):
        _, dF = _twoF_and_grad(fa, fb, A, B, C, np.sum(dai * gk), np.sum(dbi * gk),
                               2 * np.sum(a * dai), 2 * np.sum(b * dbi), np.sum(dai * b + a * dbi))
        # floor: FP64 rounding of 2F (about 1e-15 F) over the 1e-7 rad step
        assert abs(g[2 + i] - dF) <= 1e-6 * abs(dF) + 1e-8 * F, (i, g[2 + i], dF)
    # the two sky components differ, so a swap of (alpha, delta) would fail
    assert abs(g[2] - g[3]) > 0.1 * max(abs(g[2]), abs(g[3]))


def _lanczos_slope_at_integers(W):
    """w'(m) for m = -W/2 .. W/2 of w(x) = sinc(x) sinc(2x/W): (-1)^m / m
    sinc(2m/W) for m != 0, zero at m = 0 (w is even) and at |m| = W/2."""
    m = np.arange(-W // 2, W // 2 + 1)
    out = np.zeros(len(m))
    nz = m != 0
    out[nz] = (-1.0) ** m[nz] / m[nz] * np.sinc(2.0 * m[nz] / W)
    return m, out


def _delay_derivative(x, theta, v):
    """2F at zero orbit and its derivative when the total delay of sample k
    moves by -v_k (the emission-grid target T^k by +v_k), per the chain
    terms listed above; also the derivative with the heterodyne term left
    out."""
    n = SEG.n
    k = np.arange(n)
    tau = SEG.t_start + k * SEG.dt
    a, b, _, _, a_t, b_t = _beams(tau, theta[2], theta[3], DET_H, EPH0)
    xc = np.asarray(x, np.complex128)
    # interpolation slope: sum_m w'(m) x_(k-m), taps outside the segment zero
    ms, wp = _lanczos_slope_at_integers(W)
    slope = np.zeros(n, np.complex128)
    for m, wm in zip(ms, wp):
        if wm == 0.0:
            continue
        j = k - m
        ok = (j >= 0) & (j < n)
        slope[ok] += wm * xc[j[ok]]
    ph = _phase_kernel(theta[0], theta[1])
    fa, fb = np.sum(a * xc * ph), np.sum(b * xc * ph)
    da, db = a_t * v, b_t * v
    A, B, C = np.sum(a * a), np.sum(b * b), np.sum(a * b)
    out = []
    for het in (1.0, 0.0):
        dz = v / SEG.dt * slope + het * 2j * np.pi * SEG.f_het * v * xc
        dfa = np.sum((da * xc + a * dz) * ph)
        dfb = np.sum((db * xc + b * dz) * ph)
        out.append(_twoF_and_grad(fa, fb, A, B, C, dfa, dfb, 2 * np.sum(a * da), 2 * np.sum(b * db),
                                  np.sum(da * b + a * db)))
    (F, dF), (_, dF0) = out
    return F, dF, dF0


P_B, T_ASC = 40000.0, 9.0e3


def _orbit_phase():
    tau = SEG.t_start + np.arange(SEG.n) * SEG.dt
    return tau, 2.0 * np.pi * (tau - T_ASC) / P_B


def test_orbit_amplitude_derivative_matches_closed_form_at_zero_orbit():
    x, inj = _data(21)
    prob = og.PointProblem([x], [NOGAP], SEG, [DET_H], EPH0, KERNEL_LANCZOS, W, binary=True)
    theta = np.array([inj.f0 + 0.2 * DF, inj.fdot, inj.alpha, inj.delta, 0.0, P_B, T_ASC])
    g = og.gradient(prob, theta)
    _, psi = _orbit_phase()
    F, dF, dF0 = _delay_derivative(x, theta, np.sin(psi))
    assert abs(prob.twoF(theta) - F) < 1e-9 * F
    assert abs(g[4] - dF) <= 1e-6 * abs(dF) + 1e-8 * F, (g[4], dF)
    # the heterodyne term dominates: dropping it changes the derivative grossly
    assert abs(dF0 - dF) > 1e-2 * abs(dF)
    # with a_p = 0 the delay a_p S does not depend on P_b or t_asc at all
    assert g[5] == 0.0 and g[6] == 0.0


@pytest.mark.parametrize("seed", [22, 24])
def test_orbit_period_and_epoch_derivatives_at_small_amplitude(seed):
    """At a_p = e the delay is e S_k, so d2F/dP_b and d2F/dt_asc are e times
    the zero-orbit derivative along dS/dP_b = -cos(psi) 2 pi (tau - t_asc) /
    P_b^2 and dS/dt_asc = -cos(psi) 2 pi / P_b, plus O(e^2).  Richardson in e,
    2 g(e)/e - g(2e)/(2e), removes the e^2 term; steps of 1 s in P_b and
    t_asc keep the difference quotients above the FP64 rounding of t ~ 3e5 s
    (the default steps are sized for a_p near a light-second)."""
    x, inj = _data(seed)
    prob = og.PointProblem([x], [NOGAP], SEG, [DET_H], EPH0, KERNEL_LANCZOS, W, binary=True)
    steps = og.default_steps(SEG, 1, binary=True)
    steps[5] = steps[6] = 1.0
    e = 1e-5
    gs = []
    for ap in (e, 2 * e):
        theta = np.array([inj.f0 + 0.2 * DF, inj.fdot, inj.alpha, inj.delta, ap, P_B, T_ASC])
        gs.append(og.gradient(prob, theta, steps) / ap)
    lin = 2.0 * gs[0] - gs[1]
    tau, psi = _orbit_phase()
    _, dP, _ = _delay_derivative(x, theta, -np.cos(psi) * 2.0 * np.pi * (tau - T_ASC) / P_B ** 2)
    _, dT, _ = _delay_derivative(x, theta, -np.cos(psi) * 2.0 * np.pi / P_B)
    assert abs(lin[5] - dP) <= 2e-3 * abs(dP), (lin[5], dP)
    assert abs(lin[6] - dT) <= 2e-3 * abs(dT), (lin[6], dT)
    # P_b and t_asc derivatives differ, so a swap of the two would fail
    assert abs(dP - dT) > 0.5 * max(abs(dP), abs(dT))

"""Workload descriptions and seeded synthetic inputs.

This module is shared by the HIP path, the CPU oracle, the tests and the
benchmark.  It holds only descriptions (detector sites, ephemeris constants,
segment shapes, template grids) and random draws (Gaussian noise, gap
placement, injection parameters, sky positions).  It contains none of the
method's arithmetic: no Roemer delay, no beam pattern, no interpolation, no
FFT and no detection statistic.  Signals that depend on the timing model are
generated elsewhere (by the oracle, for tests).

All draws use NumPy's PCG64 seeded from ``SeedSequence(9124255 + index)``
spawned into independent streams, so every input is reproducible.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

DEG = math.pi / 180.0
DAY = 86400.0

# Physical constants used by the analytic ephemeris (SI).
AU_M = 1.495978707e11
C_MS = 299792458.0
R_EARTH_M = 6.371e6
P_ORB_S = 365.256363 * DAY          # sidereal year
P_SID_S = 86164.0905                # sidereal day
OBLIQUITY_RAD = 23.4393 * DEG

SEED_BASE = 9124255


@dataclass(frozen=True)
class Ephemeris:
    """Circular 1 AU orbit in the ecliptic plus a spherical rotating Earth.

    Angles at tau = 0 (the ephemeris epoch) are ``lambda0`` (orbital
    longitude) and ``theta0`` (Greenwich sidereal angle)."""
    au_c: float = AU_M / C_MS
    re_c: float = R_EARTH_M / C_MS
    p_orb: float = P_ORB_S
    p_sid: float = P_SID_S
    eps: float = OBLIQUITY_RAD
    lambda0: float = 0.0
    theta0: float = 0.0


@dataclass(frozen=True)
class Detector:
    """Interferometer site.  ``gamma`` is the azimuth of the arm bisector,
    counter-clockwise from local East; arms are at gamma +- 45 deg."""
    lat: float
    lon: float
    gamma: float
    sigma2: float = 1.0


# Sites of the workloads: latitude/longitude from the configurations; the
# bisector azimuths are a convention (the statistic depends on span{a, b} only).
DET_H = Detector(lat=46.45 * DEG, lon=-119.41 * DEG, gamma=171.8 * DEG, sigma2=1.0)
DET_L = Detector(lat=30.56 * DEG, lon=-90.77 * DEG, gamma=243.0 * DEG, sigma2=1.3)


@dataclass(frozen=True)
class Segment:
    """A regularly sampled heterodyned series: n samples at dt, starting at
    t_start seconds after the ephemeris epoch, heterodyned at f_het."""
    n: int
    dt: float
    t_start: float
    f_het: float


KERNEL_LANCZOS = 0
KERNEL_DIRICHLET = 1
NFFT_TWICE = 0        # N_fft = 2 N
NFFT_SMOOTH7 = 1      # smallest 2^a 3^b 5^c 7^d >= 2 N
NFFT_SMOOTH7_256 = 2  # smallest 256 x 2^a 3^b 5^c 7^d >= 2 N
STORE_F32 = 0
STORE_F16 = 1


@dataclass
class Binary:
    """Circular binary orbit of the source: projected semi-major axis a_p
    (light-seconds), period p_orb (s), time of the ascending node t_asc (s,
    on the ephemeris clock)."""
    a_p: float
    p_orb: float
    t_asc: float


@dataclass
class Injection:
    h0: float
    cosi: float
    psi: float
    phi0: float
    f0: float
    fdot: float
    alpha: float
    delta: float
    f2: float = 0.0     # second and third frequency derivatives (eq. eq4, s up to 3)
    f3: float = 0.0
    binary: Optional[Binary] = None


@dataclass
class Workload:
    name: str
    detectors: Tuple[Detector, ...]
    segment: Segment
    f_lo: float
    f_hi: float
    kernel: int
    taps: int
    nfft_policy: int = NFFT_TWICE
    storage: int = STORE_F32
    eph: Ephemeris = field(default_factory=Ephemeris)
    skies: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    fdots: np.ndarray = field(default_factory=lambda: np.zeros(0))
    injections: List[Injection] = field(default_factory=list)
    gaps: List[np.ndarray] = field(default_factory=list)   # per detector [n_gaps][2] int64
    seed: int = SEED_BASE

    @property
    def n_det(self) -> int:
        return len(self.detectors)


# ----------------------------------------------------------------------------
# Seeded draws
# ----------------------------------------------------------------------------

def streams(index: int, n: int = 6):
    """Independent PCG64 generators for one workload: noise, gaps, injections,
    templates, segments, spare."""
    ss = np.random.SeedSequence(SEED_BASE + index)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def gaussian_noise(rng: np.random.Generator, n: int, sigma2: float) -> np.ndarray:
    """Complex white noise with E|n|^2 = sigma2 (real and imaginary parts each
    N(0, sigma2/2)), as complex64."""
    s = math.sqrt(sigma2 / 2.0)
    out = np.empty(n, dtype=np.complex64)
    out.real = rng.standard_normal(n, dtype=np.float32) * np.float32(s)
    out.imag = rng.standard_normal(n, dtype=np.float32) * np.float32(s)
    return out


def random_gaps(rng: np.random.Generator, n: int, gap_len: int, n_gaps: int,
                max_tries: int = 100000) -> np.ndarray:
    """Non-overlapping, non-adjacent gaps of gap_len samples placed uniformly by
    rejection sampling; returned sorted as half-open [start, end) rows."""
    if n_gaps == 0:
        return np.zeros((0, 2), dtype=np.int64)
    if n_gaps * (gap_len + 1) > n:
        raise ValueError("gaps do not fit in the segment")
    starts: List[int] = []
    tries = 0
    while len(starts) < n_gaps:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("gap placement failed")
        s = int(rng.integers(0, n - gap_len + 1))
        if all(s + gap_len < t or t + gap_len < s for t in starts):
            starts.append(s)
    starts.sort()
    g = np.array([[s, s + gap_len] for s in starts], dtype=np.int64)
    return g


def zero_gaps(x: np.ndarray, gaps: np.ndarray) -> np.ndarray:
    """Zero-fill the gap ranges (the data contract of the input series)."""
    y = x.copy()
    for s, e in gaps:
        y[s:e] = 0
    return y


def uniform_sky(rng: np.random.Generator, n: int) -> np.ndarray:
    """n sky positions (alpha, delta) uniform on the sphere."""
    alpha = rng.uniform(0.0, 2.0 * math.pi, n)
    delta = np.arcsin(rng.uniform(-1.0, 1.0, n))
    return np.stack([alpha, delta], axis=1)


def fdot_grid(n: int, lo: float = -1e-9, hi: float = 0.0) -> np.ndarray:
    """Evenly spaced spindown grid from hi down to lo (n >= 1)."""
    if n == 1:
        return np.array([hi])
    return hi + (lo - hi) * np.arange(n) / (n - 1)


def band_bins(seg: Segment, n_fft: int, f_lo: float, f_hi: float) -> Tuple[int, int]:
    """(first signed bin, number of bins) of the band [f_lo, f_hi) on the
    frequency grid f_het + s / (n_fft dt).  Pure bookkeeping."""
    df = 1.0 / (n_fft * seg.dt)
    s_lo = int(round((f_lo - seg.f_het) / df))
    n_out = int(round((f_hi - f_lo) / df))
    return s_lo, n_out


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

def workload_c1(seed_index: int = 0) -> Workload:
    """Plain method, smallest case: one detector, 1 day at dt = 0.5 s,
    f_het = 100 Hz, one injection, Lanczos-8, 2x zero padding, full 2 Hz band."""
    seg = Segment(n=172800, dt=0.5, t_start=0.0, f_het=100.0)
    inj = Injection(h0=0.05, cosi=0.3, psi=0.4, phi0=1.0, f0=100.25,
                    fdot=-1e-10, alpha=1.2, delta=0.3)
    return Workload(name="C1", detectors=(DET_H,), segment=seg, f_lo=99.0, f_hi=101.0,
                    kernel=KERNEL_LANCZOS, taps=8, nfft_policy=NFFT_TWICE,
                    skies=np.array([[inj.alpha, inj.delta]]), fdots=np.array([inj.fdot]),
                    injections=[inj], gaps=[np.zeros((0, 2), np.int64)],
                    seed=SEED_BASE + seed_index)


def workload_c2(n_fdot: int = 1000) -> Workload:
    """Plain method with gaps: 10 days at dt = 0.25 s (3,456,000 samples),
    f_het = 101 Hz so that the reported band [100, 102) Hz is the central half
    of the 4 Hz data band, 48 half-hour gaps (10 %), four injections, one sky
    position times n_fdot spindowns on [-1e-9, 0] Hz/s, Dirichlet-16."""
    seg = Segment(n=3456000, dt=0.25, t_start=0.0, f_het=101.0)
    r_noise, r_gaps, r_inj, r_tmpl, _, _ = streams(1)
    gaps = random_gaps(r_gaps, seg.n, gap_len=int(1800 / seg.dt), n_gaps=48)
    fd = fdot_grid(n_fdot)
    injs = []
    for _ in range(4):
        injs.append(Injection(h0=0.05, cosi=float(r_inj.uniform(-1, 1)),
                              psi=float(r_inj.uniform(-math.pi / 4, math.pi / 4)),
                              phi0=float(r_inj.uniform(0, 2 * math.pi)),
                              f0=float(r_inj.uniform(100.0, 102.0)),
                              fdot=float(fd[int(r_inj.integers(0, len(fd)))]),
                              alpha=1.2, delta=0.3))
    return Workload(name="C2", detectors=(DET_H,), segment=seg, f_lo=100.0, f_hi=102.0,
                    kernel=KERNEL_DIRICHLET, taps=16, nfft_policy=NFFT_TWICE,
                    skies=np.array([[1.2, 0.3]]), fdots=fd, injections=injs, gaps=[gaps],
                    seed=SEED_BASE + 1)


def c3_segment_lengths(n_seg: int = 64) -> List[int]:
    """Segment lengths of the uneven batched workload: T ~ U[1, 30] days
    rounded to whole 1800 s, at dt = 0.5 s."""
    _, _, _, _, r_seg, _ = streams(2)
    T = r_seg.uniform(1.0, 30.0, n_seg) * DAY
    n_half_hours = np.maximum(1, np.round(T / 1800.0)).astype(int)
    return [int(h * 3600) for h in n_half_hours]


def workload_c3_segment(i: int, n_sky: int = 4096, n_fdot: int = 16) -> Workload:
    """Segment i of the batched uneven workload: 5 % gaps in half-hour blocks,
    4096 sky positions x 16 spindowns, full 2 Hz band, top-10 output."""
    lengths = c3_segment_lengths()
    t0 = float(sum(lengths[:i])) * 0.5
    seg = Segment(n=lengths[i], dt=0.5, t_start=t0, f_het=100.0)
    r_noise, r_gaps, r_inj, r_tmpl, _, _ = streams(2)
    skies = uniform_sky(r_tmpl, n_sky)
    rg = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + 2, i])))
    n_gaps = int(round(0.05 * seg.n / 3600))
    gaps = random_gaps(rg, seg.n, gap_len=3600, n_gaps=n_gaps)
    return Workload(name=f"C3[{i}]", detectors=(DET_H,), segment=seg, f_lo=99.0, f_hi=101.0,
                    kernel=KERNEL_DIRICHLET, taps=16, nfft_policy=NFFT_SMOOTH7_256,
                    skies=skies, fdots=fdot_grid(n_fdot), gaps=[gaps], seed=SEED_BASE + 2)


def workload_c4(storage: int = STORE_F32) -> Workload:
    """Precision study: two detectors (noise variances 1.0 and 1.3), 30 days
    at dt = 0.5 s, 16 sky x 16 spindowns, four injections matched to four of
    the templates in the central 1 Hz, no gaps."""
    seg = Segment(n=5184000, dt=0.5, t_start=0.0, f_het=100.0)
    r_noise, r_gaps, r_inj, r_tmpl, _, _ = streams(3)
    skies = uniform_sky(r_tmpl, 16)
    fd = fdot_grid(16)
    injs = []
    for m in range(4):
        si = int(r_inj.integers(0, 16)); fi = int(r_inj.integers(0, 16))
        injs.append(Injection(h0=0.05, cosi=float(r_inj.uniform(-1, 1)),
                              psi=float(r_inj.uniform(-math.pi / 4, math.pi / 4)),
                              phi0=float(r_inj.uniform(0, 2 * math.pi)),
                              f0=float(r_inj.uniform(99.5, 100.5)), fdot=float(fd[fi]),
                              alpha=float(skies[si, 0]), delta=float(skies[si, 1])))
    return Workload(name="C4", detectors=(DET_H, DET_L), segment=seg, f_lo=99.0, f_hi=101.0,
                    kernel=KERNEL_DIRICHLET, taps=16, nfft_policy=NFFT_TWICE, storage=storage,
                    skies=skies, fdots=fd, injections=injs,
                    gaps=[np.zeros((0, 2), np.int64), np.zeros((0, 2), np.int64)],
                    seed=SEED_BASE + 3)


def workload_c5() -> Workload:
    """Differentiation: one detector, 10 days at dt = 0.5 s, 64 injections."""
    seg = Segment(n=1728000, dt=0.5, t_start=0.0, f_het=100.0)
    r_noise, r_gaps, r_inj, r_tmpl, _, _ = streams(4)
    sk = uniform_sky(r_inj, 64)
    f0s: List[float] = []
    while len(f0s) < 64:
        f = float(r_inj.uniform(99.5, 100.5))
        if all(abs(f - g) >= 1e-3 for g in f0s):
            f0s.append(f)
    injs = [Injection(h0=0.05, cosi=float(r_inj.uniform(-1, 1)),
                      psi=float(r_inj.uniform(-math.pi / 4, math.pi / 4)),
                      phi0=float(r_inj.uniform(0, 2 * math.pi)), f0=f0s[m],
                      fdot=float(r_inj.uniform(-1e-9, 0.0)),
                      alpha=float(sk[m, 0]), delta=float(sk[m, 1])) for m in range(64)]
    return Workload(name="C5", detectors=(DET_H,), segment=seg, f_lo=99.0, f_hi=101.0,
                    kernel=KERNEL_DIRICHLET, taps=16, nfft_policy=NFFT_TWICE,
                    injections=injs, gaps=[np.zeros((0, 2), np.int64)], seed=SEED_BASE + 4)


def c5_candidates(w: Workload, df: float) -> np.ndarray:
    """1024 candidates: each injection offset by the 16 sign corners of
    (+-0.5 df, +-1e-11 Hz/s, +-1e-3 rad, +-1e-3 rad); rows (f, fdot, alpha, delta)."""
    rows = []
    for inj in w.injections:
        for c in range(16):
            s = [1.0 if (c >> b) & 1 else -1.0 for b in range(4)]
            rows.append([inj.f0 + s[0] * 0.5 * df, inj.fdot + s[1] * 1e-11,
                         inj.alpha + s[2] * 1e-3, inj.delta + s[3] * 1e-3])
    return np.array(rows, dtype=np.float64)


def small_workload(n: int = 21600, dt: float = 4.0, f_het: float = 100.0, kernel: int = KERNEL_DIRICHLET,
                   taps: int = 16, n_det: int = 1, t_start: float = 0.0,
                   band: Optional[Tuple[float, float]] = None,
                   nfft_policy: int = NFFT_TWICE) -> Workload:
    """A reduced-size workload for oracle and parity tests (same structure,
    fewer samples)."""
    seg = Segment(n=n, dt=dt, t_start=t_start, f_het=f_het)
    B = 1.0 / dt
    lo, hi = band if band is not None else (f_het - B / 2, f_het + B / 2)
    dets = (DET_H, DET_L)[:n_det]
    return Workload(name=f"small{n}", detectors=dets, segment=seg, f_lo=lo, f_hi=hi,
                    kernel=kernel, taps=taps, nfft_policy=nfft_policy,
                    gaps=[np.zeros((0, 2), np.int64) for _ in dets])


def with_detectors(w: Workload, dets) -> Workload:
    return dataclasses.replace(w, detectors=tuple(dets))


# ----------------------------------------------------------------------------
# Short Fourier transforms (the input of the frequency-domain front end)
# ----------------------------------------------------------------------------

@dataclass
class SftSet:
    """A set of SFT bands of one detector: SFT alpha starts at t_sft[alpha]
    (seconds, same clock as t_start), covers sft_len raw samples of dt_raw,
    and keeps bins k_lo .. k_lo + n_bins - 1 (frequency k / T_sft).  The front
    end turns it into x_h[n_out] at t_start + j / band, heterodyned at f_het."""
    sft_len: int
    dt_raw: float
    k_lo: int
    n_bins: int
    t_sft: np.ndarray
    t_start: float
    f_het: float
    band: float
    n_out: int
    dk: int = 8
    median_window: int = 101
    band_taper: float = 0.05
    edge_taper_s: float = 0.0

    @property
    def t_sft_len(self) -> float:
        return self.sft_len * self.dt_raw


def sft_noise(rng: np.random.Generator, n_sft: int, n_bins: int, power: float) -> np.ndarray:
    """SFT bins of white noise: complex Gaussian with E|X|^2 = power, as
    complex64 [n_sft][n_bins]."""
    return gaussian_noise(rng, n_sft * n_bins, power).reshape(n_sft, n_bins)


def sft_set_c2(n_missing: int = 48, seed_index: int = 6) -> Tuple[SftSet, np.ndarray]:
    """SFT input of the T = 10 d, dt = 0.25 s segment: 480 slots of 1800 s
    (raw rate 256 Hz), n_missing whole SFTs absent (placed uniformly by
    rejection, as the 30-min gaps of the time-domain workload), output band
    4 Hz around f_h = 101 Hz, kept bins covering the band plus the running
    median and Dirichlet margins.  Returns (description, noise bins)."""
    rng = streams(seed_index)[1]
    T_sft, dt_raw = 1800.0, 1.0 / 256.0
    n_slots = 480
    missing = set()
    while len(missing) < n_missing:
        missing.add(int(rng.integers(1, n_slots - 1)))
    t = np.array([a * T_sft for a in range(n_slots) if a not in missing], dtype=np.float64)
    f_het, band = 101.0, 4.0
    dk, w = 8, 101
    margin = w // 2 + dk + 1
    k_lo = int(round((f_het - band / 2) * T_sft)) - margin
    n_bins = int(round(band * T_sft)) + 2 * margin
    sft_len = int(round(T_sft / dt_raw))
    desc = SftSet(sft_len=sft_len, dt_raw=dt_raw, k_lo=k_lo, n_bins=n_bins, t_sft=t, t_start=0.0,
                  f_het=f_het, band=band, n_out=int(round(n_slots * T_sft * band)), dk=dk, median_window=w,
                  band_taper=0.05, edge_taper_s=60.0)
    X = sft_noise(streams(seed_index)[0], len(t), n_bins, float(sft_len))
    return desc, X

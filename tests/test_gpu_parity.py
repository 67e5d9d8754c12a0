"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.

Tolerances (FP32 bulk, FP64 timing/phase/antenna sums):
  t_m,k: 1e-9 s;  a, b: 1e-6 absolute;  z~: 3e-6 of the series rms (measured
  at most 1.0e-6 for Lanczos-8 and Dirichlet-16);
  A', B', C': 1e-10 relative;  mask: exact;
  2F: |delta| <= 1e-4 max(2F_oracle, 4) in every bin.
"""
import dataclasses

import numpy as np
import pytest

from oracle import fstat as of
from paper_0912_4255_amd import synth
from paper_0912_4255_amd.synth import Injection
from tests.helpers import make_inputs, to_gpu, twoF_tol

pytestmark = pytest.mark.gpu


def _small(kernel, taps, n=21600, dt=4.0, n_det=1, gaps=True, policy=synth.NFFT_TWICE, storage=0):
    w = synth.small_workload(n=n, dt=dt, kernel=kernel, taps=taps, n_det=n_det, nfft_policy=policy)
    w = dataclasses.replace(w, storage=storage)
    if gaps:
        rng = np.random.default_rng(5)
        w.gaps = [synth.random_gaps(rng, n, gap_len=n // 40, n_gaps=4) for _ in range(n_det)]
    return w


def _oracle_rs(w, xs, gaps, alpha, delta):
    return [of.resample(x, g, w.segment, alpha, delta, w.eph, d, w.kernel, w.taps)
            for x, g, d in zip(xs, gaps, w.detectors)]


def _inj(w, f_off_bins=3000.5, fdot=-3e-10, alpha=1.2, delta=0.3, h0=2.0):
    df = 1.0 / (2 * w.segment.n * w.segment.dt)
    return Injection(h0=h0, cosi=0.3, psi=0.4, phi0=1.0, f0=w.segment.f_het + f_off_bins * df,
                     fdot=fdot, alpha=alpha, delta=delta)


@pytest.mark.parametrize("kernel,taps,n,dt", [(synth.KERNEL_LANCZOS, 8, 21600, 4.0),
                                               (synth.KERNEL_DIRICHLET, 16, 21600, 4.0),
                                               (synth.KERNEL_DIRICHLET, 16, 172800, 0.5),
                                               (synth.KERNEL_DIRICHLET, 24, 172800, 0.5)])
def test_resample_parity(gpu_lib, kernel, taps, n, dt):
    """Short series, and series long enough (n > 10500 (W/2 + 1)) for the
    Dirichlet weights to reduce to sin(pi x) / (pi x) in FP32."""
    import torch
    w = _small(kernel, taps, n=n, dt=dt)
    xs, gaps = make_inputs(w, seed=1, injections=[_inj(w)])
    sky = np.array([[1.2, 0.3], [4.1, -0.8], [0.3, 1.4]])
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    out = plan.resample(tx, tg, torch.from_numpy(sky).cuda())
    torch.cuda.synchronize()
    for s, (al, de) in enumerate(sky):
        ref = _oracle_rs(w, xs, gaps, al, de)[0]
        o = {k: v[s].cpu().numpy() for k, v in out[0].items()}
        assert np.max(np.abs(o["tm"] - ref["tm"])) < 1e-9
        assert np.max(np.abs(o["u"] - ref["u"])) < 1e-9 / w.segment.dt
        assert np.max(np.abs(o["a"] - ref["a"])) < 1e-6
        assert np.max(np.abs(o["b"] - ref["b"])) < 1e-6
        rms = np.sqrt(np.mean(np.abs(ref["z"]) ** 2))
        zerr = np.max(np.abs(o["z"] - ref["z"])) / rms
        print(f"resample kernel {kernel} W={taps} n={n} sky {s}: max|dz|/rms = {zerr:.2e}", flush=True)
        assert zerr < 3e-6
        bits = np.unpackbits(o["mask"].view(np.uint8), bitorder="little")[: w.segment.n]
        assert np.array_equal(bits.astype(bool), ref["mask"] > 0)
        A, B, Cc = (np.sum(ref["mask"] * ref["a"] ** 2), np.sum(ref["mask"] * ref["b"] ** 2),
                    np.sum(ref["mask"] * ref["a"] * ref["b"]))
        assert np.allclose(o["abc"], [A, B, Cc], rtol=1e-10, atol=0)


@pytest.mark.parametrize("kernel,taps", [(synth.KERNEL_LANCZOS, 8), (synth.KERNEL_DIRICHLET, 16)])
def test_fstat_parity_full_band(gpu_lib, kernel, taps):
    import torch
    w = _small(kernel, taps)
    inj = _inj(w)
    xs, gaps = make_inputs(w, seed=2, injections=[inj])
    sky = np.array([[inj.alpha, inj.delta]])
    fdots = np.array([inj.fdot, 0.0, -1e-9])
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    got = plan.fstat(tx, tg, torch.from_numpy(sky).cuda(), torch.from_numpy(fdots).cuda(),
                     mode=gpu_lib.RSF_MODE_PLAIN)
    got_b = plan.fstat(tx, tg, torch.from_numpy(sky).cuda(), torch.from_numpy(fdots).cuda(),
                       mode=gpu_lib.RSF_MODE_BATCHED)
    torch.cuda.synchronize()
    got, got_b = got.cpu().numpy(), got_b.cpu().numpy()
    assert np.array_equal(got, got_b)           # plain and batched identical
    rss = _oracle_rs(w, xs, gaps, inj.alpha, inj.delta)
    for i, fd in enumerate(fdots):
        ref = of.fstat_band(rss, w.detectors, fd, plan.n_fft, plan.s_lo, plan.n_out)
        assert np.all(np.abs(got[i] - ref) <= twoF_tol(ref)), (i, np.max(np.abs(got[i] - ref) / np.maximum(ref, 4)))
    # the injection is recovered at its bin
    assert abs(int(np.argmax(got[0])) - (3000 - plan.s_lo)) <= 1


def test_fstat_parity_smooth7_ragged(gpu_lib):
    """Uneven length with a 7-smooth FFT length above 2N and a partial band."""
    import torch
    n = 10007
    w = synth.small_workload(n=n, dt=2.0, kernel=synth.KERNEL_LANCZOS, taps=8,
                             nfft_policy=synth.NFFT_SMOOTH7, band=(99.9, 100.13))
    xs, gaps = make_inputs(w, seed=3)
    plan = gpu_lib.Plan(w)
    assert plan.n_fft == 20160 and plan.n_fft > 2 * n
    tx, tg = to_gpu(xs, gaps)
    sky = np.array([[2.5, -0.4], [0.1, 0.9]])
    fd = np.array([-2e-10])
    got = plan.fstat(tx, tg, torch.from_numpy(sky).cuda(), torch.from_numpy(fd).cuda()).cpu().numpy()
    for s in range(2):
        rss = _oracle_rs(w, xs, gaps, *sky[s])
        ref = of.fstat_band(rss, w.detectors, fd[0], plan.n_fft, plan.s_lo, plan.n_out)
        assert np.all(np.abs(got[s] - ref) <= twoF_tol(ref))


def test_fstat_two_detectors(gpu_lib):
    import torch
    w = _small(synth.KERNEL_DIRICHLET, 16, n_det=2, gaps=True)
    inj = _inj(w, alpha=0.7, delta=-0.5)
    xs, gaps = make_inputs(w, seed=4, injections=[inj])
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    sky = np.array([[0.7, -0.5]])
    fd = np.array([inj.fdot, -5e-10])
    got = plan.fstat(tx, tg, torch.from_numpy(sky).cuda(), torch.from_numpy(fd).cuda()).cpu().numpy()
    rss = _oracle_rs(w, xs, gaps, 0.7, -0.5)
    for i in range(2):
        ref = of.fstat_band(rss, w.detectors, fd[i], plan.n_fft, plan.s_lo, plan.n_out)
        assert np.all(np.abs(got[i] - ref) <= twoF_tol(ref))


def test_fstat_four_detectors(gpu_lib):
    """The largest detector set the library takes (4): noise-weighted sums of
    four sites with unequal noise levels against the oracle."""
    import torch
    d3 = synth.Detector(lat=43.63 * synth.DEG, lon=10.50 * synth.DEG, gamma=115.6 * synth.DEG, sigma2=0.8)
    d4 = synth.Detector(lat=36.41 * synth.DEG, lon=137.31 * synth.DEG, gamma=28.3 * synth.DEG, sigma2=2.0)
    w = synth.with_detectors(_small(synth.KERNEL_DIRICHLET, 16, n_det=2, gaps=False),
                             [synth.DET_H, synth.DET_L, d3, d4])
    w.gaps = [np.zeros((0, 2), np.int64)] * 4
    inj = _inj(w, alpha=2.1, delta=0.4)
    xs, gaps = make_inputs(w, seed=8, injections=[inj])
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    fd = np.array([inj.fdot, 0.0])
    got = plan.fstat(tx, tg, torch.tensor([[2.1, 0.4]], dtype=torch.float64).cuda(),
                     torch.from_numpy(fd).cuda()).cpu().numpy()
    rss = _oracle_rs(w, xs, gaps, 2.1, 0.4)
    for i in range(2):
        ref = of.fstat_band(rss, w.detectors, fd[i], plan.n_fft, plan.s_lo, plan.n_out)
        assert np.all(np.abs(got[i] - ref) <= twoF_tol(ref))


def test_length_one_second_pass(gpu_lib):
    """A tiny segment with the whole transform in the first pass (L2 = 1,
    forced): the second pass runs no stage, only the 2F reduction."""
    import torch
    from paper_0912_4255_amd.api import plan_desc_from_workload
    w = _small(synth.KERNEL_LANCZOS, 8, n=1000, dt=4.0)
    xs, gaps = make_inputs(w, seed=9, injections=[_inj(w, f_off_bins=200.5)])
    d = plan_desc_from_workload(w)
    d.fft_l1 = 2000
    plan = gpu_lib.Plan(desc=d)
    assert (plan.fft_l1, plan.fft_l2) == (2000, 1)
    tx, tg = to_gpu(xs, gaps)
    fd = np.array([-3e-10])
    got = plan.fstat(tx, tg, torch.tensor([[1.2, 0.3]], dtype=torch.float64).cuda(),
                     torch.from_numpy(fd).cuda()).cpu().numpy()[0]
    rss = _oracle_rs(w, xs, gaps, 1.2, 0.3)
    ref = of.fstat_band(rss, w.detectors, fd[0], plan.n_fft, plan.s_lo, plan.n_out)
    assert np.all(np.abs(got - ref) <= twoF_tol(ref))


def test_batching_query(gpu_lib):
    w = _small(synth.KERNEL_DIRICHLET, 16)
    plan = gpu_lib.Plan(w)
    assert plan.batching(1, 1000) == (16, 64, 1)
    assert plan.batching(1, 1000, gpu_lib.RSF_MODE_PLAIN) == (1, 1, 1)
    assert plan.batching(8, 16) == (16, 64, 8)
    plan.set_batching(4, 32)
    assert plan.batching(100, 16)[:2] == (4, 32)


def test_c1_full_size(gpu_lib):
    """Workload C1 end to end: every bin of the full 2 Hz band."""
    import torch
    w = synth.workload_c1()
    xs, gaps = make_inputs(w, seed=0, injections=w.injections)
    plan = gpu_lib.Plan(w)
    assert plan.n_fft == 345600 and plan.n_out == 345600
    tx, tg = to_gpu(xs, gaps)
    got = plan.fstat(tx, tg, torch.from_numpy(w.skies).cuda(), torch.from_numpy(w.fdots).cuda())
    got = got.cpu().numpy()[0]
    inj = w.injections[0]
    rss = _oracle_rs(w, xs, gaps, inj.alpha, inj.delta)
    ref = of.fstat_band(rss, w.detectors, inj.fdot, plan.n_fft, plan.s_lo, plan.n_out)
    assert np.all(np.abs(got - ref) <= twoF_tol(ref))


def test_c1_noise_free_peak(gpu_lib):
    """C1's injection (rho^2 ~ 10 in unit noise) without the noise: the
    matched template peaks at f0 = 100.25 Hz, bin 43,200 above f_het."""
    import torch
    w = synth.workload_c1()
    xs, gaps = make_inputs(w, seed=0, injections=w.injections, noise=False)
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    got = plan.fstat(tx, tg, torch.from_numpy(w.skies).cuda(), torch.from_numpy(w.fdots).cuda())
    got = got.cpu().numpy()[0]
    assert int(np.argmax(got)) == 43200 - plan.s_lo
    inj = w.injections[0]
    rss = _oracle_rs(w, xs, gaps, inj.alpha, inj.delta)
    ref = of.fstat_bins(rss, w.detectors, inj.fdot, plan.n_fft, [43200])[0]
    assert abs(got[43200 - plan.s_lo] - ref) <= 1e-4 * max(ref, 4.0)


def test_resample_fraction_rounding_to_one(gpu_lib):
    """A Roemer delay of at most 1e-9 s (an ephemeris with R_E / c = 1e-9 s
    and no orbit) puts most resampled times a hair below a detector sample:
    the fraction u - floor(u) then rounds to 1.0 in FP32, and the
    interpolation must return the next sample (no NaN), as the oracle does.
    Long series, so the sinc form of the Dirichlet weights is the one used."""
    import torch
    w = _small(synth.KERNEL_DIRICHLET, 24, n=172800, dt=0.5, gaps=False)
    w = dataclasses.replace(w, eph=synth.Ephemeris(au_c=0.0, re_c=1e-9))
    xs, gaps = make_inputs(w, seed=3)
    sky = np.array([[1.2, 0.3], [4.1, -0.8]])
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    print("\ncase: resampled fractions rounding to 1 in FP32", flush=True)
    out = plan.resample(tx, tg, torch.from_numpy(sky).cuda())[0]
    for s_, (al, de) in enumerate(sky):
        ref = _oracle_rs(w, xs, gaps, al, de)[0]
        z = out["z"][s_].cpu().numpy()
        assert not np.isnan(z).any()
        rms = np.sqrt(np.mean(np.abs(ref["z"]) ** 2))
        assert np.max(np.abs(z - ref["z"])) / rms < 3e-6

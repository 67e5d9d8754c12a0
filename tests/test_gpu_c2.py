"""GPU parity of the headline search at full size, in the launch configuration
the benchmark times: T = 10 d at dt = 0.25 s (N = 3,456,000, 48 half-hour
gaps), one sky position x 1000 spindowns, Dirichlet-16, N_FFT = 2N, the
2 Hz band of 3,456,000 bins, batched mode with the shipped tuned
factorisation and batching (16 launches of each FFT pass: 15 of 64 templates
and a last one of 40).

The four injections of the workload are added to the noise.  The oracle
resamples the series once (all injections share the sky position) and then
gives:
* every bin of the band for two templates: one inside a full launch (the
  spindown of the second injection) and the very last template of the last,
  partial launch;
* sampled bins (both band edges, 24 seeded bins, the 7 bins around each
  injection's frequency) for the first template and the other injections'
  spindowns.
Tolerance: |delta 2F| <= 1e-4 max(2F_oracle, 4).  Each injection is also
recovered: in its own template the largest 2F within 8 bins of f0 sits on
one of the two bins next to f0.

A second test checks at the same size that the spill's cache policy (non-
temporal when one launch's spill exceeds the last-level cache) changes no
result bit."""
import numpy as np
import pytest

from oracle import fstat as of
from paper_0912_4255_amd import synth
from tests.helpers import make_inputs, to_gpu, twoF_tol

pytestmark = pytest.mark.gpu


def test_c2_full_size_in_the_benchmark_launch_configuration(gpu_lib):
    import torch
    from paper_0912_4255_amd import autotune

    w = synth.workload_c2()
    n_t = len(w.fdots)
    print(f"\ncase: C2 full size, N={w.segment.n}, {n_t} spindowns, batched, tuned plan", flush=True)
    xs, gaps = make_inputs(w, seed=0, injections=w.injections)
    plan, tuned = autotune.tuned_plan(w)
    fb, G, _ = plan.batching(1, n_t)
    assert (fb, G) == (tuned["fb"], tuned["templates"])
    assert plan.n_fft == 2 * w.segment.n and plan.n_out == 3456000
    print(f"plan: {plan.fft_l1}x{plan.fft_l2}, fb{fb}, g{G}", flush=True)

    tx, tg = to_gpu(xs, gaps)
    sky = torch.from_numpy(np.ascontiguousarray(w.skies)).cuda()
    fd = torch.from_numpy(np.ascontiguousarray(w.fdots)).cuda()
    ws = plan.workspace(gpu_lib.RSF_ENTRY_FSTAT, 1, n_t, gpu_lib.RSF_MODE_BATCHED, device="cuda")
    out = torch.empty((n_t, plan.n_out), dtype=torch.float32, device="cuda")
    plan.fstat(tx, tg, sky, fd, mode=gpu_lib.RSF_MODE_BATCHED, out=out, ws=ws)
    torch.cuda.synchronize()

    inj_t = [int(np.flatnonzero(w.fdots == inj.fdot)[0]) for inj in w.injections]
    full_t = [inj_t[1], n_t - 1]
    assert full_t[0] // G < (n_t - 1) // G                # a full launch, then the partial last one
    sampled_t = [0] + [t for t in inj_t if t not in full_t]
    rows = {t: out[t].cpu().numpy() for t in full_t + sampled_t}
    del out, ws
    torch.cuda.empty_cache()

    alpha, delta = w.skies[0]
    rss = [of.resample(xs[0], gaps[0], w.segment, alpha, delta, w.eph, w.detectors[0], w.kernel, w.taps)]
    n_fft, s_lo = plan.n_fft, plan.s_lo
    df = 1.0 / (n_fft * w.segment.dt)
    f_bin = [(inj.f0 - w.segment.f_het) / df for inj in w.injections]

    for t in full_t:
        ref = of.fstat_band(rss, w.detectors, float(w.fdots[t]), n_fft, s_lo, plan.n_out)
        bad = np.abs(rows[t] - ref) > twoF_tol(ref)
        assert not bad.any(), (t, int(np.flatnonzero(bad)[0]), int(bad.sum()))
        print(f"template {t}: every bin within tolerance", flush=True)

    rng = np.random.default_rng(11)
    picks = {0, plan.n_out - 1, *rng.integers(0, plan.n_out, 24).tolist()}
    for b in f_bin:
        picks.update(int(round(b)) - s_lo + d for d in range(-3, 4))
    picks = sorted(p for p in picks if 0 <= p < plan.n_out)
    for t in sampled_t:
        ref = of.fstat_bins(rss, w.detectors, float(w.fdots[t]), n_fft, [s_lo + p for p in picks])
        got = rows[t][picks]
        assert np.all(np.abs(got - ref) <= twoF_tol(ref)), t
        print(f"template {t}: {len(picks)} sampled bins within tolerance", flush=True)

    for t, b in zip(inj_t, f_bin):
        lo = int(np.floor(b)) - 8 - s_lo
        peak = lo + int(np.argmax(rows[t][lo:lo + 18]))
        assert peak + s_lo in (int(np.floor(b)), int(np.floor(b)) + 1), (t, b, peak + s_lo)
        assert rows[t][peak] > 100.0


def test_spill_cache_policy_leaves_results_bitwise_equal(gpu_lib):
    """At T = 10 d a launch of 64 templates spills 7 GB, more than the
    last-level cache, and takes the non-temporal stores and loads; a launch
    of 2 templates (221 MB) is stored and read normally.  Cache hints change
    no arithmetic: 128 templates give bitwise the same 2F both ways."""
    import torch
    w = synth.workload_c2(n_fdot=128)
    print("\ncase: C2 noise, 128 spindowns, batching (16, 64) against (2, 2)", flush=True)
    rng = np.random.default_rng(3)
    x = synth.zero_gaps(synth.gaussian_noise(rng, w.segment.n, 1.0), w.gaps[0])
    tx = [torch.from_numpy(x).cuda()]
    tg = [torch.from_numpy(w.gaps[0]).cuda()]
    sky = torch.from_numpy(np.ascontiguousarray(w.skies)).cuda()
    fd = torch.from_numpy(np.ascontiguousarray(w.fdots)).cuda()
    plan = gpu_lib.Plan(w)
    outs = []
    for fb, g in ((16, 64), (2, 2)):
        plan.set_batching(fb, g)
        outs.append(plan.fstat(tx, tg, sky, fd, mode=gpu_lib.RSF_MODE_BATCHED).cpu())
        torch.cuda.empty_cache()
    assert torch.equal(outs[0], outs[1])
    assert torch.isfinite(outs[0]).all()

"""GPU parity at the shape of the longest uneven segments, in the benchmark's
launch configuration for them: the segment of N = 5,011,200 samples
(T = 29.0 d at dt = 0.5 s, 5 % gaps in half-hour blocks, the 2 Hz band,
N_fft = 10,035,200 = 9800 x 1024, the shipped tuning's 24 taps).  Its first
pass runs the row plan 14 x 10 x 10 x 7 compiled at plan creation; the
top-k's second pass has 1024-point columns, one per wave, with the gate fed
from registers; the map's second pass is the LDS-stage kernel.

Two injections at the segment's first sky position, at spindowns 3 and 11
of 16 (h0 = 0.05 and 0.04).  The oracle resamples once and gives:
* every bin of both injections' rows of the map (rsf_fstat);
* the band edges and 24 seeded bins of two other rows;
* every entry of the top-10 (rsf_fstat_topk over the same 16 templates in
  two launches) at its own key; the first entry is an injection's peak.
Tolerance: |delta 2F| <= 1e-4 max(2F_oracle, 4).  The top-10 is also the
selection over the map to FP32 rounding (the two second passes differ in
their arithmetic)."""
import numpy as np
import pytest

from oracle import fstat as of
from paper_0912_4255_amd import synth
from paper_0912_4255_amd.synth import Injection
from tests.helpers import make_inputs, to_gpu, twoF_tol

pytestmark = pytest.mark.gpu

N_SEG = 5011200


def test_longest_uneven_segment_against_oracle(gpu_lib):
    import torch
    from paper_0912_4255_amd import _lib as L
    from paper_0912_4255_amd import autotune
    lengths = synth.c3_segment_lengths()
    w = synth.workload_c3_segment(lengths.index(N_SEG), n_sky=1)
    (plan,), _ = autotune.segment_plans([w])
    assert (plan.fft_l1, plan.fft_l2) == (9800, 1024) and plan.n_out == plan.n_fft == 10035200
    taps = plan.desc.taps
    n_t = 16
    fd = synth.fdot_grid(n_t)
    alpha, delta = w.skies[0]
    injs = [Injection(h0=0.05, cosi=0.3, psi=0.2, phi0=1.1, f0=99.73, fdot=float(fd[3]), alpha=alpha, delta=delta),
            Injection(h0=0.04, cosi=-0.6, psi=-0.4, phi0=2.5, f0=100.41, fdot=float(fd[11]), alpha=alpha,
                      delta=delta)]
    print(f"\ncase: uneven segment N={w.segment.n}, plan {plan.fft_l1}x{plan.fft_l2}, taps {taps}, "
          f"first pass kind {plan.first_pass}", flush=True)
    xs, gaps = make_inputs(w, seed=7, injections=injs)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.from_numpy(np.ascontiguousarray(w.skies[:1])).cuda()
    tfd = torch.from_numpy(fd).cuda()
    plan.set_batching(16, 8)                               # two launches of 8 templates
    maps = plan.fstat(tx, tg, sky, tfd)
    vals, ids = plan.topk(tx, tg, sky, tfd, k=10)
    vals, ids = vals.cpu().numpy(), ids.cpu().numpy()
    full_t, sampled_t = [3, 11], [0, 15]
    rows = {t: maps[t].cpu().numpy() for t in full_t + sampled_t}
    flat = maps.reshape(-1)
    kth = float(torch.topk(flat, 10).values[-1])
    clear = torch.nonzero(flat > kth + 2e-4 * max(kth, 4.0)).flatten().cpu().numpy()
    del maps, flat
    torch.cuda.empty_cache()

    rss = [of.resample(xs[0], gaps[0], w.segment, alpha, delta, w.eph, w.detectors[0], w.kernel, taps)]
    n_fft, s_lo = plan.n_fft, plan.s_lo
    for t in full_t:
        ref = of.fstat_band(rss, w.detectors, float(fd[t]), n_fft, s_lo, plan.n_out)
        bad = np.abs(rows[t] - ref) > twoF_tol(ref)
        assert not bad.any(), (t, int(np.flatnonzero(bad)[0]), int(bad.sum()))
        print(f"template {t}: every bin within tolerance, peak {ref.max():.1f}", flush=True)
    rng = np.random.default_rng(12)
    picks = sorted({0, plan.n_out - 1, *rng.integers(0, plan.n_out, 24).tolist()})
    for t in sampled_t:
        ref = of.fstat_bins(rss, w.detectors, float(fd[t]), n_fft, [s_lo + p for p in picks])
        assert np.all(np.abs(rows[t][picks] - ref) <= twoF_tol(ref)), t

    # the top-10: every entry against the oracle at its key
    assert np.all(ids[:, 0] == 0) and np.all(np.diff(vals) <= 0)
    for v, (_, f, b) in zip(vals, ids):
        ref = of.fstat_bins(rss, w.detectors, float(fd[f]), n_fft, [s_lo + int(b)])[0]
        assert abs(v - ref) <= twoF_tol(ref), (f, b, v, ref)
    df = 1.0 / (n_fft * w.segment.dt)
    peaks = {t: (inj.f0 - w.segment.f_het) / df - s_lo for t, inj in zip(full_t, injs)}
    assert ids[0, 1] in peaks and abs(ids[0, 2] - peaks[ids[0, 1]]) <= 1.0, (ids[0], peaks)
    # against the map's selection: every map value clearly above the 10th is chosen
    chosen = {int(f) * plan.n_out + int(b) for _, f, b in ids}
    assert all(int(c) in chosen for c in clear)
    assert plan.first_pass == L.RSF_ROWS_RUNTIME
    plan.close()

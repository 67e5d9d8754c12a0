"""Tuning knobs and the autotuner: any accepted factorisation and batching
choice computes the same statistic (bitwise for batching, within the FP32
tolerance against the oracle for factorisations)."""
import numpy as np
import pytest

from oracle import fstat as of
from paper_0912_4255_amd import synth
from tests.helpers import make_inputs, to_gpu, twoF_tol

pytestmark = pytest.mark.gpu


def _setup():
    w = synth.small_workload(n=21600, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16)
    xs, gaps = make_inputs(w, seed=11)
    return w, xs, gaps


def test_batching_knobs_do_not_change_results(gpu_lib):
    import torch
    w, xs, gaps = _setup()
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[1.0, 0.2], [2.0, -0.3]], dtype=torch.float64).cuda()
    fd = torch.from_numpy(synth.fdot_grid(7)).cuda()
    ref = plan.fstat(tx, tg, sky, fd).cpu().numpy()
    for fb, g in [(1, 1), (2, 3), (8, 16), (16, 256)]:
        plan.set_batching(fb, g)
        assert np.array_equal(plan.fstat(tx, tg, sky, fd).cpu().numpy(), ref), (fb, g)


def test_forced_factorisations_match_oracle(gpu_lib):
    import torch
    from paper_0912_4255_amd import autotune
    w, xs, gaps = _setup()
    base = gpu_lib.Plan(w)
    plans = autotune.candidate_l1(base, limit=4)
    assert len(plans) >= 2
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[1.0, 0.2]], dtype=torch.float64).cuda()
    fd = torch.tensor([-3e-10], dtype=torch.float64).cuda()
    rss = [of.resample(xs[0], gaps[0], w.segment, 1.0, 0.2, w.eph, w.detectors[0], w.kernel, w.taps)]
    ref = of.fstat_band(rss, w.detectors, -3e-10, base.n_fft, base.s_lo, base.n_out)
    for p in plans:
        got = p.fstat(tx, tg, sky, fd).cpu().numpy()[0]
        assert np.all(np.abs(got - ref) <= twoF_tol(ref)), (p.fft_l1, p.fft_l2)


@pytest.mark.parametrize("n,l1", [(31360, 7840), (38400, 9600)])
def test_long_first_pass_with_radix7_and_radix3(gpu_lib, n, l1):
    """First-pass lengths 7840 = 16 x 10 x 7 x 7 and 9600 = 10 x 5 x 4 x 4 x 4 x 3,
    whose radix-7 and radix-3 stages run 3 and 7 butterflies per thread."""
    import torch
    from paper_0912_4255_amd.api import plan_desc_from_workload
    w = synth.small_workload(n=n, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16)
    xs, gaps = make_inputs(w, seed=12)
    d = plan_desc_from_workload(w)
    d.fft_l1 = l1
    plan = gpu_lib.Plan(desc=d)
    assert (plan.fft_l1, plan.fft_l2) == (l1, 2 * n // l1)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[0.7, -0.5]], dtype=torch.float64).cuda()
    fd = torch.tensor([-4e-10, 0.0], dtype=torch.float64).cuda()
    got = plan.fstat(tx, tg, sky, fd).cpu().numpy()
    rss = [of.resample(xs[0], gaps[0], w.segment, 0.7, -0.5, w.eph, w.detectors[0], w.kernel, w.taps)]
    for i, f in enumerate((-4e-10, 0.0)):
        ref = of.fstat_band(rss, w.detectors, f, plan.n_fft, plan.s_lo, plan.n_out)
        assert np.all(np.abs(got[i] - ref) <= twoF_tol(ref)), (l1, i)


def test_autotune_and_taps_choice(gpu_lib, tmp_path, monkeypatch):
    from paper_0912_4255_amd import autotune
    monkeypatch.setenv("RSF_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    w, xs, gaps = _setup()
    best = autotune.tune(w, n_fdot=8, reps=1, fbs=(2, 4), templates=(8, 16))
    assert best["fft_l1"] * best["fft_l2"] == 2 * w.segment.n
    assert (tmp_path / "tune.json").exists()
    again = autotune.tune(w)          # served from the cache
    assert again == best
    plan, _ = autotune.tuned_plan(w)
    assert plan.fft_l1 == best["fft_l1"]
    wl = synth.small_workload(n=21600, dt=4.0, kernel=synth.KERNEL_LANCZOS, taps=8)
    W, dev = autotune.choose_taps(wl, candidates=(4, 8, 16), bound=5e-2)
    assert W in (4, 8, 16)
    assert dev[16] <= dev[4]


@pytest.mark.parametrize("n,l1", [(21600, 36), (21600, 40), (21600, 50), (21600, 96), (25088, 98), (21600, 160)])
def test_pruned_first_stage_for_each_even_radix(gpu_lib, n, l1):
    """First-pass lengths whose first (largest) radix is 6, 8, 10, 12, 14 and
    16: the zero upper half of each row is neither written nor read, and the
    first stage runs on the nonzero half only (pruned first stage)."""
    import torch
    from paper_0912_4255_amd.api import plan_desc_from_workload
    w = synth.small_workload(n=n, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16)
    xs, gaps = make_inputs(w, seed=13)
    d = plan_desc_from_workload(w)
    d.fft_l1 = l1
    plan = gpu_lib.Plan(desc=d)
    assert (plan.fft_l1, plan.fft_l2) == (l1, 2 * n // l1)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[2.2, 0.4]], dtype=torch.float64).cuda()
    fd = torch.tensor([-2e-10], dtype=torch.float64).cuda()
    got = plan.fstat(tx, tg, sky, fd).cpu().numpy()[0]
    rss = [of.resample(xs[0], gaps[0], w.segment, 2.2, 0.4, w.eph, w.detectors[0], w.kernel, w.taps)]
    ref = of.fstat_band(rss, w.detectors, -2e-10, plan.n_fft, plan.s_lo, plan.n_out)
    assert np.all(np.abs(got - ref) <= twoF_tol(ref)), l1


@pytest.mark.parametrize("n,l1", [(9262, 125), (8401, 135), (8401, 189), (8193, 343)])
def test_pruned_first_stage_for_each_odd_radix(gpu_lib, n, l1):
    """First-pass lengths 125 = 5^3, 135 = 15 x 9, 189 = 9 x 7 x 3 and
    343 = 7^3 (odd first radix 5, 15, 9, 7) on 7-smooth FFT lengths with
    padding beyond 2N, so that the nonzero rows end below L1/2: the pruned
    first stage reads inputs r < (R + 1)/2 of each radix-R butterfly only,
    and no row at or above ((R + 1)/2) L1/R is written."""
    import torch
    from paper_0912_4255_amd.api import plan_desc_from_workload
    w = synth.small_workload(n=n, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16, nfft_policy=synth.NFFT_SMOOTH7)
    xs, gaps = make_inputs(w, seed=14)
    d = plan_desc_from_workload(w)
    d.fft_l1 = l1
    plan = gpu_lib.Plan(desc=d)
    assert plan.fft_l1 == l1 and 2 * -(-n // plan.fft_l2) <= l1   # rows P <= L1 / 2
    print(f"\ncase: odd first radix, L1 x L2 = {plan.fft_l1} x {plan.fft_l2}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[0.4, -1.1]], dtype=torch.float64).cuda()
    fd = torch.tensor([3e-10], dtype=torch.float64).cuda()
    got = plan.fstat(tx, tg, sky, fd).cpu().numpy()[0]
    rss = [of.resample(xs[0], gaps[0], w.segment, 0.4, -1.1, w.eph, w.detectors[0], w.kernel, w.taps)]
    ref = of.fstat_band(rss, w.detectors, 3e-10, plan.n_fft, plan.s_lo, plan.n_out)
    assert np.all(np.abs(got - ref) <= twoF_tol(ref)), l1


def test_odd_first_pass_at_an_uneven_segment(gpu_lib):
    """A 22.6-day uneven segment (N = 1,951,200, N_fft = 3,919,104): the
    planner's L1 = 5103 = 9 x 9 x 9 x 7 (pruned first stage of radix 9)
    against L1 = 6804 (first radix 12) on the same input, one sky and four
    spindowns: the two full-band 2F maps agree within the parity bar."""
    import torch
    from paper_0912_4255_amd.api import plan_desc_from_workload
    lengths = synth.c3_segment_lengths()
    w = synth.workload_c3_segment(lengths.index(1951200), n_sky=1)
    rng = np.random.default_rng(43)
    x = synth.zero_gaps(synth.gaussian_noise(rng, w.segment.n, 1.0), w.gaps[0])
    tx, tg = to_gpu([x], [w.gaps[0]])
    sky = torch.from_numpy(np.ascontiguousarray(w.skies[:1])).cuda()
    fd = torch.from_numpy(synth.fdot_grid(4)).cuda()
    maps = []
    for l1 in (5103, 6804):
        d = plan_desc_from_workload(w)
        d.fft_l1 = l1
        plan = gpu_lib.Plan(desc=d)
        assert plan.fft_l1 == l1 and plan.n_fft == 3919104
        print(f"\ncase: uneven segment, L1 x L2 = {plan.fft_l1} x {plan.fft_l2}", flush=True)
        maps.append(plan.fstat(tx, tg, sky, fd).cpu().numpy())
        plan.close()
    assert np.all(np.abs(maps[0] - maps[1]) <= twoF_tol(maps[1]))


@pytest.mark.parametrize("n,l1", [(38880, 9720), (36864, 9216), (37632, 9408), (37044, 9261)])
def test_wide_first_pass_stages(gpu_lib, n, l1):
    """First-pass rows of one workgroup per CU whose stages hold up to 32
    complex pairs per thread: 9720 = 12 x 10 x 9 x 9, 9216 = 16 x 9 x 8 x 8,
    9408 = 16 x 12 x 7 x 7 (four stages each, against seven, six and six at
    21 pairs per thread) and 9261 = 9 x 7 x 7 x 7 x 3 (odd, not pruned),
    with 8-point columns in the second pass, full band against the oracle."""
    import torch
    from paper_0912_4255_amd.api import plan_desc_from_workload
    w = synth.small_workload(n=n, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16)
    xs, gaps = make_inputs(w, seed=15)
    d = plan_desc_from_workload(w)
    d.fft_l1 = l1
    plan = gpu_lib.Plan(desc=d)
    assert (plan.fft_l1, plan.fft_l2) == (l1, 2 * n // l1)
    print(f"\ncase: wide first pass, L1 x L2 = {plan.fft_l1} x {plan.fft_l2}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[5.1, 0.9]], dtype=torch.float64).cuda()
    fd = torch.tensor([-1e-9, 2e-10], dtype=torch.float64).cuda()
    got = plan.fstat(tx, tg, sky, fd).cpu().numpy()
    rss = [of.resample(xs[0], gaps[0], w.segment, 5.1, 0.9, w.eph, w.detectors[0], w.kernel, w.taps)]
    for i, f in enumerate((-1e-9, 2e-10)):
        ref = of.fstat_band(rss, w.detectors, f, plan.n_fft, plan.s_lo, plan.n_out)
        assert np.all(np.abs(got[i] - ref) <= twoF_tol(ref)), (l1, i)


@pytest.mark.parametrize("n,l1,policy", [(21600, 96, synth.NFFT_TWICE), (25088, 98, synth.NFFT_TWICE),
                                         (9262, 125, synth.NFFT_SMOOTH7), (31360, 7840, synth.NFFT_TWICE),
                                         (38880, 9720, synth.NFFT_TWICE), (37632, 9408, synth.NFFT_TWICE)])
def test_runtime_row_plans_against_oracle(gpu_lib, monkeypatch, n, l1, policy):
    """Row plans compiled at plan creation (RSF_RTC=all makes them for any
    size): 96 = 12 x 8, 98 = 14 x 7, 125 = 5^3 (odd first radix), 7840 =
    16 x 10 x 7 x 7, 9720 = 12 x 10 x 9 x 9, 9408 = 16 x 12 x 7 x 7; at
    spindown order 1 and, for the last two, order 2 (a second kernel made on
    set_spin_order); full band against the oracle."""
    import torch
    from paper_0912_4255_amd import _lib as L
    from paper_0912_4255_amd.api import plan_desc_from_workload
    monkeypatch.setenv("RSF_RTC", "all")
    w = synth.small_workload(n=n, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16, nfft_policy=policy)
    xs, gaps = make_inputs(w, seed=16)
    d = plan_desc_from_workload(w)
    d.fft_l1 = l1
    plan = gpu_lib.Plan(desc=d)
    assert plan.fft_l1 == l1
    assert plan.first_pass == L.RSF_ROWS_RUNTIME
    print(f"\ncase: run-time row plan, L1 x L2 = {plan.fft_l1} x {plan.fft_l2}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[3.3, -0.2]], dtype=torch.float64).cuda()
    rss = [of.resample(xs[0], gaps[0], w.segment, 3.3, -0.2, w.eph, w.detectors[0], w.kernel, w.taps)]
    fd = torch.tensor([-6e-10], dtype=torch.float64).cuda()
    got = plan.fstat(tx, tg, sky, fd).cpu().numpy()[0]
    ref = of.fstat_band(rss, w.detectors, -6e-10, plan.n_fft, plan.s_lo, plan.n_out)
    assert np.all(np.abs(got - ref) <= twoF_tol(ref)), l1
    if l1 >= 9000:
        plan.set_spin_order(2)
        assert plan.first_pass == L.RSF_ROWS_RUNTIME
        spins = np.array([[-6e-10, 3e-17]])
        got = plan.fstat(tx, tg, sky, torch.from_numpy(spins).cuda()).cpu().numpy()[0]
        ref = of.fstat_band(rss, w.detectors, tuple(spins[0]), plan.n_fft, plan.s_lo, plan.n_out)
        assert np.all(np.abs(got - ref) <= twoF_tol(ref)), (l1, "order 2")
    plan.close()


def test_first_pass_kinds(gpu_lib, monkeypatch):
    """The 10-day row (9000 = 10 x 10 x 10 x 9) runs the compiled-in plan; a
    long uneven segment's row (5103 = 9^3 x 7, N_fft = 3,919,104) a plan
    compiled at plan creation; a short transform the general stages."""
    from paper_0912_4255_amd import _lib as L
    monkeypatch.delenv("RSF_RTC", raising=False)
    from paper_0912_4255_amd import autotune
    plan, _ = autotune.tuned_plan(synth.workload_c2())
    assert plan.fft_l1 == 9000 and plan.first_pass == L.RSF_ROWS_FIXED
    plan.close()
    lengths = synth.c3_segment_lengths()
    w = synth.workload_c3_segment(lengths.index(1951200), n_sky=1)
    from paper_0912_4255_amd.api import plan_desc_from_workload
    d = plan_desc_from_workload(w)
    d.fft_l1 = 5103
    plan = gpu_lib.Plan(desc=d)
    assert plan.first_pass == L.RSF_ROWS_RUNTIME
    plan.close()
    plan = gpu_lib.Plan(synth.small_workload(n=21600, dt=4.0))
    assert plan.first_pass in (L.RSF_ROWS_GENERAL, L.RSF_ROWS_GENERAL_WIDE)
    plan.close()

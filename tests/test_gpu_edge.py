"""Degenerate and boundary cases of the search entry points.

* a segment that is one gap from end to end has A' = B' = C' = 0: every 2F is
  NaN and the degenerate flag is set, in both modes and at continuous points;
* a series of zeros gives 2F = 0 in every bin, exactly, and no flag;
* a band of a single bin (n_out = 1) matches the oracle's direct sum at that
  bin;
* two-detector segments where one detector is entirely gapped reduce to the
  other detector's statistic (the gapped one contributes nothing to the
  integrands or to A', B', C')."""
import numpy as np
import pytest

from oracle import fstat as of
from paper_0912_4255_amd import synth
from tests.helpers import make_inputs, to_gpu, twoF_tol

pytestmark = pytest.mark.gpu

N, DT = 21600, 4.0


def _workload(**kw):
    return synth.small_workload(n=N, dt=DT, kernel=synth.KERNEL_DIRICHLET, taps=16, **kw)


def test_all_gap_segment_is_degenerate(gpu_lib):
    import torch
    w = _workload()
    xs, _ = make_inputs(w, seed=21)
    gaps = [np.array([[0, N]], dtype=np.int64)]
    xs = [synth.zero_gaps(xs[0], gaps[0])]
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[1.0, 0.2], [2.5, -0.7]], dtype=torch.float64).cuda()
    fd = torch.tensor([-1e-10, 0.0, 2e-11], dtype=torch.float64).cuda()
    for mode in (gpu_lib.RSF_MODE_PLAIN, gpu_lib.RSF_MODE_BATCHED):
        ws = plan.workspace(gpu_lib.RSF_ENTRY_FSTAT, 2, 3, mode)
        out = plan.fstat(tx, tg, sky, fd, mode=mode, ws=ws)
        assert torch.isnan(out).all(), mode
        assert plan.flags(ws) & gpu_lib.RSF_FLAG_DEGENERATE, mode
        assert plan.flags(ws) == 0  # reading clears the word
    theta = torch.tensor([[100.01, -1e-10, 1.0, 0.2]], dtype=torch.float64).cuda()
    ws = plan.workspace(gpu_lib.RSF_ENTRY_POINT, 1, 1)
    assert torch.isnan(plan.point(tx, tg, theta, ws=ws)).all()
    assert plan.flags(ws) & gpu_lib.RSF_FLAG_DEGENERATE


def test_zero_series_gives_zero(gpu_lib):
    import torch
    w = _workload()
    gaps = [np.zeros((0, 2), np.int64)]
    xs = [np.zeros(N, np.complex64)]
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[0.3, 1.1]], dtype=torch.float64).cuda()
    fd = torch.tensor([-2e-10, 0.0], dtype=torch.float64).cuda()
    ws = plan.workspace(gpu_lib.RSF_ENTRY_FSTAT, 1, 2)
    out = plan.fstat(tx, tg, sky, fd, ws=ws)
    assert torch.count_nonzero(out).item() == 0
    assert plan.flags(ws) == 0


def test_single_bin_band(gpu_lib):
    import torch
    df = 1.0 / (2 * N * DT)
    s = 1234
    f_lo = 100.0 + s * df
    w = _workload(band=(f_lo, f_lo + df))
    xs, gaps = make_inputs(w, seed=22)
    plan = gpu_lib.Plan(w)
    assert plan.n_out == 1 and plan.s_lo == s
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[1.7, -0.2]], dtype=torch.float64).cuda()
    fd = torch.tensor([-1.5e-10, 3e-11], dtype=torch.float64).cuda()
    got = plan.fstat(tx, tg, sky, fd).cpu().numpy()
    rss = [of.resample(xs[0], gaps[0], w.segment, 1.7, -0.2, w.eph, w.detectors[0], w.kernel, w.taps)]
    for i, f in enumerate((-1.5e-10, 3e-11)):
        ref = of.fstat_bins(rss, w.detectors, f, plan.n_fft, [s])
        assert got.shape == (2, 1)
        assert np.all(np.abs(got[i] - ref) <= twoF_tol(ref)), i


def test_one_detector_fully_gapped(gpu_lib):
    import torch
    w1 = _workload()
    w2 = _workload(n_det=2)
    xs, _ = make_inputs(w2, seed=23)
    full_gap = np.array([[0, N]], dtype=np.int64)
    none = np.zeros((0, 2), np.int64)
    xs2 = [xs[0], synth.zero_gaps(xs[1], full_gap)]
    sky = torch.tensor([[0.9, 0.5]], dtype=torch.float64).cuda()
    fd = torch.tensor([-1e-10], dtype=torch.float64).cuda()
    p1, p2 = gpu_lib.Plan(w1), gpu_lib.Plan(w2)
    tx1, tg1 = to_gpu([xs[0]], [none])
    tx2, tg2 = to_gpu(xs2, [none, full_gap])
    one = p1.fstat(tx1, tg1, sky, fd).cpu().numpy()
    two = p2.fstat(tx2, tg2, sky, fd).cpu().numpy()
    assert np.all(np.abs(two - one) <= twoF_tol(one))

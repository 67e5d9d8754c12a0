"""Per-segment top-k through the candidate gate (order: 2F descending, ties by
the lower (sky, fdot, bin); NaN never enters), against the selection over the
full 2F map computed by the same plan:

* second passes of LB = 256, 512, 768 points select inside the kernel from
  a 2F stage in LDS, LB = 1024 straight from the transform's registers (no
  map either way); other lengths scan a map; all over several FFT
  launches, so the threshold carried from launch to launch is exercised;
* a series of zeros makes every 2F exactly 0: every value ties, every block
  takes its slow path and the result is the k lowest keys;
* an all-gap segment has NaN everywhere: no entry;
* graph replays reproduce the eager result;
* at the T = 10 d shape (two launches of the benchmark's configuration) the
  in-pass top-10 equals the selection over the full map, and at a 26.6-day
  uneven segment (N_fft = 9000 x 1024) it agrees with it to FP32 rounding.

With 1024-point columns the map comes from the LDS-stage second pass and
the top-k from the one-column-per-wave pass, so the two agree to FP32
rounding rather than bit for bit."""
import numpy as np
import pytest

from paper_0912_4255_amd import synth
from tests.helpers import make_inputs, to_gpu
from tests.test_gpu_batch import numpy_topk

pytestmark = pytest.mark.gpu

N, DT = 38400, 4.0      # N_fft = 76800 = 300 x 256 = 150 x 512 = 100 x 768 = 75 x 1024
N_FDOT = 9


def _plan(gpu_lib, w, l1):
    from paper_0912_4255_amd.api import plan_desc_from_workload
    d = plan_desc_from_workload(w)
    d.fft_l1 = l1
    plan = gpu_lib.Plan(desc=d)
    assert plan.fft_l1 == l1
    plan.set_batching(4, 8)    # 8 templates per FFT launch: several launches per call
    return plan


def _expected(maps, k, n_out):
    flat = numpy_topk(maps, k)
    ids = np.stack([flat // (n_out * N_FDOT), (flat // n_out) % N_FDOT, flat % n_out], axis=1)
    return maps.reshape(-1)[flat], ids


def _check_selection(vals, ids, maps, k, exact):
    """The top-k (vals, ids) against the selection over the 2F map `maps`
    [n_sky][n_fdot][n_out].  exact: the map came from the same second-pass
    kernel, so values and keys are identical.  Otherwise (1024-point
    columns: the map pass is the LDS-stage kind, the top-k pass the
    one-column-per-wave kind) the two agree to FP32 rounding: every value
    matches the map at its key, the values descend, and no map value clearly
    above the k-th is missing."""
    n_out = maps.shape[-1]
    if exact:
        ev, ei = _expected(maps, k, n_out)
        assert np.array_equal(ids, ei)
        assert np.array_equal(vals, ev)
        return
    tol = lambda v: 1e-5 * np.maximum(np.abs(v), 4.0)
    at = maps[ids[:, 0], ids[:, 1], ids[:, 2]]
    assert np.all(np.abs(vals - at) <= tol(at)), np.max(np.abs(vals - at))
    assert np.all(np.diff(vals) <= 0)
    assert len({tuple(i) for i in ids}) == k
    ev, _ = _expected(maps, k, n_out)
    assert abs(vals[-1] - ev[-1]) <= tol(ev[-1])
    chosen = np.zeros(maps.shape, bool)
    chosen[ids[:, 0], ids[:, 1], ids[:, 2]] = True
    assert not np.any((maps > vals[-1] + 2 * tol(vals[-1])) & ~chosen)


@pytest.mark.parametrize("l1", [300, 150, 100, 75, 160])
@pytest.mark.parametrize("k", [1, 10, 64])
def test_topk_matches_map_selection(gpu_lib, l1, k):
    import torch
    w = synth.small_workload(n=N, dt=DT, kernel=synth.KERNEL_DIRICHLET, taps=16)
    rng = np.random.default_rng(31)
    w.gaps = [synth.random_gaps(rng, N, 600, 3)]
    xs, gaps = make_inputs(w, seed=32)
    plan = _plan(gpu_lib, w, l1)
    print(f"\ncase: top-{k}, L1 x L2 = {plan.fft_l1} x {plan.fft_l2}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.from_numpy(synth.uniform_sky(np.random.default_rng(33), 3)).cuda()
    fd = torch.from_numpy(synth.fdot_grid(N_FDOT)).cuda()
    maps = plan.fstat(tx, tg, sky, fd).cpu().numpy().reshape(3, N_FDOT, plan.n_out)
    vals, ids = plan.topk(tx, tg, sky, fd, k=k)
    _check_selection(vals.cpu().numpy(), ids.cpu().numpy(), maps, k, exact=plan.fft_l2 != 1024)
    plan.close()


@pytest.mark.parametrize("l1", [150, 75, 160])
def test_all_ties_give_lowest_keys(gpu_lib, l1):
    import torch
    w = synth.small_workload(n=N, dt=DT, kernel=synth.KERNEL_DIRICHLET, taps=16)
    xs = [np.zeros(N, np.complex64)]
    gaps = [np.zeros((0, 2), np.int64)]
    plan = _plan(gpu_lib, w, l1)
    print(f"\ncase: all 2F = 0, L1 = {l1}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.from_numpy(synth.uniform_sky(np.random.default_rng(34), 2)).cuda()
    fd = torch.from_numpy(synth.fdot_grid(N_FDOT)).cuda()
    vals, ids = plan.topk(tx, tg, sky, fd, k=64)
    assert np.all(vals.cpu().numpy() == 0.0)
    exp = np.stack([np.zeros(64, int), np.zeros(64, int), np.arange(64)], axis=1)
    assert np.array_equal(ids.cpu().numpy(), exp)
    plan.close()


@pytest.mark.parametrize("l1", [150, 75, 160])
def test_all_nan_gives_no_entry(gpu_lib, l1):
    import torch
    w = synth.small_workload(n=N, dt=DT, kernel=synth.KERNEL_DIRICHLET, taps=16)
    xs = [np.zeros(N, np.complex64)]
    gaps = [np.array([[0, N]], dtype=np.int64)]
    plan = _plan(gpu_lib, w, l1)
    print(f"\ncase: all 2F NaN, L1 = {l1}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.tensor([[1.0, 0.2]], dtype=torch.float64).cuda()
    fd = torch.from_numpy(synth.fdot_grid(N_FDOT)).cuda()
    vals, ids = plan.topk(tx, tg, sky, fd, k=10)
    assert np.all(np.isneginf(vals.cpu().numpy()))
    assert np.all(ids.cpu().numpy() == -1)
    plan.close()


@pytest.mark.parametrize("l1", [100, 75])
def test_graph_replays_in_pass_topk(gpu_lib, l1):
    import torch
    w = synth.small_workload(n=N, dt=DT, kernel=synth.KERNEL_DIRICHLET, taps=16)
    xs, gaps = make_inputs(w, seed=35)
    plan = _plan(gpu_lib, w, l1)
    print(f"\ncase: graph replays of the in-pass top-k, L1 = {l1}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.from_numpy(synth.uniform_sky(np.random.default_rng(36), 2)).cuda()
    fd = torch.from_numpy(synth.fdot_grid(N_FDOT)).cuda()
    ev, ei = plan.topk(tx, tg, sky, fd, k=20)
    ev, ei = ev.cpu().numpy(), ei.cpu().numpy()
    g, kv, ki = plan.graph_topk(tx, tg, sky, fd, k=20)
    for rep in range(3):
        kv.fill_(-1.0)
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(kv.cpu().numpy(), ev) and np.array_equal(ki.cpu().numpy(), ei), rep
        plan.fstat(tx, tg, sky, fd)  # eager work between replays
        torch.cuda.synchronize()
    g.close()
    plan.close()


def _map_selection(torch, maps, k, n_out, n_fdot):
    """The k best of a 2F map on the GPU: the values at or above the k-th
    largest, ordered by value, then by key."""
    flat = maps.reshape(-1)
    kth = torch.topk(flat, k).values[-1]
    cand = torch.nonzero(flat >= kth).flatten().cpu().numpy()
    v = flat[torch.from_numpy(cand).cuda()].cpu().numpy()
    order = np.lexsort((cand, -v.astype(np.float64)))[:k]
    sel = cand[order]
    return v[order], np.stack([sel // (n_out * n_fdot), (sel // n_out) % n_fdot, sel % n_out], axis=1)


def test_topk_at_a_long_uneven_segment(gpu_lib):
    """A 26.6-day segment of the uneven set (N = 4,593,600, dt = 0.5 s,
    N_fft = 9,216,000 = 9000 x 1024: 1024-point columns, one per wave), one
    sky and 64 spindowns in launches of 32 templates: the in-pass top-10
    agrees with the selection over the full map to FP32 rounding (the map
    comes from the LDS-stage second pass)."""
    import torch
    lengths = synth.c3_segment_lengths()
    i = lengths.index(4593600)
    w = synth.workload_c3_segment(i, n_sky=1)
    from paper_0912_4255_amd.api import plan_desc_from_workload
    d = plan_desc_from_workload(w)
    d.fft_l1 = 9000
    plan = gpu_lib.Plan(desc=d)
    assert (plan.fft_l1, plan.fft_l2) == (9000, 1024)
    plan.set_batching(16, 32)
    rng = np.random.default_rng(41)
    x = synth.zero_gaps(synth.gaussian_noise(rng, w.segment.n, 1.0), w.gaps[0])
    print(f"\ncase: top-10 at N = {w.segment.n}, plan {plan.fft_l1} x {plan.fft_l2}", flush=True)
    tx, tg = to_gpu([x], [w.gaps[0]])
    sky = torch.from_numpy(np.ascontiguousarray(w.skies[:1])).cuda()
    fd = torch.from_numpy(synth.fdot_grid(64)).cuda()
    vals, ids = plan.topk(tx, tg, sky, fd, k=10)
    vals, ids = vals.cpu().numpy(), ids.cpu().numpy()
    maps = plan.fstat(tx, tg, sky, fd).reshape(1, 64, plan.n_out)
    # the selection over the map (the LDS-stage second pass) agrees to FP32 rounding
    ev, ei = _map_selection(torch, maps, 10, plan.n_out, 64)
    tol = 1e-5 * np.maximum(np.abs(ev), 4.0)
    at = maps[0, torch.from_numpy(ids[:, 1]).cuda(), torch.from_numpy(ids[:, 2]).cuda()].cpu().numpy()
    assert np.all(ids[:, 0] == 0) and np.all(np.abs(vals - at) <= tol)
    assert np.all(np.abs(vals - ev) <= tol) and np.all(np.diff(vals) <= 0)
    clear = (ev - ev[-1]) > 2 * tol[-1]          # entries clearly above the 10th must be there
    got = {tuple(i) for i in ids}
    assert all(tuple(e) in got for e in ei[clear]), (ids, ei)
    plan.close()


def test_topk_at_the_ten_day_shape(gpu_lib):
    """The T = 10 d search (N = 3,456,000, N_fft = 6,912,000, one column per
    wave in the second pass), one sky and 96 spindowns in launches of 64
    templates: the in-pass top-10 equals the selection over the full map."""
    import torch
    from paper_0912_4255_amd import autotune
    w = synth.workload_c2()
    xs, gaps = make_inputs(w, seed=5)
    plan, _ = autotune.tuned_plan(w)
    assert plan.fft_l2 in (256, 512, 768)
    print(f"\ncase: top-10 at N = {w.segment.n}, plan {plan.fft_l1} x {plan.fft_l2}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = torch.from_numpy(np.ascontiguousarray(w.skies[:1])).cuda()
    fd = torch.from_numpy(synth.fdot_grid(96)).cuda()
    vals, ids = plan.topk(tx, tg, sky, fd, k=10)
    ev, ei = _map_selection(torch, plan.fstat(tx, tg, sky, fd), 10, plan.n_out, 96)
    assert np.array_equal(ids.cpu().numpy(), ei), (ids, ei)
    assert np.array_equal(vals.cpu().numpy(), ev)
    plan.close()

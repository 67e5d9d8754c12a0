"""The second FFT pass with one column per wave (column lengths LB = 64 E,
E = 4, 8, 12) against the FP64 oracle: forced factorisations that give
LB = 256, 512 and 768, a first-pass length that is not a multiple of 8 (the
last block of eight columns is partly empty), a band narrower than the data
band (only some rows of each column are reported), several sky positions and
spindowns per launch, and the top-k path (2F rows in the workspace)."""
import numpy as np
import pytest

from oracle import fstat as of
from paper_0912_4255_amd import synth
from paper_0912_4255_amd.api import plan_desc_from_workload
from paper_0912_4255_amd.synth import Injection
from tests.helpers import make_inputs, to_gpu, twoF_tol

pytestmark = pytest.mark.gpu


def _plan(gpu_lib, w, l1):
    d = plan_desc_from_workload(w)
    d.fft_l1 = l1
    plan = gpu_lib.Plan(desc=d)
    assert plan.fft_l1 == l1 and plan.fft_l1 * plan.fft_l2 == plan.n_fft
    return plan


@pytest.mark.parametrize("n,l1,band", [(9216, 72, None), (18432, 72, None), (27648, 72, None),
                                       (28800, 75, None), (27648, 72, (100.0 - 0.05, 100.0 + 0.07))])
def test_wave_second_pass_matches_oracle(gpu_lib, n, l1, band):
    import torch
    w = synth.small_workload(n=n, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16, band=band)
    rng = np.random.default_rng(n + l1)
    w.gaps = [synth.random_gaps(rng, n, n // 50, 3)]
    df = 1.0 / (2 * n * w.segment.dt)
    inj = Injection(h0=2.0, cosi=0.3, psi=0.4, phi0=1.0, f0=w.segment.f_het + 401.0 * df, fdot=-3e-10,
                    alpha=1.2, delta=0.3)
    xs, gaps = make_inputs(w, seed=n, injections=[inj])
    plan = _plan(gpu_lib, w, l1)
    print(f"\ncase: n={n} L1={l1} L2={plan.fft_l2} band={band}", flush=True)
    tx, tg = to_gpu(xs, gaps)
    sky = np.array([[1.2, 0.3], [3.1, -0.9]])
    fdot = np.array([-3e-10, 0.0, 2e-10])
    got = plan.fstat(tx, tg, torch.from_numpy(sky).cuda(), torch.from_numpy(fdot).cuda()).cpu().numpy()
    err = 0.0
    for si in range(2):
        rss = [of.resample(xs[0], gaps[0], w.segment, *sky[si], w.eph, w.detectors[0], w.kernel, w.taps)]
        for fi in range(3):
            ref = of.fstat_band(rss, w.detectors, fdot[fi], plan.n_fft, plan.s_lo, plan.n_out)
            err = max(err, float(np.max(np.abs(got[si * 3 + fi] - ref) / np.maximum(ref, 4.0))))
            assert np.all(np.abs(got[si * 3 + fi] - ref) <= twoF_tol(ref)), (si, fi)
    print(f"max |d2F| / max(2F, 4) = {err:.2e}", flush=True)
    # plain (one template per launch) gives the same bits as batched
    pl = plan.fstat(tx, tg, torch.from_numpy(sky).cuda(), torch.from_numpy(fdot).cuda(),
                    mode=gpu_lib.RSF_MODE_PLAIN).cpu().numpy()
    assert np.array_equal(pl, got)
    # the top-k path reads the same 2F from its rows in the workspace
    vals, ids = plan.topk(tx, tg, torch.from_numpy(sky).cuda(), torch.from_numpy(fdot).cuda(), k=5)
    vals, ids = vals.cpu().numpy(), ids.cpu().numpy()
    flat = got.reshape(2, 3, -1)
    for v, (s, f, b) in zip(vals, ids):
        assert v == flat[s, f, b]
    assert vals[0] == got.max()
    plan.close()

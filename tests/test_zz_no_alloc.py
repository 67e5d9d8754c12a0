"""The no-allocation entry rsf_fstat_backward_static against
rsf_fstat_backward (same kernels, static device scratch instead of the
caller's workspace): identical 2F and gradients on two calls in a row, the
second with fewer candidates, then on a shorter segment; a candidate count
whose scratch exceeds the static array is refused before any launch."""
import numpy as np
import pytest

from paper_0912_4255_amd import synth
from paper_0912_4255_amd.synth import Injection
from tests.helpers import make_inputs, to_gpu

pytestmark = pytest.mark.gpu


def _case(gpu_lib, n, seed):
    import torch
    w = synth.small_workload(n=n, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16)
    rng = np.random.default_rng(seed)
    w.gaps = [synth.random_gaps(rng, n, n // 40, 3)]
    df = 1.0 / (2 * n * w.segment.dt)
    inj = Injection(h0=1.5, cosi=0.2, psi=-0.3, phi0=2.0, f0=w.segment.f_het + 1200.3 * df, fdot=-4e-10,
                    alpha=2.1, delta=-0.4)
    xs, gaps = make_inputs(w, seed=seed, injections=[inj])
    th = np.array([[inj.f0 + o * df, inj.fdot + 1e-12 * o, inj.alpha + 1e-4 * o, inj.delta - 1e-4 * o]
                   for o in (0.0, 0.3, -0.45, 1.1, 2.0, -3.0)])
    plan = gpu_lib.Plan(w)
    tx, tg = to_gpu(xs, gaps)
    return plan, tx, tg, torch.from_numpy(th).cuda()


def test_static_scratch_backward_matches_workspace_entry(gpu_lib):
    import torch
    print("\ncase: rsf_fstat_backward_static, n=21600 then fewer candidates, then n=10800", flush=True)
    plan, tx, tg, th = _case(gpu_lib, 21600, 5)
    g_in = torch.tensor([1.0, -0.5, 2.0, 0.25, 1.5, -1.0], dtype=torch.float32).cuda()
    F_ref, g_ref = plan.backward(tx, tg, th, g_in)
    F_s, g_s = plan.backward_static(tx, tg, th, g_in)
    torch.cuda.synchronize()
    assert torch.equal(F_s, F_ref) and torch.equal(g_s, g_ref)
    # a second call in a row with a smaller input: the first three candidates
    th3, g3 = th[:3].contiguous(), g_in[:3].contiguous()
    F_s3, g_s3 = plan.backward_static(tx, tg, th3, g3)
    F_r3, g_r3 = plan.backward(tx, tg, th3, g3)
    torch.cuda.synchronize()
    assert torch.equal(F_s3, F_r3) and torch.equal(g_s3, g_r3)
    assert torch.equal(F_s3, F_ref[:3]) and torch.equal(g_s3, g_ref[:3])
    # a shorter segment on another plan shares the same array
    plan2, tx2, tg2, th2 = _case(gpu_lib, 10800, 6)
    F_a, g_a = plan2.backward_static(tx2, tg2, th2[:2].contiguous(), g_in[:2].contiguous())
    F_b, g_b = plan2.backward(tx2, tg2, th2[:2].contiguous(), g_in[:2].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(F_a, F_b) and torch.equal(g_a, g_b)
    # more candidates than the static array holds: refused, nothing launched
    big = th[:1].repeat(65535, 1).contiguous()
    with pytest.raises(gpu_lib.RsfError, match="static"):
        plan.backward_static(tx, tg, big, torch.ones(65535, dtype=torch.float32).cuda())
    plan.close()
    plan2.close()

"""Time-domain front end on the GPU against the oracle (paper Sec. III.A.1).

Bar: |x_gpu - x_oracle| <= 1e-4 max|x_oracle| (FP32 sums over L taps of an
FP64-built filter; heterodyne phases in FP64).  Cases: no filter (D = 1,
K = 0), the 995 Hz worked example (D = 100), a ragged last tile, the
matrix-core form (D = 64, K = 8, 12, 16) over several workgroups, and the
full T = 10 d series at 256 Hz (221,184,000 raw samples, D = 64, 2049 taps)
sampled at 256 outputs."""
import numpy as np
import pytest

from oracle import heterodyne as oh

pytestmark = pytest.mark.gpu


def _run(gpu_lib, x, dt, fh, D, K, beta, n_out):
    import torch
    plan = gpu_lib.HetdecPlan(len(x), dt, fh, D, K, beta, n_out)
    out = plan.run(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("dt,fh,D,K,n_raw,n_out", [
    (1.0 / 64.0, 10.3, 1, 0, 5000, 5000),          # heterodyne only
    (1.0 / 1000.0, 995.0, 100, 12, 40000, 400),     # the worked example's rates
    (1.0 / 256.0, 100.0, 32, 12, 256 * 37 + 11, 300),  # ragged: 300 outputs, the last tile partial
    (1.0 / 256.0, 101.0, 64, 8, 256 * 80 + 5, 320),     # matrix-core form (D = 64): 2 workgroups, ragged
    (1.0 / 256.0, 101.0, 64, 12, 64 * 700 + 3, 650),    # matrix-core form, K = 12: 3 workgroups
    (1.0 / 256.0, 101.0, 64, 16, 256 * 80, 300),        # matrix-core form, 2049 taps
])
def test_matches_oracle(gpu_lib, dt, fh, D, K, n_raw, n_out):
    rng = np.random.default_rng(D + K)
    t = np.arange(n_raw) * dt
    x = (rng.standard_normal(n_raw) + 2.0 * np.cos(2 * np.pi * (fh + 0.1 / (D * dt)) * t + 0.3)).astype(np.float32)
    ref = oh.heterodyne_decimate(x.astype(np.float64), dt, fh, D, K, 8.0, n_out)
    got = _run(gpu_lib, x, dt, fh, D, K, 8.0, n_out)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"hetdec D={D} K={K}: max|d| / max|x| = {err:.2e}", flush=True)
    assert err <= 1e-4


def test_ten_day_series_sampled(gpu_lib):
    import torch
    dt, fh, D, K = 1.0 / 256.0, 101.0, 64, 16
    n_raw = 256 * 864000
    rng = np.random.default_rng(11)
    x = rng.standard_normal(n_raw, dtype=np.float32)
    n_out = n_raw // D
    plan = gpu_lib.HetdecPlan(n_raw, dt, fh, D, K, 8.0, n_out)
    got = plan.run(torch.from_numpy(x).cuda()).cpu().numpy()
    plan.close()
    js = np.concatenate([[0, 1, 2, n_out - 2, n_out - 1], rng.integers(0, n_out, 251)])
    ref = oh.heterodyne_decimate_at(x, dt, fh, D, K, 8.0, js)
    err = np.max(np.abs(got[js] - ref)) / np.max(np.abs(ref))
    print(f"hetdec 10 d: max|d| / max|x| over {len(js)} samples = {err:.2e}", flush=True)
    assert err <= 1e-4
    assert np.all(np.isfinite(got))

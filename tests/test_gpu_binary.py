"""Sources in circular binary orbits on the GPU against the oracle.

Bars as for isolated sources: the total delay d (stored t_m) within 1e-9 s,
a, b within 1e-6, z~ within 2e-5 of the series rms, the SSB mask exact, A',
B', C' to 1e-10; full-band 2F within 1e-4 max(2F, 4).  Orbit: a_p = 1.44
light-s, P_b = 68,023.7 s (2 pi a_p / P_b = 1.3e-4), segment starting at
1e5 s; an orbit of a_p = 0 must equal the isolated source."""
import numpy as np
import pytest

from oracle import fstat as of
from paper_0912_4255_amd import synth
from paper_0912_4255_amd.synth import Binary, Injection
from tests.helpers import make_inputs, to_gpu, twoF_tol

pytestmark = pytest.mark.gpu

ORBITS = [Binary(1.44, 68023.7, 2.3e4), Binary(0.6, 40000.0, 9.0e4)]


def _setup(seed, injections=()):
    w = synth.small_workload(n=21600, dt=4.0, kernel=synth.KERNEL_DIRICHLET, taps=16, t_start=1.0e5)
    rng = np.random.default_rng(seed)
    w.gaps = [synth.random_gaps(rng, w.segment.n, 500, 3)]
    xs, gaps = make_inputs(w, seed=seed, injections=list(injections))
    return w, xs, gaps


def _sky_rows(sky, orbits):
    return np.array([[a, d, o.a_p, o.p_orb, o.t_asc] for (a, d), o in zip(sky, orbits)])


def test_resample_parity_binary(gpu_lib):
    import torch
    w, xs, gaps = _setup(1)
    sky = [(1.2, 0.3), (4.1, -0.8)]
    plan = gpu_lib.Plan(w)
    plan.set_binary(True)
    tx, tg = to_gpu(xs, gaps)
    out = plan.resample(tx, tg, torch.from_numpy(_sky_rows(sky, ORBITS)).cuda())
    torch.cuda.synchronize()
    for s, ((al, de), orb) in enumerate(zip(sky, ORBITS)):
        ref = of.resample(xs[0], gaps[0], w.segment, al, de, w.eph, w.detectors[0], w.kernel, w.taps, binary=orb)
        o = {k: v[s].cpu().numpy() for k, v in out[0].items()}
        assert np.max(np.abs(o["tm"] - ref["tm"])) < 1e-9
        assert np.max(np.abs(o["a"] - ref["a"])) < 1e-6
        assert np.max(np.abs(o["b"] - ref["b"])) < 1e-6
        rms = np.sqrt(np.mean(np.abs(ref["z"]) ** 2))
        err = np.max(np.abs(o["z"] - ref["z"])) / rms
        print(f"binary resample sky {s}: max|dz|/rms = {err:.2e}", flush=True)
        assert err < 2e-5
        bits = np.unpackbits(o["mask"].view(np.uint8), bitorder="little")[: w.segment.n]
        assert np.array_equal(bits.astype(bool), ref["mask"] > 0)
        A, B, C = (np.sum(ref["mask"] * ref["a"] ** 2), np.sum(ref["mask"] * ref["b"] ** 2),
                   np.sum(ref["mask"] * ref["a"] * ref["b"]))
        assert np.allclose(o["abc"], [A, B, C], rtol=1e-10, atol=0)
    plan.close()


def test_fstat_parity_and_recovery_binary(gpu_lib):
    import torch
    df = 1.0 / (2 * 21600 * 4.0)
    orb = ORBITS[0]
    inj = Injection(h0=2.0, cosi=0.3, psi=0.2, phi0=1.0, f0=100.0 + 2800 * df, fdot=-2e-10, alpha=1.2, delta=0.3,
                    binary=orb)
    w, xs, gaps = _setup(2, [inj])
    rows = _sky_rows([(1.2, 0.3), (1.2, 0.3)], [orb, Binary(0.0, orb.p_orb, orb.t_asc)])
    fdots = np.array([-2e-10, 0.0])
    plan = gpu_lib.Plan(w)
    plan.set_binary(True)
    tx, tg = to_gpu(xs, gaps)
    ts, tf = torch.from_numpy(rows).cuda(), torch.from_numpy(fdots).cuda()
    got = plan.fstat(tx, tg, ts, tf).cpu().numpy()
    for si, orbit in enumerate((orb, None)):
        rs = [of.resample(xs[0], gaps[0], w.segment, 1.2, 0.3, w.eph, w.detectors[0], w.kernel, w.taps,
                          binary=orbit)]
        for fi in range(2):
            ref = of.fstat_band(rs, w.detectors, fdots[fi], plan.n_fft, plan.s_lo, plan.n_out)
            assert np.all(np.abs(got[si * 2 + fi] - ref) <= twoF_tol(ref)), (si, fi)
    # the matched orbit finds the injection at its bin; without the orbit it is spread out
    assert int(np.argmax(got[0])) == 2800 - plan.s_lo
    assert got[0].max() > 10 * got[2].max() / 2
    vals, ids = plan.topk(tx, tg, ts, tf, k=3)
    assert tuple(ids.cpu().numpy()[0]) == (0, 0, 2800 - plan.s_lo)
    theta = torch.tensor([[inj.f0, inj.fdot, 1.2, 0.3]], dtype=torch.float64).cuda()
    with pytest.raises(Exception, match="isolated sources only"):
        plan.point(tx, tg, theta)
    with pytest.raises(ValueError):
        plan.fstat(tx, tg, ts[:, :2].contiguous(), tf)
    plan.close()

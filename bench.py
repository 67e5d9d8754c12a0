"""Benchmark: F-statistic templates/s at T = 10 d over a 2 Hz band on one GPU.

Workload (synthetic, seeded): one detector, T = 864,000 s at dt = 0.25 s
(N = 3,456,000 complex64 samples, 10 % of them in 48 zero-filled half-hour
gaps), heterodyned at 101 Hz, Dirichlet-16 interpolation, N_fft = 6,912,000,
2F reported on [100, 102) Hz (3,456,000 bins), one sky position x 1000
spindowns on [-1e-9, 0] Hz/s.  Unit-variance Gaussian noise; injected
signals do not change the work and are left out.

A step is the whole hot path over that batch: resampling for the sky
position, the antenna sums, and for every spindown the demodulation, both
zero-padded FFTs and the 2F reduction of every bin (batched mode), captured
once into a HIP graph and replayed.  Inputs are resident in HBM before the
timed region; the timed region is exactly `--steps` replays between two
device synchronisations, with no per-kernel instrumentation inside it.
After it, replays continue until at least 5 of them and 10 s have been
timed one by one (hipEvents around each replay) and their median is
reported; then a separate instrumented pass of the same launches gives the
per-kernel durations (hipEvents on the launch stream) for the roofline.

The CPU oracle runs first, before anything touches the GPU, on bounded
samples of the same workload: one thread, all host cores (one process per
core, forked), and the oracle's finite-difference gradient of one candidate
of the gradient workload.

Printed: one JSON line with templates/s (whole job), the per-template plain
rate, the roofline of the dominant kernel and of the whole path, a measured
device-to-device copy bandwidth, and the CPU baselines.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-fdot", type=int, default=1000)
    ap.add_argument("--plain-templates", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-templates", type=int, default=2)
    ap.add_argument("--copy-check", action="store_true",
                    help="accepted for older profiling commands; the 1 GiB copy now always runs")
    ap.add_argument("--no-autotune", action="store_true", help="use the planner's default configuration")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient workload")
    ap.add_argument("--grad-candidates", type=int, default=1024)
    ap.add_argument("--no-c3", action="store_true", help="skip the uneven-segment batched search")
    ap.add_argument("--no-sft", action="store_true", help="skip the SFT front end")
    ap.add_argument("--no-hetdec", action="store_true", help="skip the time-domain front end")
    ap.add_argument("--c3-segments", type=int, default=64)
    ap.add_argument("--c3-sky", type=int, default=8)
    ap.add_argument("--replay-seconds", type=float, default=10.0,
                    help="time replays one by one for at least this long (0: only --replay-min replays)")
    ap.add_argument("--replay-min", type=int, default=5)
    return ap.parse_args()


KERNEL_SOURCES = ("rsf_fft.hip", "rsf_pass_a.h", "rsf_spill.h", "rsf_topk_gate.h", "rsf_device.h", "rsf_params.h",
                  "rsf_resample.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_fft_T10d.md")
PEAK_FP32_MFMA_TFLOPS = 157.3  # MI355X dense FP32 matrix
# Vector-instruction issue: 256 CUs x 4 SIMDs, one wave64 VALU instruction per
# SIMD every 4 cycles at 2.4 GHz (FP64 and unpacked FP32 alike).
PEAK_VALU_ISSUE_G = 256 * 4 * 2.4 / 4  # 614.4 G wave instructions/s
POINT_SOURCES = ("rsf_point.hip", "rsf_point_params.h", "rsf_device.h", "rsf_params.h")
POINT_COUNTS_FILE = os.path.join(ROOT, "profiles", "pmc_point_grad_T10d.md")


def kernel_source_hash(names=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_0912_4255_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel, config):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel calibration),
    or None when the summary is missing, was taken on another configuration,
    or the kernel sources have changed since."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    src = kernel_source_hash()
    for ln in lines:
        f = ln.strip().strip("`").split()
        # traffic <kernel> <bytes per launch> src=<hash> cfg=<L1>x<L2>,fb<fb>,g<G>
        if len(f) == 5 and f[0] == "traffic" and f[1] == kernel and f[3] == "src=" + src and f[4] == "cfg=" + config:
            return float(f[2])
    return None


def committed_point_valu(config):
    """VALU wave instructions per candidate of the gradient point kernel from
    the committed counter summary (SQ_INSTS_VALU), or None when it is missing,
    was taken on another configuration, or the point kernel's sources have
    changed since."""
    try:
        lines = open(POINT_COUNTS_FILE).read().splitlines()
    except OSError:
        return None
    src = kernel_source_hash(POINT_SOURCES)
    for ln in lines:
        f = ln.strip().strip("`").split()
        # valu_per_candidate rsf_point_k <instructions> src=<hash> cfg=<config>
        if len(f) == 5 and f[0] == "valu_per_candidate" and f[3] == "src=" + src and f[4] == "cfg=" + config:
            return float(f[2])
    return None


def host_info():
    """Host cores available to this process and the CPU model name."""
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count() or 1
    return {"nproc": avail, "cpu_count": os.cpu_count(), "model": model}


# state shared with forked oracle workers (set before the pool starts)
_CPU = {}


def _one_thread():
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(limits=1)
    except ImportError:  # pragma: no cover
        import contextlib
        return contextlib.nullcontext()


def _cpu_template(i):
    from oracle import fstat as of
    c = _CPU
    with _one_thread():
        t0 = time.perf_counter()
        of.fstat_band(c["rss"], c["dets"], float(c["fdots"][i]), c["n_fft"], c["s_lo"], c["n_out"])
        return time.perf_counter() - t0


def _cpu_grad_component(i):
    from oracle import grad as og
    c = _CPU
    with _one_thread():
        t0 = time.perf_counter()
        prob = og.PointProblem(c["gx"], c["ggaps"], c["gseg"], c["gdets"], c["geph"], c["gkernel"], c["gtaps"])
        g1 = og.central(prob.twoF, c["gtheta"], i, c["gsteps"][i])
        g2 = og.central(prob.twoF, c["gtheta"], i, c["gsteps"][i] / 2.0)
        return (4.0 * g2 - g1) / 3.0, time.perf_counter() - t0


def cpu_baseline(w, x, gaps, n_templates, n_step, synth):
    """The FP64 oracle, as it stands, on bounded samples, before the GPU is
    touched: (1) one thread: resampling for the sky position, then
    n_templates full-band templates; (2) one forked process per host core
    (at most 16), each one full-band template from the same resampled
    series; (3) the oracle's Richardson finite-difference gradient of one
    candidate of the gradient workload, its four components in four
    processes.  Rates are scaled to a step of n_step templates: one
    resampling plus n_step templates at the measured per-template time."""
    import multiprocessing as mp

    from oracle import fstat as of
    from oracle import grad as og
    host = host_info()
    with _one_thread():
        t0 = time.perf_counter()
        alpha, delta = w.skies[0]
        rss = of.resample_all([x], [gaps], w.segment, alpha, delta, w.eph, w.detectors, w.kernel, w.taps)
        t_rs = time.perf_counter() - t0
        n_fft = of.fft_length(w.segment.n, w.nfft_policy)
        df = 1.0 / (n_fft * w.segment.dt)
        s_lo = int(round((w.f_lo - w.segment.f_het) / df))
        n_out = int(round((w.f_hi - w.f_lo) / df))
        t1 = time.perf_counter()
        for i in range(n_templates):
            of.fstat_band(rss, w.detectors, float(w.fdots[i]), n_fft, s_lo, n_out)
        t_tp = (time.perf_counter() - t1) / n_templates
    single = {"templates_per_s": n_step / (t_rs + n_step * t_tp), "resample_s": round(t_rs, 2),
              "template_s": round(t_tp, 2), "templates": n_templates, "cores": 1}

    # all cores: one template per forked worker (workers only run numpy)
    P = max(1, min(16, host["nproc"]))
    _CPU.update(rss=rss, dets=w.detectors, fdots=w.fdots, n_fft=n_fft, s_lo=s_lo, n_out=n_out)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        per = pool.map(_cpu_template, range(P))
    wall = time.perf_counter() - t0
    multi = {"templates_per_s": n_step / (t_rs + n_step * wall / P), "cores": P, "templates": P,
             "wall_s": round(wall, 2), "mean_template_s": round(float(np.mean(per)), 2)}

    # gradient workload: one candidate, the oracle's FD gradient over 4 processes
    gw = synth.workload_c5()
    gx = synth.gaussian_noise(synth.streams(4)[5], gw.segment.n, 1.0)
    gdf = 1.0 / (2 * gw.segment.n * gw.segment.dt)
    _CPU.update(gx=[gx], ggaps=[np.zeros((0, 2), np.int64)], gseg=gw.segment, gdets=list(gw.detectors),
                geph=gw.eph, gkernel=gw.kernel, gtaps=gw.taps, gtheta=synth.c5_candidates(gw, gdf)[0],
                gsteps=og.default_steps(gw.segment))
    t0 = time.perf_counter()
    with ctx.Pool(4) as pool:
        res = pool.map(_cpu_grad_component, range(4))
    gwall = time.perf_counter() - t0
    gcpu = float(sum(t for _, t in res))
    grad = {"candidates_per_s": round(1.0 / gcpu, 5), "s_per_candidate_one_core": round(gcpu, 2),
            "wall_s_4_cores": round(gwall, 2),
            "sample": "T=10d dt=0.5s N=1728000 workload, one candidate, Richardson central differences "
                      "(8 evaluations of 2F per component, the series re-resampled for each sky offset)"}
    _CPU.clear()
    return {"value": multi["templates_per_s"], "unit": "templates/s", "cores": P, "kind": "oracle",
            "sample": f"T=10d workload, numpy FP64: resampling of 1 sky position ({t_rs:.1f} s, one thread), "
                      f"then {P} full-band templates in {P} forked single-thread processes ({wall:.1f} s wall); "
                      f"rate for a step of {n_step} templates = {n_step} / (resampling + {n_step} x wall / {P})",
            "host": host, "single_thread": single, "all_cores": multi, "gradient": grad}


def grad_leg(rsf, synth, torch, dev, n_cand, steps=20):
    """Gradient workload: T = 10 d at dt = 0.5 s (N = 1,728,000), n_cand
    candidates spread around 64 points; forward 2F plus the hand-written
    adjoint per candidate (candidates/s), and 20 gradient-ascent steps."""
    w = synth.workload_c5()
    rng = synth.streams(4)[5]
    x = synth.gaussian_noise(rng, w.segment.n, 1.0)
    plan = rsf.Plan(w)
    tx = [torch.from_numpy(x).to(dev)]
    theta = torch.from_numpy(synth.c5_candidates(w, plan.df)[:n_cand]).to(dev)
    g1 = torch.ones(theta.shape[0], dtype=torch.float32, device=dev)
    ws = plan.workspace(rsf.RSF_ENTRY_BACKWARD, 1, theta.shape[0], device=dev)
    plan.backward(tx, [None], theta, g1, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F, g = plan.backward(tx, [None], theta, g1, ws=ws)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    T0 = w.segment.n * w.segment.dt
    scale = torch.tensor([1 / T0, 1 / T0 ** 2, 1e-5, 1e-5], dtype=torch.float64, device=dev)
    step = torch.tensor([1e-3 / T0, 1e-3 / T0 ** 2, 1e-7, 1e-7], dtype=torch.float64, device=dev)
    th = theta.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        F, g = plan.backward(tx, [None], th, g1, ws=ws)
        gs = g * scale
        th = th + step * gs / gs.abs().amax(dim=1, keepdim=True).clamp_min(1e-30)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    # the point kernel's own duration (HIP events on the launch stream), and
    # its vector-issue rate from the committed instruction count
    plan.profile(True)
    plan.profile_read()
    plan.backward(tx, [None], theta, g1, ws=ws)
    prof = plan.profile_read()
    plan.profile(False)
    n_c = int(theta.shape[0])
    launches, ms = prof["rsf_point_k"]
    k_s = ms * 1e-3 / launches
    cfg = f"N{w.segment.n},grad,order1"
    per_cand = committed_point_valu(cfg)
    roof = {"bound": "alu", "kernel": "rsf_point_k", "avg_launch_us": round(k_s * 1e6, 1),
            "unit": "G VALU wave-instructions/s", "peak": PEAK_VALU_ISSUE_G, "config": cfg,
            "kernel_src": kernel_source_hash(POINT_SOURCES), "achieved": None, "frac": None}
    if per_cand is not None:
        rate = per_cand * n_c / k_s / 1e9
        roof.update(achieved=round(rate, 1), frac=round(rate / PEAK_VALU_ISSUE_G, 4),
                    valu_per_launch=per_cand * n_c)
    return {"workload": "T=10d dt=0.5s N=1728000, Dirichlet-16, synthetic noise",
            "candidates": n_c,
            "candidates_per_s": round(n_c / t_one, 1),
            "refine_steps": steps, "refine_s": round(t_steps, 4),
            "roofline": roof}


def c3_leg(rsf, synth, torch, dev, n_seg, n_sky, n_fdot=16, k=10, reps=3):
    """Uneven segments: the first n_seg of the 64 segments (T_i ~ U[1, 30] d,
    dt = 0.5 s, 5 % gaps, 7-smooth FFT lengths), n_sky sky positions x 16
    spindowns each, per-segment top-10, every segment with its own tuned
    taps, factorisation and batching, all segments in one HIP graph of the
    multi-segment entry (rsf_fstat_topk_segments), replayed."""
    from paper_0912_4255_amd import autotune
    wls = [synth.workload_c3_segment(i, n_sky=max(n_sky, 1)) for i in range(n_seg)]
    plans, n_tuned = autotune.segment_plans(wls)
    inputs = []
    samples = points = 0
    for i, w in enumerate(wls):
        rng = np.random.default_rng([synth.SEED_BASE + 2, 1000 + i])
        x = synth.zero_gaps(synth.gaussian_noise(rng, w.segment.n, 1.0), w.gaps[0])
        inputs.append(([torch.from_numpy(x).to(dev)], [torch.from_numpy(w.gaps[0]).to(dev)]))
        samples += w.segment.n
        points += plans[i].n_fft
    sky = torch.from_numpy(np.ascontiguousarray(wls[0].skies[:n_sky])).to(dev)
    fd = torch.from_numpy(np.ascontiguousarray(wls[0].fdots[:n_fdot])).to(dev)
    g, vals, ids = rsf.graph_topk_segments(plans, inputs, sky, fd, k=k)
    g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.launch()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    g.close()
    templates = n_seg * n_sky * n_fdot
    full = 64 * 4096 * n_fdot
    taps = sorted({p.desc.taps for p in plans})

    # semi-coherent sum over the same segments on a common grid of 1/(2 d) over [99, 101) Hz
    f_lo, df_c = 99.0, 1.0 / (2 * 86400.0)
    n_c = int(round(2.0 / df_c))
    S = torch.zeros((n_sky * n_fdot, n_c), dtype=torch.float32, device=dev)
    big = max(p.workspace_bytes(rsf.RSF_ENTRY_SEMICOHERENT, n_sky, n_fdot) for p in plans)
    wss = torch.empty(big, dtype=torch.uint8, device=dev)
    plans[0].semicoherent(*inputs[0], sky, fd, torch.zeros_like(S), 0.0, f_lo, df_c, ws=wss)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for p, (tx, tg) in zip(plans, inputs):
        p.semicoherent(tx, tg, sky, fd, S, 0.0, f_lo, df_c, ws=wss)
    torch.cuda.synchronize()
    semi_t = time.perf_counter() - t1
    for p in plans:
        p.close()
    return {"workload": f"first {n_seg} of 64 uneven segments (mean N={samples // n_seg}), "
                        f"{n_sky} sky x {n_fdot} fdot, top-{k} per segment, one HIP graph over all segments",
            "segment_templates": templates, "segment_templates_per_s": round(templates / t, 1),
            "ms_per_replay": round(t * 1e3, 2), "tuned_segments": n_tuned, "taps": taps,
            "fft_points_per_s": round(n_sky * n_fdot * points / t, 1),
            "extrapolated_full_s": round(full / (templates / t), 1),
            "extrapolation": f"64 segments x 4096 sky x {n_fdot} fdot = {full} segment-templates at the measured rate",
            "semicoherent": {"grid": f"[99, 101) Hz at 1/(2 d), {n_c} bins, t_ref = 0",
                             "segment_templates_per_s": round(templates / semi_t, 1),
                             "peak_S": round(float(S.max()), 2), "mean_S": round(float(S.mean()), 3)}}


def sft_leg(rsf, synth, torch, dev, reps=5):
    """SFT front end: the T = 10 d input (432 SFTs of 1800 s, 48 missing,
    7318 bins each) to the heterodyned 4 Hz series of 3,456,000 samples;
    inputs resident in HBM, HIP-event kernel times on the launch stream."""
    ss, X = synth.sft_set_c2()
    plan = rsf.SftPlan(ss)
    sft = torch.from_numpy(X).to(dev)
    out = torch.empty(ss.n_out, dtype=torch.complex64, device=dev)
    ws = plan.workspace(dev)
    plan.heterodyne(sft, out=out, ws=ws)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.heterodyne(sft, out=out, ws=ws)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    prof = plan.profile_read()
    plan.profile(False)
    n_sft, K = X.shape
    alg = n_sft * K * 8 + ss.n_out * 8          # SFT bins in, series out
    kern = {k: {"launches": v[0] // reps, "us_per_segment": round(v[1] / reps * 1e3, 2)} for k, v in prof.items()}
    ktime = sum(v[1] for v in prof.values()) / reps / 1e3
    res = {"workload": f"T=10d: {n_sft} SFTs x {K} bins (1800 s, 48 missing, {plan.n_chunks} chunks) -> "
                       f"{ss.n_out} samples at {ss.band:g} Hz, running median {ss.median_window}, "
                       f"Dirichlet {2 * ss.dk + 1} terms",
           "ms_per_segment": round(t * 1e3, 3), "segments_per_s": round(1.0 / t, 2),
           "kernel_ms_per_segment": round(ktime * 1e3, 3),
           "algorithmic_bytes": int(alg), "algorithmic_GBps": round(alg / t / 1e9, 1),
           "kernels": kern}
    plan.close()
    return res


def hetdec_leg(rsf, torch, dev, reps=5):
    """Time-domain front end: a real 256 Hz series of T = 10 d (221,184,000
    float32 samples) heterodyned at 101 Hz, low-pass filtered (Kaiser sinc,
    2049 taps) and downsampled by 64 to the 4 Hz series of the search."""
    dt, fh, D, K = 1.0 / 256.0, 101.0, 64, 16
    n_raw = 256 * 864000
    g = torch.Generator(device=dev)
    g.manual_seed(9124255)
    x = torch.randn(n_raw, dtype=torch.float32, device=dev, generator=g)
    n_out = n_raw // D
    plan = rsf.HetdecPlan(n_raw, dt, fh, D, K, 8.0, n_out)
    out = torch.empty(n_out, dtype=torch.complex64, device=dev)
    plan.run(x, out=out)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run(x, out=out)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    prof = plan.profile_read()
    plan.close()
    k_ms = prof["rsf_hetdec_k"][1] / reps
    alg = n_raw * 4 + n_out * 8
    taps = 2 * K * D + 1
    # the filter as a real product on the FP32 matrix cores: 4 flops (re and im
    # multiply-add) per tap and output
    tflops = 4.0 * taps * n_out / (k_ms * 1e-3) / 1e12
    return {"workload": f"T=10d real series at 256 Hz ({n_raw} samples) -> {n_out} samples at 4 Hz, "
                        f"{taps}-tap Kaiser low-pass, f_h = {fh:g} Hz",
            "ms_per_segment": round(t * 1e3, 3), "kernel_ms": round(k_ms, 3),
            "algorithmic_bytes": alg, "algorithmic_GBps": round(alg / (k_ms * 1e-3) / 1e9, 1),
            "GMAC_per_s": round(n_out * taps / (k_ms * 1e-3) / 1e9, 1),
            "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": PEAK_FP32_MFMA_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / PEAK_FP32_MFMA_TFLOPS, 4),
                         "flops": 4 * taps * n_out}}


# Compulsory bytes per template of the method at this shape: the inputs once
# (complex64 series 8 B, the resampled series with a, b and t_m 16 B per
# sample), one spill of both spectra (2 x 8 B per FFT point, written and read
# back) and the 2F outputs (4 B per bin): 24 N + 32 N_fft + 4 N_out.
def b_alg(N, Nf, No):
    return 24 * N + 32 * Nf + 4 * No


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes, timed with hipEvents: GB/s counting
    the bytes read plus the bytes written."""
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    del src, dst
    return {"bytes": 2 * nbytes, "ms": round(ms, 4), "GBps": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the path shards by template "
              "and needs no collective: run one process per GPU on disjoint template ranges.",
              file=sys.stderr)
        sys.exit(2)
    from paper_0912_4255_amd import synth

    w = synth.workload_c2(n_fdot=a.n_fdot)
    rng = synth.streams(1)[0]
    x = synth.zero_gaps(synth.gaussian_noise(rng, w.segment.n, 1.0), w.gaps[0])
    n_t = a.n_fdot

    # the CPU oracle first: its worker processes are forked before the GPU is touched
    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(w, x, w.gaps[0], a.cpu_templates, n_t, synth)

    import torch

    import paper_0912_4255_amd as rsf

    rsf.load()
    dev = torch.device("cuda:0")
    tuned = None
    if a.no_autotune:
        plan = rsf.Plan(w)
    else:
        from paper_0912_4255_amd import autotune
        plan, tuned = autotune.tuned_plan(w)
    tx = [torch.from_numpy(x).to(dev)]
    tg = [torch.from_numpy(w.gaps[0]).to(dev)]
    sky = torch.from_numpy(np.ascontiguousarray(w.skies)).to(dev)
    fd = torch.from_numpy(np.ascontiguousarray(w.fdots)).to(dev)
    out = torch.empty((n_t, plan.n_out), dtype=torch.float32, device=dev)
    ws = plan.workspace(rsf.RSF_ENTRY_FSTAT, 1, n_t, rsf.RSF_MODE_BATCHED, device=dev)

    # the step, captured once into a HIP graph
    graph, _ = plan.graph_fstat(tx, tg, sky, fd, out=out, ws=ws)
    for _ in range(a.warmup):
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        graph.launch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / a.steps
    value = n_t * a.steps / (t1 - t0)

    # replays timed one by one until >= 5 replays and >= 10 s (defaults): the median
    ev = []
    t_start = time.perf_counter()
    while len(ev) < a.replay_min or time.perf_counter() - t_start < a.replay_seconds:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.launch()
        e1.record()
        ev.append((e0, e1))
        if len(ev) % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    rep_ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    replays = {"n": int(len(rep_ms)), "total_s": round(float(rep_ms.sum()) / 1e3, 2),
               "median_ms": round(float(np.median(rep_ms)), 3), "min_ms": round(float(rep_ms.min()), 3),
               "max_ms": round(float(rep_ms.max()), 3),
               "median_templates_per_s": round(n_t / (float(np.median(rep_ms)) * 1e-3), 2)}
    graph.close()

    # per-kernel durations: a separate instrumented pass of the same launches
    # (hipEvents recorded by the library on the launch stream)
    prof_steps = max(1, min(a.steps, 5))
    plan.profile(True)
    plan.profile_read()
    for _ in range(prof_steps):
        plan.fstat(tx, tg, sky, fd, mode=rsf.RSF_MODE_BATCHED, out=out, ws=ws)
    prof = plan.profile_read()
    plan.profile(False)

    # plain per-template path on a subset of the spindowns (0 skips it)
    n_p = min(a.plain_templates, n_t)
    plain_rate = None
    if n_p > 0:
        fd_p = fd[:n_p].contiguous()
        out_p = torch.empty((n_p, plan.n_out), dtype=torch.float32, device=dev)
        ws_p = plan.workspace(rsf.RSF_ENTRY_FSTAT, 1, n_p, rsf.RSF_MODE_PLAIN, device=dev)
        plan.fstat(tx, tg, sky, fd_p, mode=rsf.RSF_MODE_PLAIN, out=out_p, ws=ws_p)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        plan.fstat(tx, tg, sky, fd_p, mode=rsf.RSF_MODE_PLAIN, out=out_p, ws=ws_p)
        torch.cuda.synchronize()
        plain_rate = round(n_p / (time.perf_counter() - tp0), 2)
        del out_p, ws_p

    # roofline of the dominant kernel: algorithmic bytes per launch (per-launch
    # bytes summed over the instrumented pass's launches) / mean launch duration
    N, Nf, No = w.segment.n, plan.n_fft, plan.n_out
    fb, G, _ = plan.batching(1, n_t)
    sizes = [min(G, n_t - f0) for f0 in range(0, n_t, G)]
    total_bytes = {
        # resampled row (z~ 8 B + a, b, t_m 4 B each) read once per group of
        # fb spindowns, both spectra (2 x 8 B per FFT sample) spilled
        "rsf_fft_pass_a_k": sum(-(-g // fb) * 20 * N + g * 16 * Nf for g in sizes),
        # both spectra read back, 2F written for the reported band
        "rsf_fft_pass_b_k": sum(g * (16 * Nf + 4 * No) for g in sizes),
        # series read, resampled series (z~ 8 B, a, b, t_m) written
        "rsf_resample_k": 8 * N + 20 * N,
    }
    kern = {k: v for k, v in prof.items() if k in total_bytes}
    dom = max(kern, key=lambda k: kern[k][1])
    launches, total_ms = kern[dom]
    avg_s = total_ms / launches / 1e3
    bytes_per_launch = total_bytes[dom] * prof_steps / launches
    achieved = bytes_per_launch / avg_s / 1e9
    cfg = f"{plan.fft_l1}x{plan.fft_l2},fb{fb},g{G}"
    traffic = committed_traffic(dom, cfg)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "bytes/launch", "config": cfg, "kernel_src": kernel_source_hash(),
                "kernel": dom, "avg_launch_us": round(avg_s * 1e6, 2),
                "bytes_per_launch": int(bytes_per_launch), "templates_per_launch": G, "fb": fb,
                "kernels": {k: {"launches": v[0], "avg_us": round(v[1] / v[0] * 1e3, 2),
                                "share": round(v[1] / sum(t for _, t in prof.values()), 4)}
                            for k, v in prof.items()}}
    copy = copy_bandwidth(torch, dev)
    B = b_alg(N, Nf, No)
    path = {"bytes_per_template": B, "formula": "24 N + 32 N_fft + 4 N_out",
            "achieved_GBps": round(value * B / 1e9, 1), "frac": round(value * B / 1e9 / HBM_PEAK_GBS, 4),
            "frac_of_copy": round(value * B / 1e9 / copy["GBps"], 4)}

    grad = None if a.no_grad else grad_leg(rsf, synth, torch, dev, a.grad_candidates)
    sft_fe = None if a.no_sft else sft_leg(rsf, synth, torch, dev)
    hetdec = None if a.no_hetdec else hetdec_leg(rsf, torch, dev)
    c3 = None if a.no_c3 else c3_leg(rsf, synth, torch, dev, a.c3_segments, a.c3_sky)
    if c3 is not None:
        # FFT points per second against the headline's (same kernels, other shapes)
        c3["fft_points_per_s_vs_headline"] = round(c3["fft_points_per_s"] / (value * Nf), 4)

    rec = {"metric": "F-stat templates/s at T=10d, 2Hz band: plain vs batched+grad; %HBM roofline",
           "value": round(value, 2), "unit": "templates/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"T=10d dt=0.25s N=3456000 10pct gaps, 1 sky x {n_t} fdot, "
                                  "Dirichlet-16, N_fft=6912000, band [100,102) Hz",
                      "templates_per_step": n_t, "n_fft": Nf, "n_out": No,
                      "fft_factors": [plan.fft_l1, plan.fft_l2], "timing": "HIP graph replays"},
           "replays": replays, "plain_templates_per_s": plain_rate,
           "autotune": tuned, "grad": grad, "c3": c3, "sft_front_end": sft_fe, "time_domain_front_end": hetdec,
           "roofline": roofline, "path_roofline": path, "copy": copy, "cpu_baseline": cpu}
    print(json.dumps(rec))


if __name__ == "__main__":
    main()

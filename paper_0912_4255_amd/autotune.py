"""Autotuner for librsfstat plans.

Times candidate configurations of the batched search on the GPU with
synthetic noise of the plan's shape and keeps the fastest:

* the FFT factorisation n_fft = L1 x L2 (rsf_plan_desc.fft_l1);
* the number of spindowns sharing one read of the resampled series in the
  first FFT pass, and the templates per FFT launch (rsf_plan_set_batching).

Results are cached in a JSON file keyed by the GPU architecture and the plan
shape (``$RSF_AUTOTUNE_CACHE``, default ``~/.cache/rsfstat/autotune.json``);
``tuned_gfx950.json`` beside this module ships entries measured on MI355X for
the standard workload shapes and is consulted after the user cache.
``choose_taps`` picks the narrowest interpolation kernel whose 2F stays within
a bound of a 32-tap reference over the central half of the band.
"""
import copy
import json
import os
import time

import numpy as np
import torch

from . import _lib as L
from . import synth
from .api import Plan, plan_desc_from_workload


def cache_path():
    return os.environ.get("RSF_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rsfstat", "autotune.json"))


def _key(desc, n_fft):
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    return f"{arch}|n={desc.n}|nfft={n_fft}|det={desc.n_det}|kernel={desc.kernel}|taps={desc.taps}|store={desc.storage}"


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_gfx950.json")


def _read(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _load():
    return _read(cache_path())


def _save(db):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _divisors(n, lo, hi):
    return [d for d in range(max(1, lo), min(n, hi) + 1) if n % d == 0]


def candidate_l1(plan, limit=8):
    """First-pass lengths that the planner accepts: those that leave a
    one-column-per-wave second pass (L2 = 768, 512, 256, then 1024, the
    top-k's) first, then the others nearest the automatic choice."""
    n_fft = plan.n_fft
    wave = [n_fft // lb for lb in (768, 512, 256, 1024) if n_fft % lb == 0 and n_fft // lb <= 10240]
    cands = _divisors(n_fft, max(8, plan.fft_l1 // 4), min(10240, plan.fft_l1 * 4))
    cands.sort(key=lambda d: abs(np.log(d / plan.fft_l1)))
    cands = wave + [d for d in cands if d not in wave]
    out = []
    for d in cands:
        desc = copy.copy(plan.desc)
        desc.fft_l1 = d
        try:
            p = Plan(desc=desc)
        except L.RsfError:
            continue
        out.append(p)
        if len(out) >= limit:
            break
    return out


def _time_plan(plan, xs, gaps, sky, fdot, reps=2):
    ws = plan.workspace(L.RSF_ENTRY_FSTAT, sky.shape[0], fdot.shape[0], L.RSF_MODE_BATCHED)
    out = torch.empty((sky.shape[0] * fdot.shape[0], plan.n_out), dtype=torch.float32, device="cuda")
    plan.fstat(xs, gaps, sky, fdot, out=out, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.fstat(xs, gaps, sky, fdot, out=out, ws=ws)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps / (sky.shape[0] * fdot.shape[0])


def tune(workload, n_fdot=32, reps=2, use_cache=True, fbs=(2, 4, 8), templates=(16, 32), verbose=False):
    """Best {fft_l1, fb, templates, s_per_template} for the workload's plan shape."""
    base = Plan(workload)
    key = _key(base.desc, base.n_fft)
    db = _load() if use_cache else {}
    if key in db:
        return db[key]
    if use_cache:
        shipped = _read(SHIPPED)
        if key in shipped:
            return dict(shipped[key], source="shipped")
    rng = np.random.default_rng(0)
    xs = [torch.from_numpy(synth.gaussian_noise(rng, base.n, d.sigma2)).cuda() for d in workload.detectors]
    gaps = [None] * len(xs)
    sky = torch.tensor([[1.0, 0.3]], dtype=torch.float64, device="cuda")
    fdot = torch.from_numpy(synth.fdot_grid(n_fdot)).cuda()
    best = None
    for p in candidate_l1(base):
        for fb in fbs:
            for g in templates:
                p.set_batching(fb, g)
                t = _time_plan(p, xs, gaps, sky, fdot, reps)
                if verbose:
                    print(f"L1={p.fft_l1} L2={p.fft_l2} fb={fb} G={g}: {t * 1e6:.1f} us/template")
                if best is None or t < best["s_per_template"]:
                    best = {"fft_l1": p.fft_l1, "fft_l2": p.fft_l2, "fb": fb, "templates": g, "s_per_template": t}
        p.close()
    db[key] = best
    if use_cache:
        _save(db)
    return best


def tuned_plan(workload, **kw):
    """A Plan built with the tuned factorisation and batching."""
    best = tune(workload, **kw)
    desc = plan_desc_from_workload(workload)
    desc.fft_l1 = best["fft_l1"]
    p = Plan(desc=desc)
    p.set_batching(best["fb"], best["templates"])
    return p, best


def choose_taps(workload, candidates=(8, 12, 16, 24), bound=1e-2, ref_taps=32, n_fdot=2, seed=0):
    """Smallest W (same kernel family) whose 2F over the central half of the
    band is within `bound` * max(2F_ref, 4) of the ref_taps kernel, on
    synthetic noise.  Returns (W, {W: max relative deviation})."""
    rng = np.random.default_rng(seed)
    xs = [torch.from_numpy(synth.gaussian_noise(rng, workload.segment.n, d.sigma2)).cuda()
          for d in workload.detectors]
    sky = torch.tensor([[2.0, -0.4]], dtype=torch.float64, device="cuda")
    fdot = torch.from_numpy(synth.fdot_grid(n_fdot)).cuda()

    def run(taps):
        d = plan_desc_from_workload(workload)
        d.taps = taps
        return Plan(desc=d).fstat(xs, [None] * len(xs), sky, fdot).cpu().numpy()

    ref = run(ref_taps)
    n = ref.shape[1]
    mid = slice(n // 4, 3 * n // 4)
    dev = {}
    for w in sorted(candidates):
        got = run(w)
        dev[w] = float(np.max(np.abs(got[:, mid] - ref[:, mid]) / np.maximum(ref[:, mid], 4.0)))
    ok = [w for w in sorted(candidates) if dev[w] <= bound]
    return (ok[0] if ok else max(candidates)), dev


def _time_topk(plan, xs, gaps, sky, fdot, reps=2, k=10):
    ws = plan.workspace(L.RSF_ENTRY_TOPK, sky.shape[0], fdot.shape[0])
    plan.topk(xs, gaps, sky, fdot, k=k, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.topk(xs, gaps, sky, fdot, k=k, ws=ws)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps / (sky.shape[0] * fdot.shape[0])


def tune_segment(workload, n_sky=8, n_fdot=16, fbs=(8, 16), templates=(32, 64, 128), l1_limit=3, taps=None,
                 verbose=False):
    """Tuning of one uneven segment for its own template loop (n_sky sky
    positions x n_fdot spindowns, per-segment top-k): the interpolation taps
    from choose_taps (unless given), then the FFT factorisation and batching
    timed on that loop.  Returns {taps, fft_l1, fft_l2, fb, templates,
    s_per_template}."""
    if taps is None:
        taps, _ = choose_taps(workload)
    desc = plan_desc_from_workload(workload)
    desc.taps = taps
    base = Plan(desc=desc)
    rng = np.random.default_rng(1)
    xs = [torch.from_numpy(synth.gaussian_noise(rng, base.n, d.sigma2)).cuda() for d in workload.detectors]
    gaps = [None] * len(xs)
    sky = torch.from_numpy(np.ascontiguousarray(synth.uniform_sky(rng, n_sky))).cuda()
    fdot = torch.from_numpy(synth.fdot_grid(n_fdot)).cuda()
    best = None
    for p in candidate_l1(base, limit=l1_limit):
        for fb in fbs:
            for g in templates:
                p.set_batching(fb, g)
                t = _time_topk(p, xs, gaps, sky, fdot)
                if verbose:
                    print(f"n={base.n} L1={p.fft_l1} fb={fb} G={g}: {t * 1e6:.1f} us/template", flush=True)
                if best is None or t < best["s_per_template"]:
                    best = {"taps": taps, "fft_l1": p.fft_l1, "fft_l2": p.fft_l2, "fb": fb, "templates": g,
                            "s_per_template": t}
        p.close()
    base.close()
    return best


SEGMENTS_KEY = "segments:c3"


def segment_plans(workloads):
    """Plans for uneven segments with the shipped per-segment tuning (taps,
    factorisation, batching), keyed by segment length; segments without an
    entry keep their workload's taps and the planner's choices."""
    table = _read(SHIPPED).get(SEGMENTS_KEY, {})
    plans, used = [], 0
    for w in workloads:
        e = table.get(str(w.segment.n))
        desc = plan_desc_from_workload(w)
        if e:
            desc.taps = e["taps"]
            desc.fft_l1 = e["fft_l1"]
        p = Plan(desc=desc)
        if e:
            p.set_batching(e["fb"], e["templates"])
            used += 1
        plans.append(p)
    return plans, used


def _standard_workloads():
    return {"T=10d dt=0.25s (N=3456000)": synth.workload_c2(n_fdot=32),
            "T=10d dt=0.5s (N=1728000)": synth.workload_c5(),
            "T=1d dt=0.5s (N=172800)": synth.workload_c1(),
            "T=30d dt=0.5s, 2 detectors (N=5184000)": synth.workload_c4()}


def main(argv=None):
    """Tune the standard workload shapes on the current GPU and write the
    entries (merged into an existing file) to --out (default: the shipped
    table beside this module).  --segments N also tunes the first N uneven
    segments (taps, factorisation and batching each)."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--out", default=SHIPPED)
    ap.add_argument("--fbs", default="2,4,8,16")
    ap.add_argument("--templates", default="16,32,64")
    ap.add_argument("--n-fdot", type=int, default=64)
    ap.add_argument("--segments", type=int, default=0)
    ap.add_argument("--segment-ids", default="", help="comma-separated segment indices to tune instead")
    ap.add_argument("--no-standard", action="store_true")
    ap.add_argument("--keep-taps", action="store_true", help="segments keep the taps of the existing table")
    a = ap.parse_args(argv)
    fbs = tuple(int(v) for v in a.fbs.split(","))
    gs = tuple(int(v) for v in a.templates.split(","))
    db = _read(a.out)
    if not a.no_standard:
        for name, w in _standard_workloads().items():
            base = Plan(w)
            key = _key(base.desc, base.n_fft)
            base.close()
            best = tune(w, n_fdot=a.n_fdot, reps=2, use_cache=False, fbs=fbs, templates=gs, verbose=True)
            best["workload"] = name
            db[key] = best
            print(name, key, best, flush=True)
            torch.cuda.empty_cache()
    ids = [int(v) for v in a.segment_ids.split(",") if v] or list(range(a.segments))
    if ids:
        table = db.setdefault(SEGMENTS_KEY, {})
        for i in ids:
            w = synth.workload_c3_segment(i, n_sky=8)
            old = table.get(str(w.segment.n))
            best = tune_segment(w, taps=old["taps"] if (a.keep_taps and old) else None)
            table[str(w.segment.n)] = best
            print(f"segment {i}: n={w.segment.n}", best, flush=True)
            torch.cuda.empty_cache()
    with open(a.out, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()

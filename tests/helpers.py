"""Shared test helpers: seeded inputs for a workload, built on the CPU, with
injected signals from the oracle's generator."""
import numpy as np

from oracle.inject import signal
from paper_0912_4255_amd import synth


def make_inputs(w, seed=0, injections=(), noise=True):
    """Per-detector complex64 series (noise + injections, zero-filled gaps)."""
    rng = np.random.default_rng(seed)
    xs = []
    for X, det in enumerate(w.detectors):
        x = (synth.gaussian_noise(rng, w.segment.n, det.sigma2).astype(np.complex128)
             if noise else np.zeros(w.segment.n, np.complex128))
        for inj in injections:
            x = x + signal(w.segment, inj, w.eph, det)
        g = w.gaps[X] if X < len(w.gaps) else np.zeros((0, 2), np.int64)
        xs.append(synth.zero_gaps(x.astype(np.complex64), g))
    gaps = [w.gaps[X] if X < len(w.gaps) else np.zeros((0, 2), np.int64) for X in range(len(w.detectors))]
    return xs, gaps


def to_gpu(xs, gaps):
    import torch
    tx = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in xs]
    tg = [torch.from_numpy(np.ascontiguousarray(g, dtype=np.int64)).cuda() if len(g) else None
          for g in gaps]
    return tx, tg


def twoF_tol(ref):
    """|delta 2F| <= 1e-4 max(2F_oracle, 4): the FP32-bulk tolerance."""
    return 1e-4 * np.maximum(ref, 4.0)

"""Write c5_gradient.json: the FP64 oracle's 2F and finite-difference
gradient for three candidates of the gradient workload (T = 10 d, dt = 0.5 s,
N = 1,728,000, Dirichlet-16).

Calls only the oracle and the seeded input generators; nothing here touches
the HIP library.  The input is unit-variance noise from
default_rng([9124255 + 4, 7]) plus the signals of the workload's first two
injections; the file records a checksum of that input so that a test can
confirm it regenerated the same series.  Each gradient is the oracle's
Richardson-extrapolated central difference with its default steps
(h_f = 1e-3 / T0, h_fdot = 1e-3 / T0^2, h_alpha = h_delta = 1e-7 rad).

Usage: python tests/golden/make_c5_gradient.py   (about 3 minutes)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import grad as og  # noqa: E402
from oracle.inject import signal  # noqa: E402
from paper_0912_4255_amd import synth  # noqa: E402

ROWS = (0, 5, 26)          # rows of synth.c5_candidates: two corners of injection 0, one of injection 1
NOISE_SEED = [synth.SEED_BASE + 4, 7]
OUT = os.path.join(HERE, "c5_gradient.json")


def c5_input(w):
    """The test series: noise plus injections 0 and 1 (complex64)."""
    x = synth.gaussian_noise(np.random.default_rng(NOISE_SEED), w.segment.n, 1.0).astype(np.complex128)
    for inj in w.injections[:2]:
        x = x + signal(w.segment, inj, w.eph, w.detectors[0])
    return x.astype(np.complex64)


def checksum(x):
    x = x.astype(np.complex128)
    k = np.arange(x.shape[0], dtype=np.float64)
    return [float(np.sum(x.real)), float(np.sum(x.imag)), float(np.sum(np.abs(x) ** 2)),
            float(np.sum(k * x.real) / x.shape[0])]


def main():
    w = synth.workload_c5()
    df = 1.0 / (2 * w.segment.n * w.segment.dt)
    x = c5_input(w)
    prob = og.PointProblem([x], [np.zeros((0, 2), np.int64)], w.segment, list(w.detectors), w.eph,
                           w.kernel, w.taps)
    cand = synth.c5_candidates(w, df)
    recs = []
    for r in ROWS:
        th = cand[r]
        F = prob.twoF(th)
        g = og.gradient(prob, th)
        recs.append({"row": r, "theta": [float(v) for v in th], "twoF": float(F), "grad": [float(v) for v in g]})
        print(r, F, g, flush=True)
    out = {"workload": "T=10d dt=0.5s N=1728000 Dirichlet-16, one detector, no gaps",
           "noise_seed": NOISE_SEED, "injections": [0, 1], "checksum": checksum(x),
           "steps": [float(v) for v in og.default_steps(w.segment)], "candidates": recs}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()

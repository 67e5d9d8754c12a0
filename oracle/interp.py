"""Interpolation of a regularly sampled series at irregular times (oracle, FP64).

Paper Sec. III.A.2 (steps 3-4 of the resampling procedure) interpolates
z(t^k) at the detector times T^k but never names the method; Sec. V.B notes
that the interpolation acts as a low-pass filter.  The workloads fix the
kernels:

* Lanczos-W ("windowed sinc"): w(x) = sinc(x) sinc(2x/W) for |x| < W/2,
  sinc(x) = sin(pi x)/(pi x);
* Dirichlet-W: the periodic band-limited kernel of an N-sample series,
  w(x) = sin(pi x) / (N tan(pi x / N)) for even N and
  sin(pi x) / (N sin(pi x / N)) for odd N, truncated to W taps;
* full Dirichlet: the same kernel over all N taps with periodic wrap (exact
  for periodic band-limited series; used only on small inputs).

For a fractional sample position u = j + frac (j = floor(u)), the W taps are
the samples j - W/2 + i, i = 1..W, at distances x_i = frac + W/2 - i; taps
outside [0, N) read zero.  Weights are not renormalised.

Parity unpinned (convention): the choice of window, and zero taps outside
the segment.
"""
import numpy as np

KERNEL_LANCZOS = 0
KERNEL_DIRICHLET = 1


def lanczos_weight(x, W):
    x = np.asarray(x, dtype=np.float64)
    w = np.sinc(x) * np.sinc(2.0 * x / W)
    return np.where(np.abs(x) < W / 2.0, w, 0.0)


def dirichlet_weight(x, N):
    x = np.asarray(x, dtype=np.float64)
    num = np.sin(np.pi * x)
    if N % 2 == 0:
        den = N * np.tan(np.pi * x / N)
    else:
        den = N * np.sin(np.pi * x / N)
    with np.errstate(invalid="ignore", divide="ignore"):
        w = num / den
    return np.where(x == 0.0, 1.0, w)


def kernel_weight(x, kernel, W, N):
    if kernel == KERNEL_LANCZOS:
        return lanczos_weight(x, W)
    if kernel == KERNEL_DIRICHLET:
        return dirichlet_weight(x, N)
    raise ValueError("unknown kernel")


def interpolate(z, u, kernel, W):
    """z~(u) = sum_{i=1..W} w(frac + W/2 - i) z[floor(u) - W/2 + i]."""
    z = np.asarray(z)
    N = z.shape[0]
    u = np.asarray(u, dtype=np.float64)
    j = np.floor(u)
    frac = u - j
    j = j.astype(np.int64)
    out = np.zeros(u.shape, dtype=np.complex128)
    for i in range(1, W + 1):
        pos = j - W // 2 + i
        x = frac + W / 2.0 - i
        ok = (pos >= 0) & (pos < N)
        tap = np.where(ok, z[np.clip(pos, 0, N - 1)], 0.0)
        out += kernel_weight(x, kernel, W, N) * tap
    return out


def interpolate_full_dirichlet(z, u):
    """Exact periodic band-limited interpolation: sum over all N samples with
    periodic distances."""
    z = np.asarray(z, dtype=np.complex128)
    N = z.shape[0]
    u = np.asarray(u, dtype=np.float64)
    out = np.zeros(u.shape, dtype=np.complex128)
    for m in range(N):
        out += dirichlet_weight(u - m, N) * z[m]
    return out

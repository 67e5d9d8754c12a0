"""The oracle's own FFT (FP64): forward DFT X[k] = sum_n x[n] exp(-2 pi i n k / N),
unnormalised, for N whose prime factors are 2, 3, 5 and 7.

Paper Sec. III.A.2 step 6 evaluates the F_a and F_b sums of eqs. eq19/eq20 on
the regular SSB grid with FFTs.  This is a radix-by-radix Stockham
(self-sorting) transform: at each stage with radix R, after Ns points have
been combined, every butterfly j reads x[j + r N/R], r = 0..R-1, multiplies by
exp(-2 pi i r (j mod Ns) / (Ns R)), takes an R-point DFT (a small matrix
product) and writes position (j div Ns) Ns R + (j mod Ns) + r Ns.  After the
last stage the output is in natural order.  Twiddles are evaluated directly
in FP64 at every stage.
"""
import numpy as np


def factorize(n):
    """Radix sequence for n: 4s first, then 2, 3, 5, 7."""
    if n < 1:
        raise ValueError("n must be positive")
    out = []
    m = n
    while m % 4 == 0:
        out.append(4)
        m //= 4
    for p in (2, 3, 5, 7):
        while m % p == 0:
            out.append(p)
            m //= p
    if m != 1:
        raise ValueError(f"{n} has a prime factor larger than 7")
    return out


def is_7smooth(n):
    try:
        factorize(n)
        return True
    except ValueError:
        return False


def next_7smooth(n):
    m = max(1, int(n))
    while not is_7smooth(m):
        m += 1
    return m


def dft_matrix(R):
    r = np.arange(R)
    return np.exp(-2j * np.pi * np.outer(r, r) / R)


def fft(x):
    """Forward transform along the last axis of a 1-D array."""
    a = np.asarray(x, dtype=np.complex128).copy()
    N = a.shape[0]
    if N == 1:
        return a
    Ns = 1
    for R in factorize(N):
        L = N // R
        j = np.arange(L)
        k = j % Ns
        v = a.reshape(R, L)                       # v[r, j] = a[j + r L]
        tw = np.exp(-2j * np.pi * np.outer(np.arange(R), k) / (Ns * R))
        V = dft_matrix(R) @ (v * tw)              # R-point DFT of each column
        out = np.empty(N, dtype=np.complex128)
        base = (j // Ns) * Ns * R + k
        for r in range(R):
            out[base + r * Ns] = V[r]
        a = out
        Ns *= R
    return a


def dft_bruteforce(x):
    """O(N^2) definition, for pinning the FFT on small N."""
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[0]
    n = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(n, n) / N) @ x

"""FP64 CPU oracle for the batched real FFT and its inverse.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module.  The GPU library and its
Python binding never import it, and this module imports nothing from them.

The paper's roadmap (Sec. 5) names the FFT beside the STFT.  The transform is
the textbook discrete Fourier transform of each row, written out as the sum
that defines it (an n x (n/2+1) matrix of exponentials applied to the rows,
in FP64):

  X[b, k] = sum_{m < n} x[b, m] exp(-2 pi i k m / n),    k = 0 .. n/2,

and its inverse for a real signal (the Hermitian-symmetric extension of the
one-sided spectrum; the imaginary parts of bins 0 and n/2 do not enter):

  y[b, m] = (1/n) (Re X[b, 0] + Re X[b, n/2] (-1)^m
                   + 2 Re sum_{k=1}^{n/2-1} X[b, k] exp(+2 pi i k m / n)).

The exponent k m is reduced mod n before the exponential, so every entry is
a correctly rounded FP64 unit-circle point.
"""
from __future__ import annotations

import numpy as np


def _phase(n: int, sign: float) -> np.ndarray:
    """[n, n/2 + 1] matrix exp(sign 2 pi i (m k mod n) / n)."""
    m = np.arange(n)[:, None]
    k = np.arange(n // 2 + 1)[None, :]
    return np.exp(sign * 2j * np.pi * ((m * k) % n) / n)


def rfft(x) -> np.ndarray:
    """One-sided DFT of every row of x ([..., n]) -> complex128 [..., n/2 + 1]."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[-1]
    return (x.reshape(-1, n) @ _phase(n, -1.0)).reshape(*x.shape[:-1], n // 2 + 1)


def irfft(X, n: int) -> np.ndarray:
    """Inverse of rfft for rows of n samples (n even)."""
    X = np.asarray(X, dtype=np.complex128)
    if X.shape[-1] != n // 2 + 1:
        raise ValueError("spectrum has %d bins, n = %d needs %d" % (X.shape[-1], n, n // 2 + 1))
    lead = X.shape[:-1]
    Xr = X.reshape(-1, n // 2 + 1)
    wgt = np.full(n // 2 + 1, 2.0)
    wgt[0] = 1.0
    wgt[n // 2] = 1.0
    E = _phase(n, 1.0)                                   # [n, n/2 + 1]
    Xw = Xr.copy()
    Xw[:, 0] = Xw[:, 0].real
    Xw[:, n // 2] = Xw[:, n // 2].real
    y = (Xw * wgt[None, :]) @ E.T                         # [B, n]
    return (y.real / n).reshape(*lead, n)

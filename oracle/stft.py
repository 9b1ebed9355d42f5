"""FP64 CPU oracle for the short-time Fourier transform and its inverse.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module.  The GPU library and its
Python binding never import it, and this module imports nothing from them.

The paper's roadmap (Sec. 5) names FFT and STFT as the next signal-processing
functions.  The transform is the textbook one, written out directly:

  frame t of channel c starts at padded sample t * hop;
  X[c, t, k] = sum_{n < n_fft} w[n] xp[c, t*hop + n] exp(-2 pi i k n / n_fft),
  k = 0 .. n_fft/2 (one-sided spectrum of a real signal),

where xp is x itself, or (``center``) x padded by n_fft/2 reflected samples
on both sides (xp[-j] = x[j], xp[N-1+j] = x[N-1-j]), and w is the window of
``win_length`` samples placed in the middle of the n_fft-sample frame (zeros
around it).  ``normalized`` scales by 1/sqrt(n_fft).  The inverse is the
weighted overlap-add: each frame's real inverse DFT times the window, summed
at its position and divided by the summed squared window, then trimmed by
n_fft/2 on the left when ``center``.  Conventions (interface, not code) are
those of ``torch.stft`` / ``torch.istft`` with ``onesided=True``, except that
the spectrum is stored frame-major: [C, T, n_fft/2 + 1].

The frame DFT uses ``numpy.fft.rfft`` / ``irfft`` as a library primitive; the
framing, padding, windowing and overlap-add are explicit loops over frames.
"""
from __future__ import annotations

import numpy as np


def _as2d(x):
    x = np.asarray(x, dtype=np.float64)
    return (x[None, :], True) if x.ndim == 1 else (x, False)


def full_window(window, n_fft: int) -> np.ndarray:
    """The window placed in the middle of an n_fft frame (rectangular when
    ``window`` is None)."""
    if window is None:
        return np.ones(n_fft)
    w = np.asarray(window, dtype=np.float64).reshape(-1)
    if w.size > n_fft:
        raise ValueError("win_length exceeds n_fft")
    out = np.zeros(n_fft)
    left = (n_fft - w.size) // 2
    out[left:left + w.size] = w
    return out


def num_frames(n: int, n_fft: int, hop: int, center: bool) -> int:
    npad = n + 2 * (n_fft // 2) if center else n
    if npad < n_fft:
        return 0
    return 1 + (npad - n_fft) // hop


def padded(x, n_fft: int, center: bool) -> np.ndarray:
    """Rows of x, reflect-padded by n_fft/2 on both sides when ``center``."""
    x, _ = _as2d(x)
    if not center:
        return x.copy()
    p = n_fft // 2
    C, N = x.shape
    if p and N <= p:
        raise ValueError("reflect padding needs more than n_fft/2 samples")
    out = np.empty((C, N + 2 * p))
    out[:, p:p + N] = x
    for j in range(1, p + 1):
        out[:, p - j] = x[:, j]
        out[:, p + N - 1 + j] = x[:, N - 1 - j]
    return out


def stft(x, n_fft: int, hop: int, window=None, center: bool = True, normalized: bool = False) -> np.ndarray:
    """Complex spectrum [C, T, n_fft/2 + 1] (or [T, n_fft/2 + 1] for 1-D x)."""
    x2, squeeze = _as2d(x)
    w = full_window(window, n_fft)
    xp = padded(x2, n_fft, center)
    T = num_frames(x2.shape[1], n_fft, hop, center)
    out = np.empty((x2.shape[0], T, n_fft // 2 + 1), dtype=np.complex128)
    for t in range(T):
        out[:, t, :] = np.fft.rfft(w * xp[:, t * hop:t * hop + n_fft], axis=-1)
    if normalized:
        out /= np.sqrt(n_fft)
    return out[0] if squeeze else out


def envelope(window, n_fft: int, hop: int, T: int) -> np.ndarray:
    """Sum over frames of the squared window at each padded sample."""
    w2 = full_window(window, n_fft) ** 2
    env = np.zeros(n_fft + hop * max(T - 1, 0))
    for t in range(T):
        env[t * hop:t * hop + n_fft] += w2
    return env


def istft(spec, n_fft: int, hop: int, window=None, center: bool = True, normalized: bool = False,
          length=None) -> np.ndarray:
    """Inverse of ``stft`` by weighted overlap-add; ``length`` trims or zero-
    extends the result (default: every sample the frames cover, less the
    centre padding).  Raises where the summed squared window vanishes."""
    s = np.asarray(spec, dtype=np.complex128)
    squeeze = s.ndim == 2
    if squeeze:
        s = s[None]
    C, T, F = s.shape
    if F != n_fft // 2 + 1:
        raise ValueError("spectrum has %d bins, n_fft %d needs %d" % (F, n_fft, n_fft // 2 + 1))
    w = full_window(window, n_fft)
    frames = np.fft.irfft(s, n=n_fft, axis=-1)
    if normalized:
        frames *= np.sqrt(n_fft)
    total = n_fft + hop * (T - 1)
    ola = np.zeros((C, total))
    for t in range(T):
        ola[:, t * hop:t * hop + n_fft] += w * frames[:, t, :]
    env = envelope(window, n_fft, hop, T)
    start = n_fft // 2 if center else 0
    end = total - (n_fft // 2 if center else 0)
    if length is not None:
        end = start + length
    keep = slice(start, min(end, total))
    if np.any(np.abs(env[keep]) < 1e-11):
        raise ValueError("window overlap-add is zero somewhere (NOLA fails)")
    y = ola[:, keep] / env[keep]
    if length is not None and y.shape[1] < length:
        y = np.concatenate([y, np.zeros((C, length - y.shape[1]))], axis=1)
    return y[0] if squeeze else y


def hann(n: int) -> np.ndarray:
    """Periodic Hann window (the usual choice for an STFT)."""
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * np.arange(n) / n)


def frame(x_row, n_fft: int, hop: int, window, center: bool, t: int, normalized: bool = False) -> np.ndarray:
    """Spectrum of frame t of one channel alone (sampled checks of long signals)."""
    x = np.asarray(x_row, dtype=np.float64).reshape(-1)
    p = n_fft // 2 if center else 0
    idx = t * hop + np.arange(n_fft) - p
    idx = np.where(idx < 0, -idx, idx)
    idx = np.where(idx >= x.size, 2 * (x.size - 1) - idx, idx)
    out = np.fft.rfft(full_window(window, n_fft) * x[idx])
    return out / np.sqrt(n_fft) if normalized else out

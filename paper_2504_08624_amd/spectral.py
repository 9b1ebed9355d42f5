"""Short-time Fourier transform and its inverse (the FFT / STFT functions on
the roadmap of Sec. 5), as thin bindings of ``tfx_stft`` / ``tfx_istft``.

The conventions are those of ``torch.stft`` / ``torch.istft`` with
``onesided=True`` and reflect padding: ``stft`` returns a complex64 tensor
shaped [C, n_fft/2 + 1, T] (or [n_fft/2 + 1, T] for a 1-D signal).  The
library stores the spectrum frame-major ([C, T, F], each frame's bins
contiguous), so the returned tensor is a transposed view of that storage;
``istft`` takes it back without a copy.  ``n_fft`` is a power of two from 16
to 4096.  There is no CPU path.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import lib
from .functional import _ptr, _signal, _stream


def _window(window, win_length: int, device):
    if window is None:
        return None
    w = torch.as_tensor(window, dtype=torch.float32)
    if w.dim() != 1 or w.numel() != win_length:
        raise ValueError("window must be 1-D with win_length = %d samples" % win_length)
    return w.to(device).contiguous()


def _lengths(n_fft, hop_length, win_length):
    hop = n_fft // 4 if hop_length is None else int(hop_length)
    wl = n_fft if win_length is None else int(win_length)
    return int(n_fft), hop, wl


def num_frames(n: int, n_fft: int, hop_length=None, center: bool = True) -> int:
    n_fft, hop, _ = _lengths(n_fft, hop_length, None)
    T = ctypes.c_int64(0)
    lib.call("tfx_stft_frames", int(n), n_fft, hop, int(bool(center)), ctypes.byref(T))
    return int(T.value)


def stft(x: torch.Tensor, n_fft: int, hop_length=None, win_length=None, window=None, center: bool = True,
         normalized: bool = False) -> torch.Tensor:
    """X[c, k, t] = sum_n w[n] xp[c, t*hop + n] exp(-2 pi i k n / n_fft)."""
    n_fft, hop, wl = _lengths(n_fft, hop_length, win_length)
    x2, squeeze, ld = _signal(x)
    C, N = x2.shape
    T = num_frames(N, n_fft, hop, center)
    F = n_fft // 2 + 1
    spec = torch.empty((C, T, F), dtype=torch.complex64, device=x.device)
    w = _window(window, wl, x.device)
    lib.call("tfx_stft", _ptr(x2), C, N, ld, n_fft, hop, _ptr(w), wl, int(bool(center)), int(bool(normalized)),
             spec.data_ptr() if spec.numel() else None, _stream(x.device))
    out = spec.transpose(1, 2)
    return out[0] if squeeze else out


def _envelope_min(w2: np.ndarray, hop: int, T: int, start: int, end: int) -> float:
    """Smallest summed squared window over padded samples [start, end).
    Samples more than n_fft + hop from both ends see every frame that can
    cover them, so the envelope there repeats with period hop and one period
    of it already lies within the first 2 (n_fft + hop) samples."""
    N = w2.size
    K = 2 * (N + hop)
    if end - start <= 2 * K:
        p = np.arange(start, end, dtype=np.int64)
    else:
        p = np.concatenate([np.arange(start, start + K), np.arange(end - K, end)]).astype(np.int64)
    if p.size == 0:
        return np.inf
    env = np.zeros(p.size)
    for j in range(N // hop + 2):
        t = p // hop - j
        n = p - t * hop
        ok = (t >= 0) & (t < T) & (n < N)
        env += np.where(ok, w2[np.clip(n, 0, N - 1)], 0.0)
    return float(env.min())


def istft(spec: torch.Tensor, n_fft: int, hop_length=None, win_length=None, window=None, center: bool = True,
          normalized: bool = False, length=None) -> torch.Tensor:
    """Weighted overlap-add inverse of ``stft``; raises, like torch.istft,
    where the summed squared window vanishes inside the output."""
    n_fft, hop, wl = _lengths(n_fft, hop_length, win_length)
    if not isinstance(spec, torch.Tensor) or spec.device.type != "cuda":
        raise TypeError("tfx runs on the GPU only")
    squeeze = spec.dim() == 2
    s3 = spec.unsqueeze(0) if squeeze else spec
    if s3.dim() != 3 or s3.shape[1] != n_fft // 2 + 1:
        raise ValueError("spectrum must be [C, n_fft/2 + 1, T]")
    C, F, T = s3.shape
    if T < 1:
        raise ValueError("no frames")
    fm = s3.transpose(1, 2).to(torch.complex64).contiguous()   # frame-major [C, T, F]
    total = n_fft + hop * (T - 1)
    start = n_fft // 2 if center else 0
    L = (total - 2 * (n_fft // 2) if center else total) if length is None else int(length)
    wnp = np.ones(wl) if window is None else torch.as_tensor(window).detach().double().cpu().numpy()
    full = np.zeros(n_fft)
    full[(n_fft - wl) // 2:(n_fft - wl) // 2 + wl] = wnp
    if _envelope_min(full * full, hop, T, start, min(start + L, total)) < 1e-11:
        raise ValueError("window overlap-add is zero somewhere (NOLA fails)")
    w = _window(window, wl, spec.device)
    y = torch.empty((C, L), dtype=torch.float32, device=spec.device)
    lib.call("tfx_istft", fm.data_ptr(), C, T, n_fft, hop, _ptr(w), wl, int(bool(center)), int(bool(normalized)),
             y.data_ptr() if L else None, L, max(L, 1), _stream(spec.device))
    return y[0] if squeeze else y


def rfft(x: torch.Tensor) -> torch.Tensor:
    """One-sided DFT of every row of a float32 tensor [..., n] (n a power of
    two from 16 to 4096): complex64 [..., n/2 + 1], numpy.fft.rfft's
    convention (no scaling)."""
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
        raise TypeError("tfx runs on the GPU only")
    if x.dtype != torch.float32:
        raise TypeError("rfft takes float32 rows")
    n = x.shape[-1]
    rows = x.reshape(-1, n)
    if rows.stride(1) != 1:
        rows = rows.contiguous()
    B = rows.shape[0]
    ld = rows.stride(0) if B > 1 else n
    spec = torch.empty((B, n // 2 + 1), dtype=torch.complex64, device=x.device)
    lib.call("tfx_rfft", _ptr(rows) if B else None, B, n, ld, spec.data_ptr() if B else None, _stream(x.device))
    return spec.reshape(*x.shape[:-1], n // 2 + 1)


def irfft(spec: torch.Tensor, n: int) -> torch.Tensor:
    """Inverse of ``rfft`` for rows of n samples: float32 [..., n] from
    complex [..., n/2 + 1] (the imaginary parts of bins 0 and n/2 are
    ignored), numpy.fft.irfft's convention (1/n scaling)."""
    if not isinstance(spec, torch.Tensor) or spec.device.type != "cuda":
        raise TypeError("tfx runs on the GPU only")
    n = int(n)
    if spec.shape[-1] != n // 2 + 1:
        raise ValueError("spectrum has %d bins, n = %d needs %d" % (spec.shape[-1], n, n // 2 + 1))
    s2 = spec.reshape(-1, n // 2 + 1).to(torch.complex64).contiguous()
    B = s2.shape[0]
    y = torch.empty((B, n), dtype=torch.float32, device=spec.device)
    lib.call("tfx_irfft", s2.data_ptr() if B else None, B, n, y.data_ptr() if B else None, n, _stream(spec.device))
    return y.reshape(*spec.shape[:-1], n)

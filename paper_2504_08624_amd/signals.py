"""Seeded synthetic test signals (float64 on the host, rounded once to fp32).

The paper's benchmarks filter white noise drawn with numpy's Gaussian
generator at 44.1 kHz, 5 s to 600 s, 1 to 12 channels (Sec. 4, "Performance
Evaluation").  The workloads here follow the same recipe and add two other
audio test signals: 1/f ("pink") noise and an exponential sine sweep.

This module only draws numbers: it holds no filtering arithmetic, so both the
GPU path and the FP64 oracle can take their inputs from it.
"""
from __future__ import annotations

import numpy as np


def rng(*key: int) -> np.random.Generator:
    """PCG64 generator keyed by a tuple of small integers, e.g. (config, channel)."""
    return np.random.default_rng(list(key))


def white(n: int, key, sigma: float = 0.1) -> np.ndarray:
    """Gaussian white noise, standard deviation ``sigma``, float64."""
    return rng(*key).standard_normal(int(n)) * sigma


def pink(n: int, key, rms: float = 0.1) -> np.ndarray:
    """1/f noise: a white Gaussian spectrum scaled by 1/sqrt(f) with the DC bin
    zeroed, transformed back and scaled to the given RMS.  float64."""
    n = int(n)
    w = rng(*key).standard_normal(n)
    spec = np.fft.rfft(w)
    f = np.arange(spec.size, dtype=np.float64)
    spec[0] = 0.0
    spec[1:] /= np.sqrt(f[1:])
    x = np.fft.irfft(spec, n)
    r = np.sqrt(np.mean(x * x)) if n else 1.0
    return x * (rms / r) if r > 0 else x


def log_sweep(n: int, fs: float, f1: float = 20.0, f2: float = 20000.0,
              amp: float = 0.5) -> np.ndarray:
    """Exponential (logarithmic) sine sweep from f1 to f2 over n samples."""
    n = int(n)
    T = n / fs
    t = np.arange(n, dtype=np.float64) / fs
    k = np.log(f2 / f1)
    return amp * np.sin(2.0 * np.pi * f1 * T / k * (np.exp(t * k / T) - 1.0))


def to_f32(x: np.ndarray) -> np.ndarray:
    """Round to float32 (round-to-nearest-even), C-contiguous."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))

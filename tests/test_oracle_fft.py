"""Pins of the FP64 batched real-FFT oracle (the FFT named in Sec. 5's
roadmap): brute-force DFT sums in scalar loops, closed forms for a delta and
a bin-centred tone, Parseval, the round trip, the inverse's disregard of the
imaginary parts of bins 0 and n/2, and numpy's FFT as an independent library
routine."""
import math

import numpy as np
import pytest

from oracle import fft as F


@pytest.mark.parametrize("n", [8, 16])
def test_brute_force_dft_sums(n):
    g = np.random.default_rng(n)
    x = g.standard_normal((3, n))
    X = F.rfft(x)
    assert X.shape == (3, n // 2 + 1)
    for b in range(3):
        for k in range(n // 2 + 1):
            acc = 0.0 + 0.0j
            for m in range(n):
                ang = 2.0 * math.pi * k * m / n
                acc += x[b, m] * complex(math.cos(ang), -math.sin(ang))
            assert abs(X[b, k] - acc) < 1e-12
    y = F.irfft(X, n)
    for b in range(3):
        for m in range(n):
            acc = X[b, 0].real + X[b, n // 2].real * (-1) ** m
            for k in range(1, n // 2):
                ang = 2.0 * math.pi * k * m / n
                acc += 2.0 * (X[b, k] * complex(math.cos(ang), math.sin(ang))).real
            assert abs(y[b, m] - acc / n) < 1e-12


@pytest.mark.parametrize("n", [16, 256, 4096])
def test_delta_and_tone_closed_forms(n):
    m0 = n // 3
    d = np.zeros(n)
    d[m0] = 1.0
    k = np.arange(n // 2 + 1)
    assert np.max(np.abs(F.rfft(d) - np.exp(-2j * np.pi * k * m0 / n))) < 1e-12
    k0, A, phi = n // 4 - 1, 0.7, 0.4
    tone = A * np.cos(2 * np.pi * k0 * np.arange(n) / n + phi)
    X = F.rfft(tone)
    expect = np.zeros(n // 2 + 1, complex)
    expect[k0] = A * n / 2 * np.exp(1j * phi)
    assert np.max(np.abs(X - expect)) < 1e-9 * n


@pytest.mark.parametrize("n", [16, 1024])
def test_parseval_and_round_trip(n):
    g = np.random.default_rng(n + 1)
    x = g.standard_normal((4, n))
    X = F.rfft(x)
    e_t = np.sum(x * x, axis=1)
    e_f = (np.abs(X[:, 0]) ** 2 + np.abs(X[:, -1]) ** 2 + 2 * np.sum(np.abs(X[:, 1:-1]) ** 2, axis=1)) / n
    assert np.max(np.abs(e_t - e_f) / e_t) < 1e-12
    assert np.max(np.abs(F.irfft(X, n) - x)) < 1e-12


def test_inverse_ignores_imaginary_parts_of_the_end_bins():
    g = np.random.default_rng(5)
    X = g.standard_normal((2, 33)) + 1j * g.standard_normal((2, 33))
    Y = X.copy()
    Y[:, 0] = Y[:, 0].real
    Y[:, 32] = Y[:, 32].real
    assert np.array_equal(F.irfft(X, 64), F.irfft(Y, 64))


@pytest.mark.parametrize("n", [32, 2048])
def test_matches_numpy_fft(n):
    g = np.random.default_rng(n + 2)
    x = g.standard_normal((2, 3, n))
    assert np.max(np.abs(F.rfft(x) - np.fft.rfft(x, axis=-1))) < 1e-10 * n
    X = g.standard_normal((5, n // 2 + 1)) + 1j * g.standard_normal((5, n // 2 + 1))
    assert np.max(np.abs(F.irfft(X, n) - np.fft.irfft(X, n, axis=-1))) < 1e-12

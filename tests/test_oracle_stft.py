"""Pins of the FP64 STFT / ISTFT oracle (the transform named in Sec. 5's
roadmap): brute-force DFT sums, closed forms for bin-centred tones,
Parseval per frame, perfect reconstruction, and torch's own CPU transforms in
float64 as an independent library routine."""
import math

import numpy as np
import pytest
import torch

from oracle import stft as S


def _reflect_index(p, N):
    """Independent reflect map of a padded index back into [0, N)."""
    while p < 0 or p >= N:
        p = -p if p < 0 else 2 * (N - 1) - p
    return p


def test_brute_force_dft_of_reflect_padded_frames():
    g = np.random.default_rng(1)
    x = g.standard_normal((2, 37))
    n_fft, hop, win = 8, 3, g.uniform(0.2, 1.0, 6)
    X = S.stft(x, n_fft, hop, win, center=True)
    T = 1 + (37 + 8 - 8) // 3
    assert X.shape == (2, T, 5)
    w = np.concatenate([[0.0], win, [0.0]])   # 6 taps in the middle of 8
    for c in range(2):
        for t in range(T):
            for k in range(5):
                acc = 0.0 + 0.0j
                for n in range(n_fft):
                    v = x[c, _reflect_index(t * hop + n - n_fft // 2, 37)]
                    ang = 2.0 * math.pi * k * n / n_fft
                    acc += w[n] * v * complex(math.cos(ang), -math.sin(ang))
                assert abs(X[c, t, k] - acc) < 1e-12


@pytest.mark.parametrize("n_fft,hop,win_len,center,normalized", [(64, 16, 64, True, False), (256, 100, 200, True, True),
                                                                 (32, 32, 32, False, False), (128, 7, 90, False, True)])
def test_matches_torch_stft_in_float64(n_fft, hop, win_len, center, normalized):
    g = np.random.default_rng(n_fft + hop)
    x = g.standard_normal((3, 1000))
    win = g.uniform(0.1, 1.0, win_len)
    X = S.stft(x, n_fft, hop, win, center=center, normalized=normalized)
    ref = torch.stft(torch.from_numpy(x), n_fft, hop, win_len, torch.from_numpy(win), center=center,
                     pad_mode="reflect", normalized=normalized, onesided=True, return_complex=True)
    ref = ref.numpy().transpose(0, 2, 1)
    assert X.shape == ref.shape
    assert np.max(np.abs(X - ref)) < 1e-10


def test_bin_centred_tone_closed_form():
    n_fft, k0 = 64, 5
    n = np.arange(10 * n_fft)
    x = np.cos(2 * np.pi * k0 * n / n_fft + 0.3)
    X = S.stft(x, n_fft, n_fft, None, center=False)
    assert X.shape == (10, 33)
    expect = np.zeros(33, complex)
    expect[k0] = n_fft / 2 * np.exp(0.3j)
    assert np.max(np.abs(X - expect[None, :])) < 1e-10


def test_parseval_per_frame():
    g = np.random.default_rng(2)
    x = g.standard_normal(3000)
    n_fft, hop = 512, 128
    win = S.hann(n_fft)
    X = S.stft(x, n_fft, hop, win, center=True)
    xp = S.padded(x, n_fft, True)[0]
    for t in (0, 7, X.shape[0] - 1):
        seg = win * xp[t * hop:t * hop + n_fft]
        e = np.abs(X[t]) ** 2
        spec_energy = (e[0] + e[-1] + 2 * e[1:-1].sum()) / n_fft
        assert abs(spec_energy - np.sum(seg ** 2)) < 1e-9 * np.sum(seg ** 2)


@pytest.mark.parametrize("n_fft,hop,center", [(256, 64, True), (512, 128, False), (64, 16, True)])
def test_istft_reconstructs_and_matches_torch(n_fft, hop, center):
    g = np.random.default_rng(n_fft)
    x = g.standard_normal((2, 4000))
    win = S.hann(n_fft) + 0.05          # nonzero at the ends: the envelope never vanishes
    X = S.stft(x, n_fft, hop, win, center=center)
    y = S.istft(X, n_fft, hop, win, center=center, length=4000 if center else None)
    ref = torch.istft(torch.from_numpy(X.transpose(0, 2, 1).copy()), n_fft, hop, n_fft, torch.from_numpy(win),
                      center=center, length=4000 if center else None).numpy()
    assert y.shape == ref.shape
    assert np.max(np.abs(y - ref)) < 1e-10
    m = y.shape[1]
    lo, hi = (0, m) if center else (n_fft, m - n_fft)    # without padding the ends lack full overlap
    assert np.max(np.abs(y[:, lo:hi] - x[:, lo:hi])) < 1e-10


def test_istft_length_zero_extends_and_nola_failure_raises():
    n_fft, hop = 64, 16
    X = S.stft(np.random.default_rng(3).standard_normal(500), n_fft, hop, S.hann(n_fft))
    y = S.istft(X, n_fft, hop, S.hann(n_fft), length=600)
    assert y.shape == (600,) and np.all(y[n_fft // 2 + hop * (X.shape[0] - 1):] == 0.0)
    with pytest.raises(ValueError, match="NOLA"):
        S.istft(S.stft(np.ones(500), 16, 32, None, center=False), 16, 32, None, center=False)


def test_frame_counts():
    assert S.num_frames(1000, 256, 64, True) == 1 + 1000 // 64
    assert S.num_frames(1000, 256, 64, False) == 1 + (1000 - 256) // 64
    assert S.num_frames(100, 256, 64, False) == 0


def test_single_frame_helper_agrees_with_the_framed_transform():
    g = np.random.default_rng(4)
    x = g.standard_normal(3000)
    for center in (True, False):
        X = S.stft(x, 256, 77, S.hann(200), center=center, normalized=True)
        for t in (0, 5, X.shape[0] - 1):
            assert np.max(np.abs(S.frame(x, 256, 77, S.hann(200), center, t, True) - X[t])) < 1e-12

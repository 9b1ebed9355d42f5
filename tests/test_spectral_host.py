"""Host-side logic of the STFT binding: the envelope check that decides when
the inverse raises (its shortcut for long signals samples only the ends and
one period of the interior) against the oracle's full envelope."""
import numpy as np
import pytest

from oracle import stft as OS
from paper_2504_08624_amd.spectral import _envelope_min


@pytest.mark.parametrize("n_fft,hop,wl,T,center", [(64, 16, 64, 3, True), (64, 16, 40, 500, True),
                                                   (256, 100, 200, 2000, False), (32, 32, 32, 50, False),
                                                   (16, 40, 16, 20, False), (2048, 512, 2048, 11251, True),
                                                   (512, 128, 300, 9, True)])
def test_envelope_minimum_matches_the_full_envelope(n_fft, hop, wl, T, center):
    g = np.random.default_rng(n_fft + hop + T)
    for win in (OS.hann(wl), g.uniform(0.0, 1.0, wl), np.ones(wl)):
        full = OS.full_window(win, n_fft)
        env = OS.envelope(win, n_fft, hop, T)
        start = n_fft // 2 if center else 0
        end = env.size - (n_fft // 2 if center else 0)
        got = _envelope_min(full * full, hop, T, start, end)
        assert abs(got - env[start:end].min()) <= 1e-12 * max(1.0, env.max())

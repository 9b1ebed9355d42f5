"""Seeded synthetic workloads (signals + FP64-designed, fp32-rounded coefficients).

Shapes follow the paper's benchmark recipe (Sec. 4: numpy white noise at a
fixed audio rate, 5-600 s, 1-12 channels; an 8-channel, 2-minute, 4-filter
IIR chain) scaled to one MI355X:

  chain_short  2 x 480,000 @48 kHz, white noise; 101-tap LP | Butterworth HP (2 SOS)
  chain_mid    8 x 5,760,000 @48 kHz, pink noise + log sweep;
               1023-tap BP | Chebyshev-I LP (4 SOS) | 2 peaking EQs
  fir_long     64 x 5,760,000 @96 kHz, white noise; 8191-tap LP
  ragged       256 clips @44.1 kHz, 1-30 s, 1-16 ch, own random cascade (1-6 SOS)
  learnable    32 x 2 x 192,000 @48 kHz; 255-tap FIR | 8 biquads (pole/zero)
  high_q       2 x 30 s @48 kHz, 6 resonators with pole radius in [0.999, 0.99995]

Every size can be overridden (C, N, clip count) so the tests can run the same
recipe at oracle-friendly sizes.  Nothing here filters a signal.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import design, signals


@dataclass
class Workload:
    name: str
    fs: float
    x: np.ndarray                       # float32 [C, N]
    stages: list                        # [("fir", f32[M]) | ("sos", f32[S, 5])]
    extra: dict = field(default_factory=dict)

    @property
    def samples(self) -> int:
        return int(self.x.size)


def _stack(rows, N):
    return np.ascontiguousarray(np.stack(rows).astype(np.float32)) if rows else np.zeros((0, N), np.float32)


def chain_short(C: int = 2, N: int = 480_000) -> Workload:
    fs = 48_000.0
    x = _stack([signals.white(N, (1, c)) for c in range(C)], N)
    h = design.fir_lowpass(101, 8_000.0, fs).astype(np.float32)
    hp = design.butterworth(4, 100.0, fs, "highpass").astype(np.float32)
    return Workload("chain_short", fs, x, [("fir", h), ("sos", hp)])


def chain_mid(C: int = 8, N: int = 5_760_000) -> Workload:
    fs = 48_000.0
    sweep = signals.log_sweep(N, fs, 20.0, 20_000.0, 0.5)
    x = _stack([signals.pink(N, (2, c)) + sweep for c in range(C)], N)
    h = design.fir_bandpass(1023, 200.0, 6_000.0, fs).astype(np.float32)
    cheb = design.chebyshev1(8, 1.0, 12_000.0, fs).astype(np.float32)
    peq = np.concatenate([design.peaking(250.0, 0.7, 6.0, fs),
                          design.peaking(3_000.0, 8.0, -12.0, fs)]).astype(np.float32)
    return Workload("chain_mid", fs, x, [("fir", h), ("sos", cheb), ("sos", peq)])


def chain_mid_short_fir(C: int = 8, N: int = 5_760_000) -> Workload:
    """chain_short's filters on chain_mid's shape (8 x 5.76 M)."""
    w = chain_short(C=C, N=N)
    w.name = "chain_short_large"
    return w


def fir_long(C: int = 64, N: int = 5_760_000, M: int = 8191) -> Workload:
    fs = 96_000.0
    x = _stack([signals.white(N, (3, c)) for c in range(C)], N)
    h = design.fir_lowpass(M, 8_000.0, fs).astype(np.float32)
    return Workload("fir_long", fs, x, [("fir", h)])


def ragged(nclips: int = 256, max_seconds: float = 30.0, min_seconds: float = 1.0,
           max_channels: int = 16, fs: float = 44_100.0):
    """List of (x_i [C_i, N_i] f32, sos_i [S_i, 5] f32)."""
    g = signals.rng(4)
    Ns = np.rint(g.uniform(min_seconds, max_seconds, nclips) * fs).astype(np.int64)
    Cs = g.integers(1, max_channels + 1, nclips)
    Ss = g.integers(1, 7, nclips)
    clips = []
    for i in range(nclips):
        sec = design.random_sections(signals.rng(4, 1000 + i), int(Ss[i])).astype(np.float32)
        x = _stack([signals.white(int(Ns[i]), (4, i, c)) for c in range(int(Cs[i]))], int(Ns[i]))
        clips.append((x, sec))
    return clips


def learnable(B: int = 32, C: int = 2, N: int = 192_000):
    """Differentiable chain: returns (x [B*C, N] f32, init params, target stages).
    Parameters: taps h [255]; pole/zero logits (rho_p, phi_p, rho_z, phi_z) and
    gains k per section; r = 0.99 sigmoid(rho), theta = pi sigmoid(phi)."""
    fs = 48_000.0
    x = _stack([signals.white(N, (5, c)) for c in range(B * C)], N)
    g = signals.rng(5, 999)
    target = [("fir", design.fir_lowpass(255, 4_000.0, fs).astype(np.float32)),
              ("sos", design.random_sections(g, 8, 0.3, 0.9).astype(np.float32))]
    gi = signals.rng(5, 998)
    params = {
        "h": design.fir_lowpass(255, 6_000.0, fs).astype(np.float32),
        "rho_p": gi.normal(0.0, 1.0, 8), "phi_p": gi.normal(0.0, 1.0, 8),
        "rho_z": gi.normal(0.0, 1.0, 8), "phi_z": gi.normal(0.0, 1.0, 8),
        "k": np.ones(8),
    }
    return x, params, target


def high_q(C: int = 2, N: int = 1_440_000) -> Workload:
    fs = 48_000.0
    g = signals.rng(6)
    sec = design.random_sections(g, 6, 0.999, 0.99995)
    x = _stack([signals.white(N, (6, c)) for c in range(C)], N)
    return Workload("high_q", fs, x, [("sos", sec.astype(np.float32))])

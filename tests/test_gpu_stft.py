"""GPU parity of the STFT / ISTFT (tfx_stft, tfx_istft) against the FP64
oracle: every transform size 16 .. 4096, centred and plain framing, windows
shorter than the frame, rectangular windows, odd and single frame counts,
hops longer than the frame, normalisation, explicit output lengths; the
round trip; and sampled frames at the full size of the audio benchmark
signal.

Tolerance: per-channel relative RMS error 1e-5 over all spectrum values (or
output samples).  An fp32 radix-4 FFT of 2^L points accumulates about
sqrt(L) rounding steps of relative size 2^-24 per value (a few 1e-7 at
L = 12); 1e-5 is the bound the fp32 FFT-based FIR is held to as well."""
import numpy as np
import pytest
import torch

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import signals, spectral, workloads
from oracle import stft as OS
from tests.metrics import assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-5


def _x(C, N, key):
    return signals.to_f32(np.stack([signals.white(N, (*key, c), 0.1) for c in range(C)]).reshape(C, N))


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _ri(spec_ctf):
    """[C, T, F] complex -> [C, 2 T F] real, for the per-channel metric."""
    s = np.asarray(spec_ctf)
    return np.concatenate([s.real.reshape(s.shape[0], -1), s.imag.reshape(s.shape[0], -1)], axis=1)


def _win(kind, n, seed):
    if kind is None:
        return None
    if kind == "hann":
        return OS.hann(n).astype(np.float32)
    return np.random.default_rng(seed).uniform(0.2, 1.0, n).astype(np.float32)


CASES = [  # n_fft, hop, win_length, window, center, normalized, C, N
    (16, 4, 16, "hann", True, False, 2, 1001),
    (32, 7, 20, "rand", False, True, 3, 2000),
    (64, 64, 64, None, True, False, 1, 4097),
    (128, 200, 100, "rand", False, False, 2, 30000),    # hop longer than the frame
    (256, 64, 256, "hann", True, True, 2, 50001),
    (512, 128, 400, "rand", True, False, 3, 40000),
    (1024, 256, 1024, "hann", True, False, 2, 100000),
    (2048, 512, 2048, "hann", True, False, 2, 96001),
    (2048, 333, 1500, "rand", False, True, 1, 77777),
    (4096, 1024, 4096, "hann", True, False, 2, 65536),
    (4096, 4096, 4096, None, False, False, 1, 4096),    # exactly one frame
]


@pytest.mark.parametrize("n_fft,hop,wl,wkind,center,normalized,C,N", CASES)
def test_stft_matches_the_oracle(n_fft, hop, wl, wkind, center, normalized, C, N):
    x = _x(C, N, (600, n_fft, hop))
    w = _win(wkind, wl, n_fft + hop)
    X = tfx.stft(torch.from_numpy(x).to(DEV), n_fft, hop, wl, None if w is None else torch.from_numpy(w),
                 center=center, normalized=normalized)
    ref = OS.stft(x, n_fft, hop, w if w is not None else (None if wl == n_fft else np.ones(wl)), center, normalized)
    assert tuple(X.shape) == (C, n_fft // 2 + 1, ref.shape[1])
    got = _cpu(X).transpose(0, 2, 1)
    assert_close(_ri(got), _ri(ref), TOL, "stft n_fft=%d hop=%d" % (n_fft, hop))


# the inverse needs the summed squared window to stay positive: frames must
# overlap, and a window shorter than an uncentred frame leaves the first
# samples uncovered (torch.istft rejects both as well)
@pytest.mark.parametrize("n_fft,hop,wl,wkind,center,normalized,C,N",
                         [c for c in CASES if c[1] <= c[0] and (c[4] or c[2] == c[0])])
def test_istft_matches_the_oracle(n_fft, hop, wl, wkind, center, normalized, C, N):
    x = _x(C, N, (601, n_fft, hop))
    w = _win(wkind, wl, n_fft + hop + 1)
    if w is not None:
        w = (w + 0.05).astype(np.float32)   # keep the envelope away from zero at the frame ends
    wref = w if w is not None else (None if wl == n_fft else np.ones(wl))
    spec = OS.stft(x, n_fft, hop, wref, center, normalized).astype(np.complex64)
    # perturb so the input is not an exact STFT (the overlap-add then really averages)
    g = np.random.default_rng(n_fft)
    spec = (spec + 0.01 * (g.standard_normal(spec.shape) + 1j * g.standard_normal(spec.shape))).astype(np.complex64)
    length = N if center else None
    y = tfx.istft(torch.from_numpy(spec.transpose(0, 2, 1).copy()).to(DEV), n_fft, hop, wl,
                  None if w is None else torch.from_numpy(w), center=center, normalized=normalized, length=length)
    ref = OS.istft(spec, n_fft, hop, wref, center, normalized, length)
    assert_close(_cpu(y), ref, TOL, "istft n_fft=%d hop=%d" % (n_fft, hop))


@pytest.mark.parametrize("n_fft,hop", [(16, 4), (512, 128), (4096, 1024)])
def test_round_trip_restores_the_signal(n_fft, hop):
    x = _x(2, 20000, (602, n_fft))
    xt = torch.from_numpy(x).to(DEV)
    w = torch.from_numpy(OS.hann(n_fft).astype(np.float32)).to(DEV)
    y = tfx.istft(tfx.stft(xt, n_fft, hop, window=w), n_fft, hop, window=w, length=20000)
    assert_close(_cpu(y), x, TOL, "round trip n_fft=%d" % n_fft)


def test_edge_cases():
    # one channel given 1-D; shortest centred signal; output length past the frames (zeros)
    x = _x(1, 129, (603,))[0]
    X = tfx.stft(torch.from_numpy(x).to(DEV), 256, 64)
    assert tuple(X.shape) == (129, 1 + 129 // 64)
    ref = OS.stft(x, 256, 64, None, True)
    assert_close(_ri(_cpu(X).T[None]), _ri(ref[None]), TOL, "short centred signal")
    w = OS.hann(256).astype(np.float32) + 0.1
    spec = OS.stft(x, 256, 64, w, True).astype(np.complex64)
    y = tfx.istft(torch.from_numpy(spec.T.copy()).to(DEV), 256, 64, window=torch.from_numpy(w), length=400)
    refy = OS.istft(spec, 256, 64, w, True, length=400)
    assert_close(_cpu(y)[None], refy[None], TOL, "length past the frames")
    covered = 256 + 64 * (spec.shape[0] - 1) - 128
    assert covered < 400 and np.all(_cpu(y)[covered:] == 0.0)
    # no frames at all
    X0 = tfx.stft(torch.zeros(2, 100, device=DEV), 256, 64, center=False)
    assert tuple(X0.shape) == (2, 129, 0)
    # a vanishing envelope is an error, as in torch.istft
    with pytest.raises(ValueError, match="NOLA"):
        tfx.istft(torch.zeros(129, 10, dtype=torch.complex64, device=DEV), 256, 512, center=False)


def test_full_size_audio_signal_sampled_frames():
    """The audio benchmark's signal (8 x 5,760,000 samples of 1/f noise plus
    a log sweep), n_fft 2048, hop 512, Hann: 48 sampled frames, including the
    first and last of each channel, against the oracle's single-frame
    transform."""
    n_fft, hop = 2048, 512
    x = workloads.chain_mid().x
    C, N = x.shape
    w = OS.hann(n_fft).astype(np.float32)
    X = tfx.stft(torch.from_numpy(x).to(DEV), n_fft, hop, window=torch.from_numpy(w).to(DEV))
    T = spectral.num_frames(N, n_fft, hop, True)
    assert tuple(X.shape) == (C, n_fft // 2 + 1, T)
    g = np.random.default_rng(5)
    picks = [(c, t) for c in range(C) for t in (0, T - 1)] + [(int(g.integers(C)), int(g.integers(T)))
                                                              for _ in range(32)]
    Xc = X.transpose(1, 2)
    got = np.stack([Xc[c, t].cpu().numpy() for c, t in picks])
    ref = np.stack([OS.frame(x[c], n_fft, hop, w, True, t) for c, t in picks])
    assert_close(_ri(got[None]), _ri(ref[None]), TOL, "sampled frames")


def test_row_strides_through_the_c_abi():
    """Input rows with a stride larger than their length (a column slice) and
    an output with a padded row stride, called through the C ABI directly."""
    from paper_2504_08624_amd import lib
    C, N, n_fft, hop = 3, 7000, 512, 160
    wide = _x(C, N + 333, (605,))
    w = OS.hann(n_fft).astype(np.float32) + 0.05
    xt = torch.from_numpy(wide).to(DEV)[:, :N]
    assert xt.stride(0) == N + 333
    X = tfx.stft(xt, n_fft, hop, window=torch.from_numpy(w))
    ref = OS.stft(wide[:, :N], n_fft, hop, w, True)
    assert_close(_ri(_cpu(X).transpose(0, 2, 1)), _ri(ref), TOL, "strided input")
    T = ref.shape[1]
    spec = torch.from_numpy(ref.astype(np.complex64)).to(DEV).contiguous()
    wt = torch.from_numpy(w).to(DEV)
    ldy = N + 100
    y = torch.full((C, ldy), 7.0, dtype=torch.float32, device=DEV)
    lib.call("tfx_istft", spec.data_ptr(), C, T, n_fft, hop, wt.data_ptr(), n_fft, 1, 0, y.data_ptr(), N, ldy,
             torch.cuda.current_stream().cuda_stream)
    yy = _cpu(y)
    assert_close(yy[:, :N], OS.istft(ref.astype(np.complex64), n_fft, hop, w, True, length=N), TOL, "strided output")
    assert np.all(yy[:, N:] == 7.0)   # the row padding is left alone

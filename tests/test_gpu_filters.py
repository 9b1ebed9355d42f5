"""GPU parity of the filter classes and the Wave pipe (Sec. 3) against the FP64
oracle: the pipe's fused chain, the three chain forms the paper shows (a
module class, a Sequential with the rate given, a Sequential bound by the
pipe), mixed FIR/IIR pipes, and gradients of trainable stages."""
import numpy as np
import pytest
import torch
from torch import nn
from torch.nn import Sequential

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import signals
from oracle import oracle as O
from tests.metrics import TOL_IIR_F32, assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FS = 44100.0


def _signal(C, N, key):
    return signals.to_f32(np.stack([signals.white(N, (*key, c), 0.1) for c in range(C)]).reshape(C, N))


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _stages(filters):
    return [(f.kind, f.coefficients("cpu").numpy()) for f in filters]


def test_pipe_runs_the_fused_chain():
    x = _signal(2, 3 * 3072 + 5, (500,))
    w = tfx.Wave(torch.from_numpy(x).to(DEV), FS)
    hs, ls = tfx.HiShelving(1000), tfx.LoShelving(2000)
    out = w | hs | ls
    y = _cpu(out.y)
    assert not out.pending and out.fs == FS
    assert_close(y, O.chain(x, _stages([hs, ls])), TOL_IIR_F32, "HiShelving | LoShelving")


def test_the_three_chain_forms_agree():
    x = _signal(3, 20000, (501,))
    xt = torch.from_numpy(x).to(DEV)
    sig = tfx.Wave(xt, FS)

    class FilterChain(nn.Module):
        def __init__(self, sample_rate):
            super().__init__()
            self.f1 = tfx.HiShelving(1000, sample_rate)
            self.f2 = tfx.LoShelving(2000, sample_rate)

        def forward(self, y):
            return self.f2(self.f1(y))

    a = _cpu(FilterChain(sig.fs)(sig.y))
    b = _cpu(Sequential(tfx.HiShelving(1000, sample_rate=sig.fs), tfx.LoShelving(2000, sample_rate=sig.fs))(sig.y))
    c = _cpu((sig | Sequential(tfx.HiShelving(1000), tfx.LoShelving(2000))).y)
    ref = O.chain(x, _stages([tfx.HiShelving(1000, FS), tfx.LoShelving(2000, FS)]))
    for name, y in (("class", a), ("sequential", b), ("pipe", c)):
        assert_close(y, ref, TOL_IIR_F32, name)


def test_mixed_fir_and_iir_pipe():
    x = _signal(4, 50000, (502,))
    fs = [tfx.WindowedSincFIR(300.0, num_taps=255, cutoff_hi=6000.0), tfx.Butterworth(120.0, order=4, btype="highpass"),
          tfx.Peaking(1000.0, q=2.0, gain_db=4.0), tfx.Chebyshev1(9000.0, order=6, ripple_db=0.5)]
    w = tfx.Wave(torch.from_numpy(x).to(DEV), FS)
    for f in fs:
        w = w | f
    assert len(w.pending) == 4
    assert_close(_cpu(w.y), O.chain(x, _stages(fs)), TOL_IIR_F32, "FIR | Butterworth | Peaking | Chebyshev1")


def test_pending_stages_run_before_another_module():
    x = _signal(1, 5000, (503,))
    w = tfx.Wave(torch.from_numpy(x).to(DEV), FS) | tfx.Peaking(2000.0, gain_db=-3.0)
    w = w | (lambda y: 0.5 * y)
    ref = 0.5 * O.chain(x, _stages([tfx.Peaking(2000.0, FS, gain_db=-3.0)]))
    assert_close(_cpu(w.y), ref, TOL_IIR_F32, "pending stage then a gain")


def test_trainable_stages_get_gradients_through_the_pipe():
    x = _signal(2, 4000, (504,))
    g = _signal(2, 4000, (505,))
    h = np.hanning(33).astype(np.float32) / 16.0
    sec = np.array([[0.5, 0.2, 0.1, -0.6, 0.3]], np.float32)
    fir, sos = tfx.FIR(h, learnable=True).to(DEV), tfx.SOS(sec, learnable=True).to(DEV)
    y = (tfx.Wave(torch.from_numpy(x).to(DEV), FS) | fir | sos).y
    (y * torch.from_numpy(g).to(DEV)).sum().backward()
    rgx, (rgh, rgs) = O.chain_backward(g, x, [("fir", h), ("sos", sec)])
    gh, gs = _cpu(fir.taps.grad), _cpu(sos.sections.grad)
    assert np.linalg.norm(gh - rgh) <= 1e-4 * np.linalg.norm(rgh)
    assert np.linalg.norm(gs - np.reshape(rgs, gs.shape)) <= 1e-4 * np.linalg.norm(rgs)


def test_further_designed_families_through_the_pipe():
    x = _signal(3, 4 * 3072 + 29, (506,))
    fs = [tfx.Chebyshev2(5000.0, order=6, atten_db=50.0), tfx.ButterworthBand(300.0, 3000.0, order=3),
          tfx.Notch(1000.0, q=10.0), tfx.AllPass(2000.0, q=0.7), tfx.BandPass(800.0, q=1.5),
          tfx.ButterworthBand(4000.0, 6000.0, order=2, btype="bandstop")]
    w = tfx.Wave(torch.from_numpy(x).to(DEV), FS)
    for f in fs:
        w = w | f
    assert_close(_cpu(w.y), O.chain(x, _stages(fs)), TOL_IIR_F32, "Chebyshev2 | bands | notch | all-pass")


def _stable_tf(g, zeros_pairs, poles_pairs, rmax):
    def poly(n, r):
        roots = []
        for _ in range(n):
            rr, t = r * np.sqrt(g.uniform(0.1, 1.0)), g.uniform(0.1, np.pi - 0.1)
            roots += [rr * np.exp(1j * t), rr * np.exp(-1j * t)]
        roots.append(g.uniform(-r, r))
        return np.real(np.poly(roots))
    return 0.3 * poly(zeros_pairs, 1.2), poly(poles_pairs, rmax)


@pytest.mark.parametrize("seed,zp,pp,C,N", [(11, 3, 3, 3, 3 * 3072 + 17), (12, 1, 4, 2, 5000), (13, 4, 2, 1, 100)])
def test_lfilter_matches_the_oracle_on_its_sections(seed, zp, pp, C, N):
    from scipy.signal import lfilter as sp_lfilter
    from paper_2504_08624_amd import design
    g = np.random.default_rng(seed)
    b, a = _stable_tf(g, zp, pp, 0.97)
    x = _signal(C, N, (507, seed))
    y = _cpu(tfx.lfilter(torch.from_numpy(x).to(DEV), b, a))
    rows = design.tf2sos(b, a).astype(np.float32)
    assert_close(y, O.sos(x, rows), TOL_IIR_F32, "lfilter vs oracle cascade")
    # the direct form in FP64 differs only by the fp32 rounding of the sections
    ref = sp_lfilter(b, a, x.astype(np.float64), axis=1)
    assert_close(y, ref, TOL_IIR_F32, "lfilter vs FP64 direct form")


def test_lfilter_with_a_scalar_denominator_is_a_fir():
    x = _signal(2, 7000, (508,))
    h = np.hanning(21)
    y = _cpu(tfx.lfilter(torch.from_numpy(x).to(DEV), h, [2.0]))
    assert_close(y, O.fir(x, (h / 2.0).astype(np.float32)), 1e-5, "lfilter FIR form")

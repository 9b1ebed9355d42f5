"""Host-side behaviour of the filter classes and the Wave pipe (Sec. 3): lazy
sample-rate binding, stage collection, designs, errors.  Nothing here runs a
kernel."""
import numpy as np
import pytest
import torch
from torch.nn import Sequential

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import design


def _wave(C=2, N=64, fs=48000.0):
    return tfx.Wave(torch.zeros(C, N), fs)


def test_pipe_binds_the_sample_rate_lazily_and_records_stages():
    hs, ls = tfx.HiShelving(1000), tfx.LoShelving(2000)
    assert hs.sample_rate is None
    w = _wave() | hs | ls
    assert [type(f) for f in w.pending] == [tfx.HiShelving, tfx.LoShelving]
    assert hs.sample_rate == 48000.0 and ls.sample_rate == 48000.0
    assert w.fs == 48000.0 and w.channels == 2 and len(w) == 64


def test_sequential_is_flattened_into_the_pipe():
    chain = Sequential(tfx.HiShelving(1000), Sequential(tfx.Peaking(3000), tfx.LoShelving(2000)))
    w = _wave() | chain
    assert [type(f) for f in w.pending] == [tfx.HiShelving, tfx.Peaking, tfx.LoShelving]


def test_designs_match_the_fp64_design_functions():
    fs = 44100.0
    cases = [
        (tfx.Butterworth(150.0, fs, order=5, btype="highpass"), design.butterworth(5, 150.0, fs, "highpass")),
        (tfx.Chebyshev1(8000.0, fs, order=8, ripple_db=1.0), design.chebyshev1(8, 1.0, 8000.0, fs)),
        (tfx.Peaking(1000.0, fs, q=2.0, gain_db=-4.0), design.peaking(1000.0, 2.0, -4.0, fs)),
        (tfx.HiShelving(5000.0, fs, gain_db=3.0), design.shelf(5000.0, 3.0, fs, "high")),
        (tfx.LoShelving(200.0, fs, gain_db=-6.0, slope=0.8), design.shelf(200.0, -6.0, fs, "low", 0.8)),
        (tfx.WindowedSincFIR(6000.0, fs, num_taps=65), design.fir_lowpass(65, 6000.0, fs)),
        (tfx.WindowedSincFIR(300.0, fs, num_taps=129, cutoff_hi=3000.0), design.fir_bandpass(129, 300.0, 3000.0, fs)),
        (tfx.Chebyshev2(3000.0, fs, order=6, atten_db=50.0), design.chebyshev2(6, 50.0, 3000.0, fs)),
        (tfx.ButterworthBand(200.0, 4000.0, fs, order=3, btype="bandstop"),
         design.butterworth_band(3, 200.0, 4000.0, fs, "bandstop")),
        (tfx.Notch(60.0, fs, q=30.0), design.notch(60.0, 30.0, fs)),
        (tfx.AllPass(700.0, fs, q=0.5), design.allpass(700.0, 0.5, fs)),
        (tfx.BandPass(2500.0, fs, q=4.0), design.bandpass_biquad(2500.0, 4.0, fs)),
    ]
    for f, ref in cases:
        c = f.coefficients("cpu").numpy()
        np.testing.assert_array_equal(c, np.asarray(ref, np.float64).astype(np.float32))
        assert f.kind == ("fir" if isinstance(f, tfx.WindowedSincFIR) else "sos")


def test_a_filter_built_for_another_rate_is_rejected():
    with pytest.raises(ValueError, match="44100"):
        _wave(fs=48000.0) | tfx.HiShelving(1000, 44100)


def test_a_filter_without_a_sample_rate_cannot_design():
    with pytest.raises(ValueError, match="sample rate"):
        tfx.Peaking(1000).coefficients("cpu")


def test_explicit_coefficients_need_no_rate_and_can_be_trainable():
    f = tfx.FIR(np.ones(8) / 8, learnable=True)
    s = tfx.SOS([[1.0, 0.0, 0.0, -0.5, 0.0]])
    assert isinstance(f.taps, torch.nn.Parameter) and not isinstance(s.sections, torch.nn.Parameter)
    w = _wave() | f | s
    assert len(w.pending) == 2 and f.sample_rate is None
    assert [n for n, _ in f.named_parameters()] == ["taps"]


def test_other_modules_apply_at_once():
    w = tfx.Wave(torch.ones(1, 10), 8000.0) | (lambda y: 2.0 * y)
    assert not w.pending and torch.equal(w.y, 2.0 * torch.ones(1, 10))


def test_wave_shapes():
    assert tfx.Wave(torch.zeros(100), 16000).channels == 1
    assert tfx.Wave(np.zeros((3, 5), np.float32), 16000).duration == 5 / 16000
    with pytest.raises(ValueError):
        tfx.Wave(torch.zeros(1, 2, 3), 16000)
    with pytest.raises(ValueError):
        tfx.Wave(torch.zeros(1, 3), 0)


def test_direct_form_factors_once_and_rejects_unstable_denominators():
    b, a = [0.2, 0.3, 0.1, 0.05], [1.0, -0.9, 0.4, -0.1]
    f = tfx.DirectForm(b, a)
    np.testing.assert_array_equal(f.coefficients("cpu").numpy(), design.tf2sos(b, a).astype(np.float32))
    assert f.kind == "sos" and (_wave() | f).pending == [f]
    with pytest.raises(ValueError, match="unit circle"):
        tfx.DirectForm([1.0], [1.0, -1.5])
    with pytest.raises(ValueError, match="unit circle"):
        tfx.lfilter(torch.zeros(1, 8), [1.0], [1.0, 0.0, 1.0])   # poles on the circle
    with pytest.raises(ValueError, match="nonzero"):
        tfx.lfilter(torch.zeros(1, 8), [1.0], [0.0])


def test_differentiable_chain_rejects_low_precision_fir():
    # the adjoint is fp32 only: refused when the forward is asked for, before
    # any device work (a CPU tensor would otherwise be rejected later)
    x = torch.zeros(2, 16, requires_grad=True)
    with pytest.raises(ValueError, match="fp32 only"):
        tfx.chain(x, [("fir", torch.ones(5))], compute="bf16")

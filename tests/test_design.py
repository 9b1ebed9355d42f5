"""Pins of the FP64 coefficient design (host-side input preparation)."""
import numpy as np
import pytest
import scipy.signal as ss

from paper_2504_08624_amd import design as D


def _H(sos5, f, fs):
    z1 = np.exp(-2j * np.pi * np.asarray(f, dtype=np.float64) / fs)
    H = np.ones_like(z1)
    for b0, b1, b2, a1, a2 in np.asarray(sos5).reshape(-1, 5):
        H *= (b0 + b1 * z1 + b2 * z1 ** 2) / (1 + a1 * z1 + a2 * z1 ** 2)
    return H


def _db(v):
    return 20 * np.log10(np.abs(v))


@pytest.mark.parametrize("order,fc", [(2, 1000.0), (4, 100.0), (5, 3000.0)])
def test_butterworth_lowpass(order, fc):
    fs = 48000.0
    sos = D.butterworth(order, fc, fs, "lowpass")
    assert abs(_db(_H(sos, fc, fs)) + 10 * np.log10(2)) < 1e-9
    assert abs(abs(_H(sos, 0.0, fs)) - 1) < 1e-12
    assert abs(_H(sos, fs / 2, fs)) < 1e-9


def test_butterworth_highpass_zeros_at_dc():
    fs = 48000.0
    sos = D.butterworth(4, 100.0, fs, "highpass")
    assert sos.shape == (2, 5)
    for b0, b1, b2, _, _ in sos:          # each numerator is b0 (1 - z^-1)^2
        assert np.allclose([b1 / b0, b2 / b0], [-2, 1], atol=1e-12)
    assert abs(_db(_H(sos, 100.0, fs)) + 10 * np.log10(2)) < 1e-9
    assert abs(abs(_H(sos, fs / 2, fs)) - 1) < 1e-12
    radii = [max(abs(np.roots([1, r[3], r[4]]))) for r in sos]
    assert radii == sorted(radii)


def test_chebyshev1_even_order_ripple_points():
    fs = 48000.0
    sos = D.chebyshev1(8, 1.0, 12000.0, fs)
    assert sos.shape == (4, 5)
    assert abs(_db(_H(sos, 0.0, fs)) + 1.0) < 1e-9
    assert abs(_db(_H(sos, 12000.0, fs)) + 1.0) < 1e-9
    f = np.linspace(0, 12000, 2000)
    assert np.max(_db(_H(sos, f, fs))) < 1e-9 and np.min(_db(_H(sos, f, fs))) > -1.0 - 1e-9


@pytest.mark.parametrize("f0,q,g", [(250.0, 0.7, 6.0), (3000.0, 8.0, -12.0)])
def test_peaking_gain_points(f0, q, g):
    fs = 48000.0
    sos = D.peaking(f0, q, g, fs)
    assert abs(_H(sos, 0.0, fs) - 1) < 1e-12 and abs(_H(sos, fs / 2, fs) - 1) < 1e-12
    assert abs(_db(_H(sos, f0, fs)) - g) < 1e-9


def test_shelves():
    fs = 48000.0
    lo = D.shelf(200.0, 6.0, fs, "low")
    hi = D.shelf(5000.0, -4.0, fs, "high")
    assert abs(_db(_H(lo, 0.0, fs)) - 6.0) < 1e-9 and abs(_H(lo, fs / 2, fs) - 1) < 1e-9
    assert abs(_db(_H(hi, fs / 2, fs)) + 4.0) < 1e-9 and abs(_H(hi, 0.0, fs) - 1) < 1e-9


def test_windowed_sinc_lowpass():
    h = D.fir_lowpass(101, 8000.0, 48000.0)
    assert abs(h.sum() - 1) < 1e-14
    assert np.array_equal(h, h[::-1])
    raw = D._ideal_lp(101, 8000.0, 48000.0)
    assert abs(raw[50] - 2 * 8000.0 / 48000.0) < 1e-15
    assert np.allclose(h, ss.firwin(101, 8000.0, fs=48000.0, window="hamming"), atol=1e-15)


def test_windowed_sinc_bandpass_unit_centre_gain():
    fs = 48000.0
    h = D.fir_bandpass(1023, 200.0, 6000.0, fs)
    f0 = np.sqrt(200.0 * 6000.0)
    H0 = np.sum(h * np.exp(-2j * np.pi * f0 / fs * np.arange(h.size)))
    assert abs(abs(H0) - 1) < 1e-12
    assert np.allclose(h, h[::-1], atol=0)


@pytest.mark.parametrize("kind,args", [("butter", (4, 100.0, "highpass")),
                                       ("butter", (6, 2000.0, "lowpass")),
                                       ("cheby", (8, 1.0, 12000.0, "lowpass"))])
def test_design_matches_scipy(kind, args):
    fs = 48000.0
    if kind == "butter":
        mine = D.butterworth(args[0], args[1], fs, args[2])
        ref = ss.butter(args[0], args[1], args[2], fs=fs, output="sos")
    else:
        mine = D.chebyshev1(args[0], args[1], args[2], fs, args[3])
        ref = ss.cheby1(args[0], args[1], args[2], args[3], fs=fs, output="sos")
    f = np.linspace(1.0, fs / 2 - 1, 777)
    _, Hr = ss.sosfreqz(ref, worN=f, fs=fs)
    assert np.max(np.abs(_H(mine, f, fs) - Hr)) < 1e-9


def test_random_sections_are_stable_and_normalised():
    g = np.random.default_rng(7)
    sec = D.random_sections(g, 6, 0.5, 0.999)
    assert sec.shape == (6, 5)
    assert D.max_pole_radius(sec) < 0.999

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


# ---------------------------------------------- further families, direct form

def _resp_scipy(ref_sos, f, fs):
    _, H = ss.sosfreqz(ref_sos, worN=f, fs=fs)
    return H


@pytest.mark.parametrize("order,atten,fc,btype", [(4, 40.0, 2000.0, "lowpass"), (5, 60.0, 300.0, "highpass"),
                                                  (8, 50.0, 8000.0, "lowpass"), (3, 30.0, 12000.0, "highpass")])
def test_chebyshev2_matches_scipy_and_its_stopband(order, atten, fc, btype):
    fs = 48000.0
    mine = D.chebyshev2(order, atten, fc, fs, btype)
    f = np.linspace(1.0, fs / 2 - 1, 901)
    ref = ss.cheby2(order, atten, fc, btype, fs=fs, output="sos")
    assert np.max(np.abs(_H(mine, f, fs) - _resp_scipy(ref, f, fs))) < 1e-9
    # the stopband edge sits exactly atten dB down, and no stopband point is higher
    assert abs(_db(_H(mine, fc, fs)) + atten) < 1e-8
    stop = f[f > fc * 1.0001] if btype == "lowpass" else f[f < fc * 0.9999]
    assert np.max(_db(_H(mine, stop, fs))) < -atten + 1e-8
    assert D.max_pole_radius(mine) < 1.0


@pytest.mark.parametrize("order,f1,f2,btype", [(2, 300.0, 3000.0, "bandpass"), (3, 500.0, 1500.0, "bandstop"),
                                               (4, 100.0, 12000.0, "bandpass"), (1, 1000.0, 2000.0, "bandstop")])
def test_butterworth_band_matches_scipy_and_its_edges(order, f1, f2, btype):
    fs = 48000.0
    mine = D.butterworth_band(order, f1, f2, fs, btype)
    assert mine.shape == (order, 5)
    f = np.linspace(1.0, fs / 2 - 1, 901)
    ref = ss.butter(order, [f1, f2], btype, fs=fs, output="sos")
    assert np.max(np.abs(_H(mine, f, fs) - _resp_scipy(ref, f, fs))) < 1e-9
    # both band edges are 3 dB points
    for fe in (f1, f2):
        assert abs(_db(_H(mine, fe, fs)) + 10 * np.log10(2)) < 1e-8


def test_rbj_notch_bandpass_allpass_identities():
    fs, f0, q = 48000.0, 1234.0, 3.0
    n, bp, ap = D.notch(f0, q, fs), D.bandpass_biquad(f0, q, fs), D.allpass(f0, q, fs)
    f = np.linspace(0.0, fs / 2, 513)
    Hn, Hb, Ha = _H(n, f, fs), _H(bp, f, fs), _H(ap, f, fs)
    # same denominator: notch + band-pass is the identity, notch - band-pass the all-pass
    assert np.max(np.abs(Hn + Hb - 1)) < 1e-12
    assert np.max(np.abs(Hn - Hb - Ha)) < 1e-12
    assert np.max(np.abs(np.abs(Ha) - 1)) < 1e-12
    assert abs(_H(n, f0, fs)) < 1e-12 and abs(_H(bp, f0, fs) - 1) < 1e-12
    assert abs(_H(ap, f0, fs) + 1) < 1e-12
    assert abs(abs(_H(n, 0.0, fs)) - 1) < 1e-12 and abs(_H(bp, 0.0, fs)) < 1e-12


def _poly_from_roots(g, n_pairs, n_real, rmax):
    roots = []
    for _ in range(n_pairs):
        r, t = rmax * np.sqrt(g.uniform(0.05, 1.0)), g.uniform(0.05, np.pi - 0.05)
        roots += [r * np.exp(1j * t), r * np.exp(-1j * t)]
    roots += list(g.uniform(-rmax, rmax, n_real))
    return np.real(np.poly(roots)) if roots else np.ones(1)


@pytest.mark.parametrize("seed,zp,zr,pp,pr,delay", [(1, 2, 1, 3, 0, 0), (2, 0, 0, 2, 1, 0), (3, 3, 2, 1, 1, 1),
                                                    (4, 1, 0, 0, 2, 2), (5, 4, 0, 4, 0, 3), (6, 0, 1, 0, 0, 0)])
def test_tf2sos_keeps_the_transfer_function(seed, zp, zr, pp, pr, delay):
    g = np.random.default_rng(seed)
    b = np.concatenate([np.zeros(delay), 0.7 * _poly_from_roots(g, zp, zr, 1.3)])
    a = 2.0 * _poly_from_roots(g, pp, pr, 0.95)
    rows = D.tf2sos(b, a)
    f = np.linspace(0.0, 0.5, 777)
    _, Href = ss.freqz(b, a, worN=2 * np.pi * f)
    assert np.max(np.abs(_H(rows, f, 1.0) - Href)) < 1e-9 * max(1.0, np.max(np.abs(Href)))
    # the time-domain run agrees with the direct form too
    x = g.standard_normal(400)
    y = x.copy()
    for b0, b1, b2, a1, a2 in rows:
        y = ss.lfilter([b0, b1, b2], [1.0, a1, a2], y)
    assert np.max(np.abs(y - ss.lfilter(b, a, x))) < 1e-9 * max(1.0, np.max(np.abs(y)))
    assert D.max_pole_radius(rows) < 0.95 + 1e-9


def test_tf2sos_pairs_each_pole_pair_with_its_nearest_zeros():
    # two resonances, each with a zero pair just beside it: pairing keeps them together
    p1, p2 = 0.9 * np.exp(0.5j), 0.8 * np.exp(2.0j)
    z1, z2 = 0.95 * np.exp(0.55j), 0.9 * np.exp(2.1j)
    b = np.real(np.poly([z1, np.conj(z1), z2, np.conj(z2)]))
    a = np.real(np.poly([p1, np.conj(p1), p2, np.conj(p2)]))
    rows = D.tf2sos(b, a)
    assert rows.shape == (2, 5)
    for row, (p, z) in zip(rows, [(p2, z2), (p1, z1)]):   # increasing pole radius
        assert np.allclose(sorted(np.abs(np.roots([1.0, row[3], row[4]]))), [abs(p)] * 2)
        assert np.allclose(np.abs(np.roots(row[:3])), [abs(z)] * 2)


def test_tf2sos_degenerate_forms():
    assert np.allclose(D.tf2sos([2.0], [4.0]), [[0.5, 0, 0, 0, 0]])
    assert np.allclose(D.tf2sos([0.0, 0.0, 3.0], [1.0]), [[3.0, 0, 0, 0, 0], [0, 0, 1.0, 0, 0]])
    assert np.allclose(D.tf2sos([0.0], [1.0, 0.5]), 0.0)
    with pytest.raises(ValueError):
        D.tf2sos([1.0], [0.0, 1.0])

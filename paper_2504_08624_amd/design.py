"""FP64 coefficient design on the host.

The paper's library offers one class per filter type (Butterworth, Chebyshev,
peaking, shelving, windowed FIR; Sec. 3) and computes coefficients outside the
timed region (Sec. 4).  The recipes below are the textbook ones, computed in
float64 and cast to fp32 only at the end:

* windowed-sinc FIR (symmetric Hamming window) low-pass / band-pass;
* Butterworth and Chebyshev type I low/high-pass: analog prototype poles,
  bilinear transform prewarped at the edge frequency, conjugate pole pairs
  grouped into second-order sections ordered by increasing pole radius, the
  overall gain placed on the first section;
* RBJ audio-EQ-cookbook peaking and shelving biquads;
* random stable sections and the pole/zero -> section map used by the
  learnable cascade.

Every section is returned as a row [b0, b1, b2, a1, a2] with a0 normalised to
1 in float64.  No filtering is done here.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------- FIR design


def hamming(M: int) -> np.ndarray:
    """Symmetric Hamming window 0.54 - 0.46 cos(2 pi n / (M - 1))."""
    if M == 1:
        return np.ones(1)
    n = np.arange(M, dtype=np.float64)
    return 0.54 - 0.46 * np.cos(2.0 * np.pi * n / (M - 1))


def _ideal_lp(M: int, fc: float, fs: float) -> np.ndarray:
    n = np.arange(M, dtype=np.float64) - (M - 1) / 2.0
    wc = 2.0 * fc / fs
    return wc * np.sinc(wc * n)


def fir_lowpass(M: int, fc: float, fs: float) -> np.ndarray:
    """Hamming windowed-sinc low-pass, scaled to unit DC gain (sum h = 1)."""
    h = _ideal_lp(M, fc, fs) * hamming(M)
    h = 0.5 * (h + h[::-1])                 # exactly symmetric (linear phase)
    return h / h.sum()


def fir_bandpass(M: int, f1: float, f2: float, fs: float) -> np.ndarray:
    """Hamming windowed-sinc band-pass [f1, f2], unit gain at sqrt(f1 f2)."""
    h = (_ideal_lp(M, f2, fs) - _ideal_lp(M, f1, fs)) * hamming(M)
    h = 0.5 * (h + h[::-1])
    f0 = np.sqrt(f1 * f2)
    g = abs(np.sum(h * np.exp(-2j * np.pi * f0 / fs * np.arange(M))))
    return h / g


# --------------------------------------------------------------- IIR design


def _bilinear_zpk(z_s, p_s, fs):
    """Map analog poles/zeros to the z-plane: z = (2fs + s) / (2fs - s)."""
    c = 2.0 * fs
    p = (c + np.asarray(p_s)) / (c - np.asarray(p_s))
    z = (c + np.asarray(z_s)) / (c - np.asarray(z_s)) if len(z_s) else np.zeros(0)
    return z, p


def _pair_sections(zeros, poles):
    """Group conjugate pole pairs (and any real pole) into sections, ordered
    by increasing pole radius; zeros are handed out in the same groups
    (all zeros here sit at z = +1 or z = -1, so the pairing is trivial)."""
    poles = np.asarray(poles, dtype=np.complex128)
    zeros = list(np.asarray(zeros, dtype=np.complex128))
    upper = [p for p in poles if p.imag > 1e-12]
    real = [p.real for p in poles if abs(p.imag) <= 1e-12]
    groups = [(abs(p), "c", p) for p in upper] + [(abs(r), "r", r) for r in real]
    # two real poles share a section when there are several
    groups.sort(key=lambda g: g[0])
    rows = []
    reals = [g for g in groups if g[1] == "r"]
    cplx = [g for g in groups if g[1] == "c"]
    items = []
    for g in cplx:
        items.append((g[0], [g[2], np.conj(g[2])]))
    while len(reals) >= 2:
        a, b = reals.pop(0), reals.pop(0)
        items.append((max(a[0], b[0]), [a[2], b[2]]))
    if reals:
        items.append((reals[0][0], [reals[0][2]]))
    items.sort(key=lambda it: it[0])
    for _, ps in items:
        npl = len(ps)
        zs = [zeros.pop(0) for _ in range(min(npl, len(zeros)))]
        a = np.real(np.poly(ps))
        b = np.real(np.poly(zs)) if zs else np.ones(1)
        a = np.concatenate([a, np.zeros(3 - a.size)])
        b = np.concatenate([b, np.zeros(3 - b.size)])
        rows.append(np.concatenate([b, a]))
    return np.array(rows)  # [S, 6]: b0 b1 b2 a0 a1 a2


def _normalise(rows6: np.ndarray) -> np.ndarray:
    rows6 = np.asarray(rows6, dtype=np.float64).reshape(-1, 6)
    a0 = rows6[:, 3:4]
    return np.concatenate([rows6[:, 0:3] / a0, rows6[:, 4:6] / a0], axis=1)


def sos_response(sos5: np.ndarray, w) -> np.ndarray:
    """Complex response of a cascade at normalised angular frequencies w
    (used only to place the overall gain during design)."""
    z1 = np.exp(-1j * np.asarray(w, dtype=np.float64))
    H = np.ones_like(z1)
    for b0, b1, b2, a1, a2 in np.asarray(sos5).reshape(-1, 5):
        H = H * (b0 + b1 * z1 + b2 * z1 * z1) / (1.0 + a1 * z1 + a2 * z1 * z1)
    return H


def _finish(z, p, gain_w, gain_target):
    rows = _normalise(_pair_sections(z, p))
    g = abs(sos_response(rows, [gain_w])[0])
    rows[0, 0:3] *= gain_target / g
    return rows


def butterworth(order: int, fc: float, fs: float, btype: str = "lowpass") -> np.ndarray:
    """Butterworth low/high-pass as [S, 5] sections (bilinear, prewarped)."""
    k = np.arange(order)
    proto = np.exp(1j * np.pi * (2 * k + order + 1) / (2.0 * order))
    wc = 2.0 * fs * np.tan(np.pi * fc / fs)
    if btype == "lowpass":
        _, p = _bilinear_zpk([], wc * proto, fs)
        return _finish(-np.ones(order), p, 0.0, 1.0)
    if btype == "highpass":
        _, p = _bilinear_zpk([], wc / proto, fs)
        return _finish(np.ones(order), p, np.pi, 1.0)
    raise ValueError(btype)


def chebyshev1(order: int, ripple_db: float, fc: float, fs: float,
               btype: str = "lowpass") -> np.ndarray:
    """Chebyshev type I (passband ripple ``ripple_db``, edge ``fc`` where the
    gain is -ripple_db) as [S, 5] sections."""
    eps = np.sqrt(10.0 ** (ripple_db / 10.0) - 1.0)
    mu = np.arcsinh(1.0 / eps) / order
    th = np.pi * (2 * np.arange(order) + 1) / (2.0 * order)
    proto = -np.sinh(mu) * np.sin(th) + 1j * np.cosh(mu) * np.cos(th)
    wc = 2.0 * fs * np.tan(np.pi * fc / fs)
    g_pass = 1.0 if order % 2 else 1.0 / np.sqrt(1.0 + eps * eps)
    if btype == "lowpass":
        _, p = _bilinear_zpk([], wc * proto, fs)
        return _finish(-np.ones(order), p, 0.0, g_pass)
    if btype == "highpass":
        _, p = _bilinear_zpk([], wc / proto, fs)
        return _finish(np.ones(order), p, np.pi, g_pass)
    raise ValueError(btype)


def peaking(f0: float, q: float, gain_db: float, fs: float) -> np.ndarray:
    """RBJ cookbook peaking EQ, one [1, 5] section."""
    A = 10.0 ** (gain_db / 40.0)
    w0 = 2.0 * np.pi * f0 / fs
    al = np.sin(w0) / (2.0 * q)
    c = np.cos(w0)
    return _normalise([[1 + al * A, -2 * c, 1 - al * A, 1 + al / A, -2 * c, 1 - al / A]])


def shelf(f0: float, gain_db: float, fs: float, kind: str, slope: float = 1.0) -> np.ndarray:
    """RBJ cookbook low/high shelf, one [1, 5] section."""
    A = 10.0 ** (gain_db / 40.0)
    w0 = 2.0 * np.pi * f0 / fs
    c, s = np.cos(w0), np.sin(w0)
    al = s / 2.0 * np.sqrt((A + 1.0 / A) * (1.0 / slope - 1.0) + 2.0)
    r = 2.0 * np.sqrt(A) * al
    if kind == "low":
        row = [A * ((A + 1) - (A - 1) * c + r), 2 * A * ((A - 1) - (A + 1) * c),
               A * ((A + 1) - (A - 1) * c - r), (A + 1) + (A - 1) * c + r,
               -2 * ((A - 1) + (A + 1) * c), (A + 1) + (A - 1) * c - r]
    elif kind == "high":
        row = [A * ((A + 1) + (A - 1) * c + r), -2 * A * ((A - 1) + (A + 1) * c),
               A * ((A + 1) + (A - 1) * c - r), (A + 1) - (A - 1) * c + r,
               2 * ((A - 1) - (A + 1) * c), (A + 1) - (A - 1) * c - r]
    else:
        raise ValueError(kind)
    return _normalise([row])


def from_polar(r_p, th_p, r_z, th_z, k) -> np.ndarray:
    """Sections from pole/zero polar coordinates: b = k [1, -2 rz cos tz, rz^2],
    a = [1, -2 rp cos tp, rp^2]."""
    r_p, th_p, r_z, th_z, k = (np.asarray(v, dtype=np.float64) for v in (r_p, th_p, r_z, th_z, k))
    return np.stack([k, -2 * k * r_z * np.cos(th_z), k * r_z * r_z,
                     -2 * r_p * np.cos(th_p), r_p * r_p], axis=-1)


def random_sections(rng: np.random.Generator, S: int, r_lo: float = 0.5,
                    r_hi: float = 0.999) -> np.ndarray:
    """Random stable resonators: poles r e^{+-j theta} with r ~ U(r_lo, r_hi),
    theta ~ U(0, pi); zeros on the unit circle at angle phi ~ U(0, pi); each
    section scaled to unit gain at its pole angle."""
    r = rng.uniform(r_lo, r_hi, S)
    th = rng.uniform(0.0, np.pi, S)
    ph = rng.uniform(0.0, np.pi, S)
    rows = from_polar(r, th, np.ones(S), ph, np.ones(S))
    for i in range(S):
        g = abs(sos_response(rows[i:i + 1], [th[i]])[0])
        rows[i, 0:3] /= g
    return rows


def max_pole_radius(sos5: np.ndarray) -> float:
    """Largest pole magnitude of a cascade (1 + a1 z^-1 + a2 z^-2 per row)."""
    rmax = 0.0
    for row in np.asarray(sos5, dtype=np.float64).reshape(-1, 5):
        rts = np.roots([1.0, row[3], row[4]])
        if rts.size:
            rmax = max(rmax, float(np.max(np.abs(rts))))
    return rmax


# ------------------------------------------- further families, direct form

def _groups(roots, tol=1e-9):
    """Split roots into conjugate pairs (upper-half member) and reals."""
    r = np.asarray(roots, dtype=np.complex128)
    upper = [v for v in r if v.imag > tol]
    reals = sorted([v.real for v in r if abs(v.imag) <= tol])
    return upper, reals


def _pair_general(zeros, poles, k):
    """Sections of H(z) = k prod(1 - z_i/z) / prod(1 - p_j/z), any zeros.
    Pole groups (a conjugate pair, or two real poles) are taken from the one
    closest to the unit circle; each gets the nearest remaining zero group
    (a conjugate pair, or up to two reals).  Sections are returned by
    increasing pole radius, the gain k on the first one.  Groups without
    poles (more zeros than poles) become FIR sections."""
    pu, pr = _groups(poles)
    zu, zr = _groups(zeros)
    pg = [[p, np.conj(p)] for p in pu]
    while len(pr) >= 2:
        pg.append([pr.pop(0), pr.pop(0)])
    if pr:
        pg.append([pr.pop(0)])
    zg = [[z, np.conj(z)] for z in zu]
    while len(zr) >= 2:
        zg.append([zr.pop(0), zr.pop(0)])
    if zr:
        zg.append([zr.pop(0)])
    pg.sort(key=lambda g: -max(abs(v) for v in g))
    secs = []
    for g in pg:
        c = np.mean(g)
        if zg:
            j = min(range(len(zg)), key=lambda i: abs(np.mean(zg[i]) - c))
            secs.append((g, zg.pop(j)))
        else:
            secs.append((g, []))
    secs.extend(([], zgrp) for zgrp in zg)
    secs.sort(key=lambda s: max((abs(v) for v in s[0]), default=0.0))
    rows = []
    for ps, zs in secs:
        a = np.real(np.poly(ps)) if ps else np.ones(1)
        b = np.real(np.poly(zs)) if zs else np.ones(1)
        rows.append(np.concatenate([b, np.zeros(3 - b.size), a[1:], np.zeros(3 - a.size)]))
    if not rows:
        rows = [np.array([1.0, 0.0, 0.0, 0.0, 0.0])]
    rows = np.asarray(rows, dtype=np.float64)
    rows[0, 0:3] *= k
    return rows


def tf2sos(b, a) -> np.ndarray:
    """Direct-form transfer function b(z^-1) / a(z^-1) (any orders, a[0] != 0)
    as [S, 5] sections with the same response.  Leading zero coefficients of
    b are pure delays (sections z^-1 or z^-2)."""
    b = np.trim_zeros(np.atleast_1d(np.asarray(b, dtype=np.float64)), "b")
    a = np.trim_zeros(np.atleast_1d(np.asarray(a, dtype=np.float64)), "b")
    if a.size == 0 or a[0] == 0.0:
        raise ValueError("a[0] must be nonzero")
    if b.size == 0:
        return np.array([[0.0, 0.0, 0.0, 0.0, 0.0]])
    d = 0
    while b[d] == 0.0:
        d += 1
    bb = b[d:]
    rows = _pair_general(np.roots(bb), np.roots(a), bb[0] / a[0])
    delays = []
    while d >= 2:
        delays.append([0.0, 0.0, 1.0, 0.0, 0.0])
        d -= 2
    if d:
        delays.append([0.0, 1.0, 0.0, 0.0, 0.0])
    return np.concatenate([rows, np.asarray(delays).reshape(-1, 5)]) if delays else rows


def chebyshev2(order: int, atten_db: float, fc: float, fs: float, btype: str = "lowpass") -> np.ndarray:
    """Chebyshev type II (stopband attenuation ``atten_db``, stopband edge
    ``fc``) low/high-pass as [S, 5] sections (bilinear, prewarped)."""
    eps = 1.0 / np.sqrt(10.0 ** (atten_db / 10.0) - 1.0)
    mu = np.arcsinh(1.0 / eps) / order
    th = np.pi * (2 * np.arange(order) + 1) / (2.0 * order)
    p1 = -np.sinh(mu) * np.sin(th) + 1j * np.cosh(mu) * np.cos(th)
    proto_p = 1.0 / p1
    cz = np.cos(th)
    proto_z = np.array([1j / c for c in cz if abs(c) > 1e-12])
    wc = 2.0 * fs * np.tan(np.pi * fc / fs)
    nz_inf = order - proto_z.size
    if btype == "lowpass":
        z, p = _bilinear_zpk(wc * proto_z, wc * proto_p, fs)
        z = np.concatenate([z, -np.ones(nz_inf)])
        gain_w, target = 0.0, 1.0
    elif btype == "highpass":
        z, p = _bilinear_zpk(wc / proto_z, wc / proto_p, fs)
        z = np.concatenate([z, np.ones(nz_inf)])
        gain_w, target = np.pi, 1.0
    else:
        raise ValueError(btype)
    rows = _pair_general(z, p, 1.0)
    rows[0, 0:3] *= target / abs(sos_response(rows, [gain_w])[0])
    return rows


def butterworth_band(order: int, f1: float, f2: float, fs: float, btype: str = "bandpass") -> np.ndarray:
    """Butterworth band-pass / band-stop between ``f1`` and ``f2`` of
    prototype order ``order`` (2 order poles): the low-pass prototype through
    the analog band transformation, then the bilinear map (edges prewarped)."""
    k = np.arange(order)
    proto = np.exp(1j * np.pi * (2 * k + order + 1) / (2.0 * order))
    w1, w2 = (2.0 * fs * np.tan(np.pi * f / fs) for f in (f1, f2))
    w0, bw = np.sqrt(w1 * w2), w2 - w1
    if btype == "bandpass":
        t = proto * bw / 2.0
        ps = np.concatenate([t + np.sqrt(t * t - w0 * w0), t - np.sqrt(t * t - w0 * w0)])
        _, p = _bilinear_zpk([], ps, fs)
        z = np.concatenate([np.ones(order), -np.ones(order)])  # s = 0 and s = infinity
        gain_w = 2.0 * np.arctan(w0 / (2.0 * fs))
    elif btype == "bandstop":
        t = bw / (2.0 * proto)
        ps = np.concatenate([t + np.sqrt(t * t - w0 * w0), t - np.sqrt(t * t - w0 * w0)])
        _, p = _bilinear_zpk([], ps, fs)
        zc = (2.0 * fs + 1j * w0) / (2.0 * fs - 1j * w0)
        z = np.concatenate([np.full(order, zc), np.full(order, np.conj(zc))])
        gain_w = 0.0
    else:
        raise ValueError(btype)
    rows = _pair_general(z, p, 1.0)
    rows[0, 0:3] *= 1.0 / abs(sos_response(rows, [gain_w])[0])
    return rows


def _rbj(f0: float, q: float, fs: float):
    w0 = 2.0 * np.pi * f0 / fs
    return np.cos(w0), np.sin(w0) / (2.0 * q)


def notch(f0: float, q: float, fs: float) -> np.ndarray:
    """RBJ cookbook notch at ``f0`` (one section; unit gain far from f0)."""
    c, al = _rbj(f0, q, fs)
    return _normalise([[1.0, -2 * c, 1.0, 1 + al, -2 * c, 1 - al]])


def allpass(f0: float, q: float, fs: float) -> np.ndarray:
    """RBJ cookbook second-order all-pass centred at ``f0`` (one section)."""
    c, al = _rbj(f0, q, fs)
    return _normalise([[1 - al, -2 * c, 1 + al, 1 + al, -2 * c, 1 - al]])


def bandpass_biquad(f0: float, q: float, fs: float) -> np.ndarray:
    """RBJ cookbook band-pass with 0 dB peak at ``f0`` (one section)."""
    c, al = _rbj(f0, q, fs)
    return _normalise([[al, 0.0, -al, 1 + al, -2 * c, 1 - al]])

"""Pins of the FP64 oracle against facts that do not come from the oracle.

The paper prints no numerical outputs, so every pin here is a closed form, a
library routine written by someone else (numpy.convolve, scipy.signal), an
invariant of linear time-invariant systems, or a finite-difference check of
the adjoint.  Each is chosen so that a plausible slip in the oracle (a dropped
term, a wrong sign, an off-by-one in the causal bound, a transposed operand in
a gradient) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.signal as ss

from oracle import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _sos6(sos5):
    sos5 = np.asarray(sos5, dtype=np.float64).reshape(-1, 5)
    return np.hstack([sos5[:, :3], np.ones((sos5.shape[0], 1)), sos5[:, 3:]])


def _H(sos5, w):
    """Cascade frequency response by direct polynomial evaluation."""
    z1 = np.exp(-1j * np.asarray(w))
    H = np.ones_like(z1)
    for b0, b1, b2, a1, a2 in np.asarray(sos5).reshape(-1, 5):
        H *= (b0 + b1 * z1 + b2 * z1 ** 2) / (1 + a1 * z1 + a2 * z1 ** 2)
    return H


RNG = np.random.default_rng(12345)


# ----------------------------------------------------------------------- FIR

@pytest.mark.parametrize("M", [1, 2, 7, 64, 101])
def test_fir_impulse_is_taps(M):
    h = RNG.standard_normal(M)
    N = M + 37
    x = np.zeros(N)
    x[0] = 1.0
    y = O.fir(x, h)
    assert np.array_equal(y[:M], h)
    assert np.all(y[M:] == 0.0)


def test_fir_shifted_impulse():
    h = RNG.standard_normal(13)
    x = np.zeros((2, 50))
    x[0, 5] = 1.0
    x[1, 40] = -2.0
    y = O.fir(x, h)
    assert np.array_equal(y[0, 5:18], h) and np.all(y[0, :5] == 0) and np.all(y[0, 18:] == 0)
    assert np.array_equal(y[1, 40:50], -2.0 * h[:10]) and np.all(y[1, :40] == 0)


def test_fir_single_tap_scales():
    x = RNG.standard_normal((3, 100))
    assert np.array_equal(O.fir(x, [0.75]), 0.75 * x)


@pytest.mark.parametrize("M,N", [(5, 3), (17, 17), (33, 1000), (300, 257)])
def test_fir_matches_numpy_convolve(M, N):
    h = RNG.standard_normal(M)
    x = RNG.standard_normal((2, N))
    y = O.fir(x, h)
    ref = np.stack([np.convolve(r, h)[:N] for r in x])
    assert _rel(y, ref) < 1e-13


def test_fir_at_matches_full():
    h = RNG.standard_normal(40)
    x = RNG.standard_normal((3, 500))
    pos = np.array([0, 1, 39, 40, 41, 250, 499])
    assert np.array_equal(O.fir_at(x, h, pos), O.fir(x, h)[:, pos])


def test_fir_linear_and_time_invariant():
    h = RNG.standard_normal(21)
    x1, x2 = RNG.standard_normal((2, 300))
    a, b = 0.3, -1.7
    assert _rel(O.fir(a * x1 + b * x2, h), a * O.fir(x1, h) + b * O.fir(x2, h)) < 1e-14
    d = 17
    xs = np.concatenate([np.zeros(d), x1])[:300]
    assert _rel(O.fir(xs, h)[d:], O.fir(x1, h)[:300 - d]) < 1e-15


# ----------------------------------------------------------------------- SOS

@pytest.mark.parametrize("p", [0.5, -0.9, 0.995])
def test_one_pole_impulse_is_power(p):
    N = 400
    x = np.zeros(N)
    x[0] = 1.0
    y = O.sos(x, [[1.0, 0.0, 0.0, -p, 0.0]])
    assert np.max(np.abs(y - p ** np.arange(N))) < 1e-14


@pytest.mark.parametrize("r,th", [(0.9, 0.3), (0.99, 2.0), (0.5, 1.2)])
def test_two_pole_impulse_closed_form(r, th):
    N = 600
    x = np.zeros(N)
    x[0] = 1.0
    y = O.sos(x, [[1.0, 0.0, 0.0, -2 * r * np.cos(th), r * r]])
    n = np.arange(N)
    ref = r ** n * np.sin((n + 1) * th) / np.sin(th)
    assert np.max(np.abs(y - ref)) < 1e-13


def test_section_without_poles_is_three_tap_fir():
    b = RNG.standard_normal(3)
    x = RNG.standard_normal((2, 200))
    y = O.sos(x, [[b[0], b[1], b[2], 0.0, 0.0]])
    ref = np.stack([np.convolve(r, b)[:200] for r in x])
    assert _rel(y, ref) < 1e-15


def test_identity_section_copies():
    x = RNG.standard_normal((2, 64))
    assert np.array_equal(O.sos(x, [[1, 0, 0, 0, 0]]), x)


def test_cascade_matches_scipy_sosfilt():
    sos = np.array([[0.2, 0.4, 0.2, -1.2, 0.5], [1.0, -2.0, 1.0, -1.9, 0.95],
                    [0.5, 0.1, -0.3, 0.3, 0.2]])
    x = RNG.standard_normal((3, 5000))
    assert _rel(O.sos(x, sos), ss.sosfilt(_sos6(sos), x)) < 1e-13


def test_cascade_equals_product_transfer_function():
    sos = np.array([[0.2, 0.4, 0.2, -1.2, 0.5], [1.0, -2.0, 1.0, -1.9, 0.95]])
    b = np.polymul(sos[0, :3], sos[1, :3])
    a = np.polymul([1, *sos[0, 3:]], [1, *sos[1, 3:]])
    x = np.zeros(3000)
    x[0] = 1.0
    assert _rel(O.sos(x, sos), ss.lfilter(b, a, x)) < 1e-12


@pytest.mark.parametrize("w", [0.0, np.pi, 0.05, 0.7, 2.3])
def test_steady_state_gain_matches_transfer_function(w):
    sos = np.array([[0.3, 0.1, 0.2, -0.9, 0.6], [1.0, 0.5, 0.25, 0.4, 0.3]])
    rmax = max(np.max(np.abs(np.roots([1, r[3], r[4]]))) for r in sos)
    N = int(60 / (1 - rmax)) + 200
    n = np.arange(N)
    yc = O.sos(np.cos(w * n), sos)
    ys = O.sos(np.sin(w * n), sos)
    H = (yc[-1] + 1j * ys[-1]) / np.exp(1j * w * (N - 1))
    assert abs(H - _H(sos, w)) < 1e-12 * max(1, abs(_H(sos, w)))


def test_dc_and_nyquist_gain_closed_form():
    sos = np.array([[0.3, 0.1, 0.2, -0.9, 0.6]])
    N = 2000
    dc = O.sos(np.ones(N), sos)[-1]
    assert abs(dc - sos[0, :3].sum() / (1 + sos[0, 3] + sos[0, 4])) < 1e-13
    ny = O.sos((-1.0) ** np.arange(N), sos)[-1] * (-1.0) ** (N - 1)
    assert abs(ny - (sos[0, 0] - sos[0, 1] + sos[0, 2]) / (1 - sos[0, 3] + sos[0, 4])) < 1e-13


def test_split_and_resume_equals_one_shot():
    sos = np.array([[0.2, 0.4, 0.2, -1.2, 0.5], [1.0, -2.0, 1.0, -1.9, 0.95]])
    x = RNG.standard_normal((2, 1000))
    full, st_full = O.sos(x, sos, return_state=True)
    k = 377
    y1, st = O.sos(x[:, :k], sos, return_state=True)
    y2, st2 = O.sos(x[:, k:], sos, state_in=st, return_state=True)
    assert np.array_equal(np.concatenate([y1, y2], axis=1), full)
    assert np.array_equal(st2, st_full)


def test_state_convention_is_tdf2_registers():
    # after a single sample x0 from zero state: s1 = (b1 - a1 b0) x0, s2 = (b2 - a2 b0) x0
    b0, b1, b2, a1, a2 = 0.7, -0.2, 0.4, 0.3, -0.1
    _, st = O.sos(np.array([[2.0]]), [[b0, b1, b2, a1, a2]], return_state=True)
    assert np.allclose(st[0, 0], [(b1 - a1 * b0) * 2.0, (b2 - a2 * b0) * 2.0], rtol=0, atol=1e-15)


def test_sos_linear_and_time_invariant():
    sos = np.array([[0.2, 0.4, 0.2, -1.2, 0.5]])
    x1, x2 = RNG.standard_normal((2, 500))
    assert _rel(O.sos(2 * x1 - x2, sos), 2 * O.sos(x1, sos) - O.sos(x2, sos)) < 1e-13
    d = 31
    xs = np.concatenate([np.zeros(d), x1])[:500]
    assert _rel(O.sos(xs, sos)[d:], O.sos(x1, sos)[:500 - d]) < 1e-15


def test_chain_commutes_and_is_in_order():
    h = RNG.standard_normal(15)
    sos = np.array([[0.2, 0.4, 0.2, -1.2, 0.5]])
    x = RNG.standard_normal((2, 700))
    a = O.chain(x, [("fir", h), ("sos", sos)])
    b = O.chain(x, [("sos", sos), ("fir", h)])
    assert _rel(a, b) < 1e-13
    assert np.array_equal(a, O.sos(O.fir(x, h), sos))


# ------------------------------------------------------------------ adjoint

def _dot(a, b):
    return float(np.sum(np.asarray(a) * np.asarray(b)))


def test_fir_adjoint_dot_product():
    h = RNG.standard_normal(23)
    x = RNG.standard_normal((2, 300))
    g = RNG.standard_normal((2, 300))
    gx, _ = O.fir_backward(g, x, h)
    assert abs(_dot(O.fir(x, h), g) - _dot(x, gx)) < 1e-12 * abs(_dot(x, gx)) + 1e-12


def test_sos_adjoint_dot_product():
    sos = np.array([[0.2, 0.4, 0.2, -1.2, 0.5], [1.0, -2.0, 1.0, -1.9, 0.95]])
    x = RNG.standard_normal((2, 400))
    g = RNG.standard_normal((2, 400))
    gx, _ = O.sos_backward(g, x, sos)
    assert abs(_dot(O.sos(x, sos), g) - _dot(x, gx)) < 1e-11 * abs(_dot(x, gx))


def _fd(f, theta, eps):
    grad = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        d = eps * max(1.0, abs(theta.flat[i]))
        tp.flat[i] += d
        tm.flat[i] -= d
        grad.flat[i] = (f(tp) - f(tm)) / (2 * d)
    return grad


def test_fir_tap_gradient_finite_difference():
    h = RNG.standard_normal(9)
    x = RNG.standard_normal((3, 120))
    g = RNG.standard_normal((3, 120))
    _, gh = O.fir_backward(g, x, h)
    fd = _fd(lambda t: _dot(O.fir(x, t), g), h, 1e-6)
    assert _rel(gh, fd) < 1e-8


def test_sos_coefficient_gradient_finite_difference():
    sos = np.array([[0.2, 0.4, 0.2, -1.2, 0.5], [1.0, -1.5, 0.7, -1.6, 0.8],
                    [0.3, 0.0, 0.1, 0.2, 0.1]])
    x = RNG.standard_normal((2, 256))
    g = RNG.standard_normal((2, 256))
    gx, gs = O.sos_backward(g, x, sos)
    fd = _fd(lambda t: _dot(O.sos(x, t), g), sos.copy(), 1e-6)
    assert _rel(gs, fd) < 1e-7
    fdx = _fd(lambda t: _dot(O.sos(t, sos), g), x.copy(), 1e-6)
    assert _rel(gx, fdx) < 1e-8


def test_one_pole_gradient_closed_form():
    p = 0.93
    N = 300
    x = np.zeros(N)
    x[0] = 1.0
    g = RNG.standard_normal(N)
    _, gs = O.sos_backward(g, x, [[1.0, 0.0, 0.0, -p, 0.0]])
    n = np.arange(N)
    d_dp = np.sum(n * p ** np.maximum(n - 1, 0) * g)
    assert abs(gs[0, 3] - (-d_dp)) < 1e-11 * abs(d_dp)
    assert abs(gs[0, 0] - np.sum(g * p ** n)) < 1e-12 * np.abs(g).sum()


def test_chain_backward_finite_difference():
    h = RNG.standard_normal(6)
    sos = np.array([[0.5, 0.2, 0.1, -0.8, 0.3]])
    stages = [("fir", h), ("sos", sos)]
    x = RNG.standard_normal((2, 100))
    g = RNG.standard_normal((2, 100))
    gx, (gh, gs) = O.chain_backward(g, x, stages)
    assert _rel(gh, _fd(lambda t: _dot(O.chain(x, [("fir", t), ("sos", sos)]), g), h.copy(), 1e-6)) < 1e-8
    assert _rel(gs, _fd(lambda t: _dot(O.chain(x, [("fir", h), ("sos", t)]), g), sos.copy(), 1e-6)) < 1e-8
    assert _rel(gx, _fd(lambda t: _dot(O.chain(t, stages), g), x.copy(), 1e-6)) < 1e-8

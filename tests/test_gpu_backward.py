"""GPU parity of the adjoint: libtfx's backward kernels (through the C ABI)
against the FP64 oracle's gradients (themselves pinned on the CPU by finite
differences, adjoint dot-products and a closed form).

Tolerances: relative error over the whole gradient (||a - b|| / ||b||),
1e-5 for the input gradient of an FP32 FIR, 1e-4 for everything that passes
through the IIR scan or a tap-gradient correlation (a sum over C*N products
computed tile by tile with fp32 FFTs).
"""
import numpy as np
import pytest
import torch

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import design, lib, signals, workloads
from oracle import oracle as O
from tests.metrics import TOL_FIR_F32, TOL_IIR_F32, assert_close, channel_errors

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
T = 3072
TOL_GRAD = 1e-4


def _x(C, N, key, sigma=0.1):
    return signals.to_f32(np.stack([signals.white(N, (*key, c), sigma) for c in range(C)]).reshape(C, N))


def _sections(S, key, r_lo=0.5, r_hi=0.99):
    return design.random_sections(signals.rng(*key), S, r_lo, r_hi).astype(np.float32)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


def assert_rel(a, b, tol, what):
    e = rel(a, b)
    assert np.isfinite(e) and e <= tol, "%s: rel err %.3e > %.1e" % (what, e, tol)
    return e


def report(what, err, bar, floor=None):
    """Prints a gradient's measured error beside its fixed bar (and the
    sequential fp32 adjoint's error on the same inputs, when computed)."""
    extra = "" if floor is None else ", sequential fp32 adjoint %.3e" % floor
    print("%s: GPU rel err %.3e (bar %.1e%s)" % (what, err, bar, extra), flush=True)


# ------------------------------------------------------------------- SOS

@pytest.mark.parametrize("S", [1, 3, 8])
@pytest.mark.parametrize("N", [1, 100, 3 * T + 17, 20000])
def test_sos_backward_parity(S, N):
    print("sos_backward S=%d N=%d" % (S, N), flush=True)
    C = 3
    x = _x(C, N, (301, S, N))
    g = _x(C, N, (302, S, N), 1.0)
    sec = _sections(S, (303, S))
    xg, secg = _gpu(x), _gpu(sec)
    _, ck = tfx.sos(xg, secg, return_ckpt=True)
    gx, gs = tfx.sos_backward(xg, _gpu(g), secg, ck)
    rgx, rgs = O.sos_backward(g, x, sec)
    assert_close(_cpu(gx), rgx, TOL_GRAD, "gx")
    assert_rel(_cpu(gs), rgs, TOL_GRAD, "gsos")


def _fp32_floor(g, x, sec):
    """Errors (gx, gsos) of a plain sequential fp32 adjoint against the FP64
    oracle: section signals by scipy's float32 lfilter, the adjoint signal
    v = (1/A) applied to g in reversed time, then the coefficient gradients as
    FP64 sums of those fp32 signals (sum v[n] x_s[n-i], -sum v[n] y_s[n-i]).
    This is the conditioning floor of the cascade in fp32."""
    import scipy.signal as ss
    S = sec.shape[0]
    sig = [x.astype(np.float32)]
    for s in range(S):
        a = np.array([1.0, sec[s, 3], sec[s, 4]], np.float32)
        sig.append(ss.lfilter(sec[s, :3].astype(np.float32), a, sig[-1], axis=1).astype(np.float32))
    gcur = g.astype(np.float32)
    gs = np.zeros((S, 5))
    for s in range(S - 1, -1, -1):
        a = np.array([1.0, sec[s, 3], sec[s, 4]], np.float32)
        v = ss.lfilter([np.float32(1.0)], a, gcur[:, ::-1], axis=1).astype(np.float32)[:, ::-1]
        xs, ys = sig[s].astype(np.float64), sig[s + 1].astype(np.float64)
        vd = v.astype(np.float64)
        for i in range(3):
            gs[s, i] = np.sum(vd[:, i:] * xs[:, :xs.shape[1] - i])
        for i in (1, 2):
            gs[s, 2 + i] = -np.sum(vd[:, i:] * ys[:, :ys.shape[1] - i])
        gcur = ss.lfilter(sec[s, :3].astype(np.float32), [np.float32(1.0)], v[:, ::-1],
                          axis=1).astype(np.float32)[:, ::-1]
        gcur = np.ascontiguousarray(gcur)
    rgx, rgs = O.sos_backward(g, x, sec)
    return channel_errors(gcur, rgx).max(), rel(gs, rgs)


def test_sos_backward_many_tiles():
    # 150 tiles per channel: the reverse-time look-back crosses windows
    C, N = 2, 150 * T + 77
    x = _x(C, N, (304,))
    g = _x(C, N, (305,), 1.0)
    sec = _sections(4, (104,), r_hi=0.995)
    xg, secg = _gpu(x), _gpu(sec)
    _, ck = tfx.sos(xg, secg, return_ckpt=True)
    gx, gs = tfx.sos_backward(xg, _gpu(g), secg, ck)
    rgx, rgs = O.sos_backward(g, x, sec)
    assert_close(_cpu(gx), rgx, TOL_GRAD, "gx")
    assert_rel(_cpu(gs), rgs, TOL_GRAD, "gsos")


def test_sos_backward_xcd_window_order():
    # 3 channel pairs x 120 tiles = 360 workgroups: on the whole 256-CU chip
    # the cascade adjoint takes the XCD window order (one full window of 256
    # workgroup ids, then a partial one)
    C, N = 5, 120 * T + 77
    x = _x(C, N, (306,))
    g = _x(C, N, (307,), 1.0)
    sec = _sections(3, (308,), r_hi=0.995)
    xg, secg = _gpu(x), _gpu(sec)
    _, ck = tfx.sos(xg, secg, return_ckpt=True)
    gx, gs = tfx.sos_backward(xg, _gpu(g), secg, ck)
    rgx, rgs = O.sos_backward(g, x, sec)
    assert_close(_cpu(gx), rgx, TOL_GRAD, "gx")
    assert_rel(_cpu(gs), rgs, TOL_GRAD, "gsos")


# Fixed bars of the three ill-conditioned cases, set from measured errors: a
# plain sequential fp32 adjoint (the cascade's conditioning floor in fp32)
# already exceeds 1e-4 on the input gradient or the high-pass's coefficient
# gradients there.
BAR_ILL_GX, BAR_ILL_GSOS = 6e-4, 1e-4
BAR_S16_GX, BAR_S16_GSOS = 1e-4, 2.5e-4
BAR_SHORT_HP = 1.5e-3


def test_sos_backward_ill_conditioned_cascade():
    # a cascade whose gain is ~2e-5 of its input: a sequential fp32 adjoint
    # loses ~1.8e-4 on the input gradient
    C, N = 2, 150 * T + 77
    x = _x(C, N, (304,))
    g = _x(C, N, (305,), 1.0)
    sec = _sections(4, (306,), r_hi=0.995)
    fx, fs = _fp32_floor(g, x, sec)
    xg, secg = _gpu(x), _gpu(sec)
    _, ck = tfx.sos(xg, secg, return_ckpt=True)
    gx, gs = tfx.sos_backward(xg, _gpu(g), secg, ck)
    rgx, rgs = O.sos_backward(g, x, sec)
    ex = float(channel_errors(_cpu(gx), rgx).max())
    es = rel(_cpu(gs), rgs)
    report("ill-conditioned gx", ex, BAR_ILL_GX, fx)
    report("ill-conditioned gsos", es, BAR_ILL_GSOS, fs)
    assert_close(_cpu(gx), rgx, BAR_ILL_GX, "gx")
    assert_rel(_cpu(gs), rgs, BAR_ILL_GSOS, "gsos")


def test_sos_backward_high_q():
    # pole radius above 0.999: the carry runs in FP64 both ways
    C, N = 2, 40 * T + 5
    x = _x(C, N, (307,))
    g = _x(C, N, (308,), 1.0)
    sec = design.random_sections(signals.rng(309), 3, 0.999, 0.9999).astype(np.float32)
    xg, secg = _gpu(x), _gpu(sec)
    _, ck = tfx.sos(xg, secg, return_ckpt=True)
    gx, gs = tfx.sos_backward(xg, _gpu(g), secg, ck)
    rgx, rgs = O.sos_backward(g, x, sec)
    assert_close(_cpu(gx), rgx, TOL_GRAD, "gx high-Q")
    assert_rel(_cpu(gs), rgs, TOL_GRAD, "gsos high-Q")


def test_sos_backward_strided_rows():
    C, N = 3, 2 * T + 9
    x = _x(C, N, (310,))
    g = _x(C, N, (311,), 1.0)
    sec = _sections(2, (312,))
    xb = torch.zeros((C, N + 13), dtype=torch.float32, device=DEV)
    xb[:, :N] = _gpu(x)
    gb = torch.zeros((C, N + 7), dtype=torch.float32, device=DEV)
    gb[:, :N] = _gpu(g)
    secg = _gpu(sec)
    _, ck = tfx.sos(xb[:, :N], secg, return_ckpt=True)
    gx, gs = tfx.sos_backward(xb[:, :N], gb[:, :N], secg, ck)
    rgx, rgs = O.sos_backward(g, x, sec)
    assert_close(_cpu(gx), rgx, TOL_GRAD, "gx strided")
    assert_rel(_cpu(gs), rgs, TOL_GRAD, "gsos strided")


def test_sos_backward_sixteen_sections():
    # the longest cascade the adjoint takes; 16 chained sections of fp32
    # rounding: a sequential fp32 adjoint loses ~1.5e-4 on the section
    # gradients
    C, N = 1, 5 * T + 1
    x = _x(C, N, (313,))
    g = _x(C, N, (314,), 1.0)
    sec = _sections(16, (315,), 0.3, 0.9)
    fx, fs = _fp32_floor(g, x, sec)
    xg, secg = _gpu(x), _gpu(sec)
    _, ck = tfx.sos(xg, secg, return_ckpt=True)
    gx, gs = tfx.sos_backward(xg, _gpu(g), secg, ck)
    rgx, rgs = O.sos_backward(g, x, sec)
    report("S=16 gx", float(channel_errors(_cpu(gx), rgx).max()), BAR_S16_GX, fx)
    report("S=16 gsos", rel(_cpu(gs), rgs), BAR_S16_GSOS, fs)
    assert_close(_cpu(gx), rgx, BAR_S16_GX, "gx S=16")
    assert_rel(_cpu(gs), rgs, BAR_S16_GSOS, "gsos S=16")


# ------------------------------------------------------------------- FIR

@pytest.mark.parametrize("M,algo", [(1, "direct"), (17, "direct"), (48, "auto"), (101, "fft"), (101, "direct"),
                                    (1023, "auto"), (1025, "fft"), (1500, "direct"), (3000, "auto")])
@pytest.mark.parametrize("N", [5000, 3 * T + 17])
def test_fir_backward_parity(M, algo, N):
    print("fir_backward M=%d %s N=%d" % (M, algo, N), flush=True)
    C = 3
    x = _x(C, N, (320, M, N))
    g = _x(C, N, (321, M, N), 1.0)
    h = design.fir_lowpass(M, 4000.0, 48000.0).astype(np.float32) if M > 1 else np.array([0.7], np.float32)
    gx, gh = tfx.fir_backward(_gpu(x), _gpu(g), _gpu(h), algo=algo)
    rgx, rgh = O.fir_backward(g, x, h)
    assert_close(_cpu(gx), rgx, TOL_FIR_F32, "gx")
    assert_rel(_cpu(gh), rgh, TOL_GRAD, "gh")


def test_fir_backward_odd_channels_and_short():
    for C, N in [(1, 7), (5, 1000), (7, 3 * T)]:
        x = _x(C, N, (322, C, N))
        g = _x(C, N, (323, C, N), 1.0)
        h = design.fir_lowpass(101, 6000.0, 48000.0).astype(np.float32)
        gx, gh = tfx.fir_backward(_gpu(x), _gpu(g), _gpu(h))
        rgx, rgh = O.fir_backward(g, x, h)
        assert_close(_cpu(gx), rgx, TOL_FIR_F32, "gx C=%d N=%d" % (C, N))
        assert_rel(_cpu(gh), rgh, TOL_GRAD, "gh C=%d N=%d" % (C, N))


# ------------------------------------------------------------------ chain

def _chain_check(x, g, stages, what, stage_tol=None, floors=None):
    xg = _gpu(x)
    st = [(k, _gpu(c)) for k, c in stages]
    has_sos = any(k == "sos" for k, _ in stages)
    if has_sos:
        _, ck = tfx.chain(xg, st, return_ckpt=True)
    else:
        ck = None
    gx, grads = tfx.chain_backward(xg, _gpu(g), st, ck)
    rgx, rgrads = O.chain_backward(g, x, stages)
    report(what + " gx", float(channel_errors(_cpu(gx), rgx).max()), TOL_GRAD)
    assert_close(_cpu(gx), rgx, TOL_GRAD, what + " gx")
    for i, (a, b) in enumerate(zip(grads, rgrads)):
        tol = (stage_tol or {}).get(i, TOL_GRAD)
        e = assert_rel(_cpu(a).reshape(np.shape(b)), b, tol, what + " stage %d" % i)
        report(what + " stage %d" % i, e, tol, (floors or {}).get(i))


def test_chain_backward_short():
    # the 100 Hz Butterworth high-pass has poles at radius 0.995 and
    # coefficients near (1, -2, 1): its coefficient gradients lose ~5e-4 even
    # in a sequential fp32 adjoint, so that stage has a fixed bar of its own
    w = workloads.chain_short(C=2, N=20000)
    g = _x(2, 20000, (330,), 1.0)
    f = O.fir(w.x, w.stages[0][1]).astype(np.float32)
    _, fs = _fp32_floor(g, f, w.stages[1][1])
    _chain_check(w.x, g, w.stages, "chain_short", {1: BAR_SHORT_HP}, {1: fs})


def test_chain_backward_mid_reduced():
    N = 9 * T + 5
    w = workloads.chain_mid(C=3, N=N)
    g = _x(3, N, (331,), 1.0)
    _chain_check(w.x, g, w.stages, "chain_mid")


def test_chain_backward_two_firs_and_sos():
    C, N = 2, 4 * T + 3
    x = _x(C, N, (332,))
    g = _x(C, N, (333,), 1.0)
    stages = [("fir", design.fir_lowpass(31, 9000.0, 48000.0).astype(np.float32)),
              ("sos", _sections(2, (334,))),
              ("fir", design.fir_lowpass(21, 5000.0, 48000.0).astype(np.float32)),
              ("sos", _sections(1, (335,)))]
    _chain_check(x, g, stages, "fir|sos|fir|sos")


def test_chain_backward_fir_only_and_sos_only():
    C, N = 3, 2 * T + 11
    x = _x(C, N, (336,))
    g = _x(C, N, (337,), 1.0)
    _chain_check(x, g, [("fir", design.fir_lowpass(65, 7000.0, 48000.0).astype(np.float32))], "fir only")
    _chain_check(x, g, [("sos", _sections(3, (338,)))], "sos only")


@pytest.mark.parametrize("M", [101, 1025])
def test_chain_backward_input_gradient_only(M):
    """Input gradient without coefficient gradients: the FFT FIR's fused
    gradient kernel then skips the tap-gradient spectra."""
    print("chain_backward gx only M=%d" % M, flush=True)
    C, N = 5, 3 * T + 101
    x = _x(C, N, (350, M))
    g = _x(C, N, (351, M), 1.0)
    h = design.fir_lowpass(M, 5000.0, 48000.0).astype(np.float32)
    for stages in ([("fir", h)], [("fir", h), ("sos", _sections(2, (352, M)))]):
        xg = _gpu(x)
        st = [(k, _gpu(c)) for k, c in stages]
        ck = tfx.chain(xg, st, return_ckpt=True)[1] if len(stages) > 1 else None
        gx, grads = tfx.chain_backward(xg, _gpu(g), st, ck, need_coef=False)
        assert all(gr is None for gr in grads)
        rgx, _ = O.chain_backward(g, x, stages)
        assert_close(_cpu(gx), rgx, TOL_GRAD, "gx only, %d stages" % len(stages))


def test_backward_deterministic():
    w = workloads.chain_mid(C=2, N=6 * T + 1)
    g = _gpu(_x(2, w.x.shape[1], (339,), 1.0))
    xg = _gpu(w.x)
    st = [(k, _gpu(c)) for k, c in w.stages]
    _, ck = tfx.chain(xg, st, return_ckpt=True)
    a = tfx.chain_backward(xg, g, st, ck)
    b = tfx.chain_backward(xg, g, st, ck)
    assert torch.equal(a[0], b[0])
    for u, v in zip(a[1], b[1]):
        assert torch.equal(u, v)


# --------------------------------------------------------------- autograd

def _pole_zero_sections(p):
    """Sections from the pole/zero parameterisation (torch ops on tiny
    tensors): r = 0.99 sigmoid(rho), theta = pi sigmoid(phi)."""
    rp = 0.99 * torch.sigmoid(p["rho_p"])
    tp = np.pi * torch.sigmoid(p["phi_p"])
    rz = 0.99 * torch.sigmoid(p["rho_z"])
    tz = np.pi * torch.sigmoid(p["phi_z"])
    k = p["k"]
    b0 = k
    b1 = -2.0 * k * rz * torch.cos(tz)
    b2 = k * rz * rz
    a1 = -2.0 * rp * torch.cos(tp)
    a2 = rp * rp
    return torch.stack([b0, b1, b2, a1, a2], dim=1).float()


def test_autograd_learnable_reduced():
    x, params, target = workloads.learnable(B=2, C=2, N=4 * T + 100)
    t = O.chain(x, target)
    xg = _gpu(x).requires_grad_(True)
    h = _gpu(params["h"]).requires_grad_(True)
    p = {k: torch.tensor(v, dtype=torch.float64, device=DEV, requires_grad=True)
         for k, v in params.items() if k != "h"}
    sec = _pole_zero_sections(p)
    sec.retain_grad()
    y = tfx.chain(xg, [("fir", h), ("sos", sec)])
    loss = torch.mean((y - _gpu(t.astype(np.float32))) ** 2)
    loss.backward()
    # oracle: the same loss gradient through the FP64 adjoint
    sec_np = sec.detach().cpu().numpy()
    yo = O.chain(x, [("fir", params["h"]), ("sos", sec_np)])
    go = 2.0 * (yo - t) / yo.size
    rgx, (rgh, rgs) = O.chain_backward(go, x, [("fir", params["h"]), ("sos", sec_np)])
    assert_close(_cpu(xg.grad), rgx, TOL_GRAD, "dL/dx")
    assert_rel(_cpu(h.grad), rgh, TOL_GRAD, "dL/dh")
    assert_rel(_cpu(sec.grad), rgs, TOL_GRAD, "dL/dsections")
    for k, v in p.items():
        assert v.grad is not None and torch.all(torch.isfinite(v.grad)), k


def test_autograd_full_learnable_size():
    # the differentiable workload at its full size: 32 x 2 channels x 192,000
    x, params, target = workloads.learnable()
    sec = target[1][1]
    h = params["h"]
    stages = [("fir", h), ("sos", sec)]
    g = _x(x.shape[0], x.shape[1], (340,), 1e-3)
    xg = _gpu(x).requires_grad_(True)
    hg = _gpu(h).requires_grad_(True)
    sg = _gpu(sec).requires_grad_(True)
    y = tfx.chain(xg, [("fir", hg), ("sos", sg)])
    y.backward(_gpu(g))
    rgx, (rgh, rgs) = O.chain_backward(g, x, stages)
    assert_close(_cpu(xg.grad), rgx, TOL_GRAD, "dL/dx full")
    assert_rel(_cpu(hg.grad), rgh, TOL_GRAD, "dL/dh full")
    assert_rel(_cpu(sg.grad), rgs, TOL_GRAD, "dL/dsections full")


def test_learnable_full_size_jvp_vs_fd():
    """Four random directions at the differentiable workload's full size
    (64 x 192,000, 255-tap FIR | 8 sections): the directional derivative of
    L = <g, chain(x; h, sos)> from the GPU adjoint against a central finite
    difference of L computed by the FP64 oracle on the host.  Directions:
    the taps, the section coefficients, the input, all three together."""
    x, params, target = workloads.learnable()
    h, sec = target[0][1], target[1][1]
    stages = [("fir", h), ("sos", sec)]
    g = _x(x.shape[0], x.shape[1], (345,), 1.0)
    xg = _gpu(x)
    st = [(k, _gpu(c)) for k, c in stages]
    _, ck = tfx.chain(xg, st, return_ckpt=True)
    gx, (gh, gs) = tfx.chain_backward(xg, _gpu(g), st, ck)
    gx, gh, gs = _cpu(gx).astype(np.float64), _cpu(gh).astype(np.float64), _cpu(gs).astype(np.float64)
    gd = g.astype(np.float64)

    def loss(xx, hh, ss):
        return float(np.sum(gd * O.chain(xx, [("fir", hh), ("sos", ss)])))

    rng = np.random.default_rng(346)
    x64, h64, s64 = x.astype(np.float64), h.astype(np.float64), sec.astype(np.float64)
    for name, (use_x, use_h, use_s) in [("taps", (0, 1, 0)), ("sections", (0, 0, 1)), ("input", (1, 0, 0)),
                                        ("all", (1, 1, 1))]:
        dx = rng.standard_normal(x.shape) * 0.1 * use_x
        dh = rng.standard_normal(h.shape) * np.abs(h).max() * use_h
        ds = rng.standard_normal(sec.shape) * 0.01 * use_s
        eps = 1e-5
        fd = (loss(x64 + eps * dx, h64 + eps * dh, s64 + eps * ds)
              - loss(x64 - eps * dx, h64 - eps * dh, s64 - eps * ds)) / (2 * eps)
        jvp = float(np.sum(gx * dx) + np.sum(gh * dh) + np.sum(gs * ds))
        err = abs(jvp - fd) / abs(fd)
        report("full-size JVP (%s)" % name, err, TOL_GRAD)
        assert err <= TOL_GRAD, "JVP along %s: GPU %.9e, FD %.9e, rel err %.3e" % (name, jvp, fd, err)


def test_autograd_only_coefficients():
    # x without requires_grad: the adjoint still gives coefficient gradients
    C, N = 2, 3 * T
    x = _x(C, N, (341,))
    sec = _sections(2, (342,))
    sg = _gpu(sec).requires_grad_(True)
    y = tfx.sos(_gpu(x), sg)
    g = _x(C, N, (343,), 1.0)
    y.backward(_gpu(g))
    _, rgs = O.sos_backward(g, x, sec)
    assert_rel(_cpu(sg.grad), rgs, TOL_GRAD, "dL/dsections")


def test_backward_empty_signal_zeroes_gradients():
    x = torch.zeros((2, 0), dtype=torch.float32, device=DEV)
    sec = _gpu(_sections(2, (344,)))
    h = _gpu(np.ones(5, np.float32))
    gx, grads = tfx.chain_backward(x, x.clone(), [("fir", h), ("sos", sec)], None)
    assert gx.shape == (2, 0)
    assert torch.count_nonzero(grads[0]) == 0 and torch.count_nonzero(grads[1]) == 0


def test_backward_rejects_missing_checkpoints():
    C, N = 1, 100
    x = _gpu(_x(C, N, (345,)))
    sec = _gpu(_sections(1, (346,)))
    with pytest.raises(lib.TfxError) as ei:
        tfx.sos_backward(x, x.clone(), sec, None)
    assert ei.value.status == 1

"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every case draws seeded inputs, runs libtfx on cuda:0 and compares element
by element with the oracle on the same fp32 inputs promoted to float64.
Tolerances (per-channel relative RMS): FP32 FIR 1e-5, FP32 IIR and chains
1e-4.
"""
import numpy as np
import pytest
import torch

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import design, lib, signals, workloads
from oracle import oracle as O
from tests.metrics import TOL_FIR_LOWP, TOL_FIR_F32, TOL_IIR_F32, assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
T = 3072  # samples per IIR tile (tfx_sos_tile_length)


def _x(C, N, key, sigma=0.1):
    return signals.to_f32(np.stack([signals.white(N, (*key, c), sigma) for c in range(C)]).reshape(C, N))


def _sections(S, key, r_hi=0.99):
    return design.random_sections(signals.rng(*key), S, 0.5, r_hi).astype(np.float32)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ------------------------------------------------------------------- SOS

@pytest.mark.parametrize("S", [1, 2, 6, 8])
@pytest.mark.parametrize("N", [1, 31, 32, 33, 8191, 8192, 8193, 3 * T + 17, 70000])
def test_sos_parity(S, N):
    C = 3
    x = _x(C, N, (101, S, N))
    sec = _sections(S, (102, S))
    y = _cpu(tfx.sos(_gpu(x), _gpu(sec)))
    assert_close(y, O.sos(x, sec), TOL_IIR_F32, "sos S=%d N=%d" % (S, N))


def _mixed_sections(key, S, nres, r_lo, r_hi):
    """nres resonators with poles at radius r_lo..r_hi (unit gain at the pole
    angle) followed by mild sections (pole radius 0.3-0.6, unit DC gain); all
    zeros at radius 0.5.  Unlike cascades of many unit-circle-zero resonators
    (gains of 1e-20 and below), the whole cascade stays well conditioned in
    fp32 (a sequential fp32 filter loses at most ~1.5e-5)."""
    g = signals.rng(*key)
    r = np.concatenate([g.uniform(r_lo, r_hi, nres), g.uniform(0.3, 0.6, S - nres)])
    th = g.uniform(0.1, np.pi - 0.1, S)
    ph = g.uniform(0.0, np.pi, S)
    rows = design.from_polar(r, th, np.full(S, 0.5), ph, np.ones(S))
    for i in range(S):
        gain = abs(design.sos_response(rows[i:i + 1], [th[i] if i < nres else 0.0])[0])
        rows[i, 0:3] /= gain
    return rows.astype(np.float32)


@pytest.mark.parametrize("S,nres,r_lo,r_hi", [(3, 3, 0.997, 0.999), (8, 2, 0.997, 0.999), (10, 2, 0.995, 0.999),
                                               (12, 1, 0.998, 0.999)])
def test_sos_slow_decay_deep_lookback(S, nres, r_lo, r_hi):
    # poles just below the FP64-carry threshold: the tile transition decays
    # slowly, so the look-back reaches several tiles back (up to 8 sections as
    # one cascade state, beyond that section by section); impulses every
    # 5000 samples excite the long tails
    C, N = 3, 120 * T + 11
    x = _x(C, N, (105, S))
    x[:, ::5000] += 1.0
    sec = _mixed_sections((106, S), S, nres, r_lo, r_hi)
    y = _cpu(tfx.sos(_gpu(x), _gpu(sec)))
    assert_close(y, O.sos(x, sec), TOL_IIR_F32, "sos S=%d r in [%g, %g]" % (S, r_lo, r_hi))


@pytest.mark.parametrize("S,fir", [(3, False), (7, False), (3, True)])
def test_xcd_window_order_deep_lookback(S, fir):
    # 3 channel pairs x 400 tiles = 1200 workgroups: on the whole 256-CU chip
    # the forward kernels take the XCD window order (4 full windows of 256
    # workgroup ids and a partial one), with slowly decaying sections whose
    # tiles look several predecessors back (S = 7: the matrix-core cascade)
    C, N = 5, 400 * T + 19
    x = _x(C, N, (107, S))
    x[:, ::7000] += 1.0
    sec = _mixed_sections((108, S), S, 2, 0.997, 0.999)
    if fir:
        stages = [("fir", workloads.chain_short(C=1, N=16).stages[0][1]), ("sos", sec)]
        y = _cpu(tfx.chain(_gpu(x), [(k, _gpu(c)) for k, c in stages]))
        ref = O.chain(x, stages)
    else:
        y = _cpu(tfx.sos(_gpu(x), _gpu(sec)))
        ref = O.sos(x, sec)
    assert_close(y, ref, TOL_IIR_F32, "xcd order S=%d fir=%s" % (S, fir))


def test_sos_many_tiles_lookback_windows():
    # 200 tiles per channel: look-back crosses several 64-tile windows
    C, N = 2, 200 * T + 5
    x = _x(C, N, (103,))
    sec = _sections(4, (104,), r_hi=0.995)
    y = _cpu(tfx.sos(_gpu(x), _gpu(sec)))
    assert_close(y, O.sos(x, sec), TOL_IIR_F32, "sos long")


def test_sos_zero_sections_is_copy():
    x = _x(2, 1000, (105,))
    y = _cpu(tfx.sos(_gpu(x), np.zeros((0, 5), np.float32)))
    assert np.array_equal(y, x)


@pytest.mark.parametrize("N", [1, 100, T, 2 * T + 300])
def test_sos_state_out_matches_oracle(N):
    C, S = 2, 3
    x = _x(C, N, (106, N))
    sec = _sections(S, (107,))
    si = (np.random.default_rng(N).standard_normal((C, S, 2)) * 0.1).astype(np.float32)
    y, so = tfx.sos(_gpu(x), _gpu(sec), state_in=_gpu(si), return_state=True)
    ref, rs = O.sos(x, sec, state_in=si, return_state=True)
    assert_close(_cpu(y), ref, TOL_IIR_F32, "with state_in")
    assert_close(_cpu(so).reshape(C, -1), rs.reshape(C, -1), TOL_IIR_F32, "state_out")


def test_sos_split_and_resume():
    C, S, N = 2, 4, 3 * T + 123
    x = _x(C, N, (108,))
    sec = _sections(S, (109,))
    full = _cpu(tfx.sos(_gpu(x), _gpu(sec)))
    k = T + 1000
    y1, st = tfx.sos(_gpu(x[:, :k]), _gpu(sec), return_state=True)
    y2 = tfx.sos(_gpu(x[:, k:]), _gpu(sec), state_in=st)
    both = np.concatenate([_cpu(y1), _cpu(y2)], axis=1)
    assert_close(both, O.sos(x, sec), TOL_IIR_F32, "split")
    assert_close(both, full, TOL_IIR_F32, "split vs one-shot")


def _resume_from_ckpt(xin, sec, ck_t, t0, t1):
    """Oracle output over samples [t0, t1) started from a checkpointed state."""
    return O.sos(xin[:, t0:t1], sec, state_in=ck_t)


def test_sos_checkpoints_are_tile_entering_states():
    C, S, N = 2, 3, 4 * T + 77
    x = _x(C, N, (110,))
    sec = _sections(S, (111,))
    _, ck = tfx.sos(_gpu(x), _gpu(sec), return_ckpt=True)
    ck = _cpu(ck)
    assert ck.shape == (C, 5, S, 2)
    assert np.all(ck[:, 0] == 0)
    ref = O.sos(x, sec)
    for t in range(1, 5):
        # restarting the cascade from the checkpoint reproduces the tile
        t1 = min(N, (t + 1) * T)
        got = _resume_from_ckpt(x, sec, ck[:, t], t * T, t1)
        assert_close(got, ref[:, t * T:t1], TOL_IIR_F32, "resume at tile %d" % t)


def test_sos_high_q_fp64_carry():
    w = workloads.high_q(C=2, N=400_000)
    sec = w.stages[0][1]
    assert design.max_pole_radius(sec) > 0.999
    y = _cpu(tfx.sos(_gpu(w.x), _gpu(sec)))
    assert_close(y, O.sos(w.x, sec), TOL_IIR_F32, "high-Q")


def test_sos_strided_rows():
    C, N, ld = 3, 20000, 20480
    big = _x(C, ld, (112,))
    sec = _sections(2, (113,))
    xt = _gpu(big)[:, :N]
    assert xt.stride(0) == ld
    y = _cpu(tfx.sos(xt, _gpu(sec)))
    assert_close(y, O.sos(big[:, :N], sec), TOL_IIR_F32, "strided")


def test_sos_deterministic():
    x = _gpu(_x(4, 5 * T + 9, (114,)))
    sec = _gpu(_sections(6, (115,)))
    a = _cpu(tfx.sos(x, sec))
    b = _cpu(tfx.sos(x, sec))
    assert np.array_equal(a, b)


def test_sos_nan_stays_in_its_channel():
    # the matrix-core cascade multiplies whole 32-sample chunks (0 x NaN is
    # NaN), so a non-finite sample reaches back to the start of its chunk;
    # nothing before that chunk and no other channel is touched
    x = _x(3, 2 * T, (116,))
    x[1, 5000] = np.nan
    sec = _sections(2, (117,))
    y = _cpu(tfx.sos(_gpu(x), _gpu(sec)))
    assert np.all(np.isfinite(y[0])) and np.all(np.isfinite(y[2]))
    c0 = 5000 // 32 * 32
    assert np.all(np.isfinite(y[1, :c0])) and np.all(np.isnan(y[1, 5000:5100]))
    assert_close(y[1, :c0], O.sos(x[1, :c0], sec), TOL_IIR_F32, "channel 1 before the NaN's chunk")
    assert_close(y[[0, 2]], O.sos(x[[0, 2]], sec), TOL_IIR_F32, "other channels")


# ------------------------------------------------------------------- FIR

@pytest.mark.parametrize("M", [1, 2, 15, 16, 17, 101, 255, 1023, 1500])
@pytest.mark.parametrize("N", [1, 100, T + 1, 3 * T - 5])
def test_fir_direct_parity(M, N):
    C = 2
    x = _x(C, N, (120, M, N))
    h = (np.random.default_rng(M).standard_normal(M) / np.sqrt(M)).astype(np.float32)
    y = _cpu(tfx.fir(_gpu(x), _gpu(h), algo="direct"))
    assert_close(y, O.fir(x, h), TOL_FIR_F32, "fir M=%d N=%d" % (M, N))


@pytest.mark.parametrize("M", [1, 2, 49, 101, 255, 1023, 1024, 1025])
@pytest.mark.parametrize("C,N", [(1, 1), (2, 100), (3, T + 1), (4, 5 * T - 5), (1, 20000)])
def test_fir_fft_parity(M, C, N):
    x = _x(C, N, (131, M, C, N))
    h = (np.random.default_rng(M + 7).standard_normal(M) / np.sqrt(M)).astype(np.float32)
    y = _cpu(tfx.fir(_gpu(x), _gpu(h), algo="fft"))
    assert_close(y, O.fir(x, h), TOL_FIR_F32, "fft fir M=%d C=%d N=%d" % (M, C, N))


def test_fir_fft_lowpass_designed_taps():
    w = workloads.chain_mid(C=3, N=4 * T + 17)
    h = w.stages[0][1]
    y = _cpu(tfx.fir(_gpu(w.x), _gpu(h), algo="fft"))
    assert_close(y, O.fir(w.x, h), TOL_FIR_F32, "fft band-pass 1023")


@pytest.mark.parametrize("M", [1026, 2050, 2051, 3000, 8191])
@pytest.mark.parametrize("C,N", [(1, 500), (2, 3 * T + 5), (3, 9000)])
def test_fir_fft_partitioned_parity(M, C, N):
    # taps beyond 1025: partitions of 1025 taps summed in the frequency domain
    x = _x(C, N, (132, M, C, N))
    h = (np.random.default_rng(M + 11).standard_normal(M) / np.sqrt(M)).astype(np.float32)
    y = _cpu(tfx.fir(_gpu(x), _gpu(h), algo="fft"))
    assert_close(y, O.fir(x, h), TOL_FIR_F32, "partitioned fft fir M=%d C=%d N=%d" % (M, C, N))


def test_fir_long_lowpass_reduced():
    # the 8191-tap low-pass of the long-filter workload on 2 x 40,000 samples
    w = workloads.fir_long(C=2, N=40_000)
    y = _cpu(tfx.fir(_gpu(w.x), _gpu(w.stages[0][1])))
    assert_close(y, O.fir(w.x, w.stages[0][1]), TOL_FIR_F32, "fir_long 8191 taps")


def test_fir_longer_than_one_lds_pass():
    C, N, M = 2, 2 * T + 3, 3000
    x = _x(C, N, (121,))
    h = (np.random.default_rng(7).standard_normal(M) / np.sqrt(M)).astype(np.float32)
    y = _cpu(tfx.fir(_gpu(x), _gpu(h)))
    assert_close(y, O.fir(x, h), TOL_FIR_F32, "fir 3000 taps")


def test_fir_impulse_gives_taps():
    h = np.random.default_rng(1).standard_normal(101).astype(np.float32)
    x = np.zeros((1, 500), np.float32)
    x[0, 0] = 1.0
    y = _cpu(tfx.fir(_gpu(x), _gpu(h), algo="direct"))      # bit-exact: one product per output
    assert np.array_equal(y[0, :101], h) and np.all(y[0, 101:] == 0)
    yf = _cpu(tfx.fir(_gpu(x), _gpu(h), algo="fft"))        # FFT: exact up to rounding
    assert np.max(np.abs(yf[0, :101] - h)) < 1e-6 * np.abs(h).max()
    assert np.max(np.abs(yf[0, 101:])) < 1e-6 * np.abs(h).max()


# ----------------------------------------------------------------- chains

def test_chain_short_full_size():
    w = workloads.chain_short()
    y = _cpu(tfx.chain(_gpu(w.x), w.stages))
    assert_close(y, O.chain(w.x, w.stages), TOL_IIR_F32, "chain_short")


def test_chain_mid_reduced():
    w = workloads.chain_mid(C=3, N=150_000)
    y = _cpu(tfx.chain(_gpu(w.x), w.stages))
    assert_close(y, O.chain(w.x, w.stages), TOL_IIR_F32, "chain_mid reduced")


@pytest.mark.parametrize("C", [1, 2, 5])
def test_chain_fft_fused_odd_and_even_channels(C):
    w = workloads.chain_short(C=C, N=7 * T + 123)
    y = _cpu(tfx.chain(_gpu(w.x), w.stages))
    assert_close(y, O.chain(w.x, w.stages), TOL_IIR_F32, "chain_short C=%d" % C)


def test_chain_direct_fir_with_sections():
    # 40 taps -> the direct path is picked; fused with a 3-section cascade
    x = _x(3, 4 * T + 9, (133,))
    h = design.fir_lowpass(40, 6000.0, 48000.0).astype(np.float32)
    sec = _sections(3, (134,))
    stages = [("fir", h), ("sos", sec)]
    y = _cpu(tfx.chain(_gpu(x), stages))
    assert_close(y, O.chain(x, stages), TOL_IIR_F32, "direct fir | sos")


def test_chain_two_fir_stages_merge():
    x = _x(2, 3 * T + 11, (122,))
    h1 = design.fir_lowpass(31, 5000.0, 48000.0).astype(np.float32)
    h2 = design.fir_lowpass(17, 9000.0, 48000.0).astype(np.float32)
    sec = _sections(2, (123,))
    stages = [("fir", h1), ("sos", sec), ("fir", h2)]
    y = _cpu(tfx.chain(_gpu(x), stages))
    assert_close(y, O.chain(x, stages), TOL_IIR_F32, "fir|sos|fir")


def test_chain_checkpoints_are_section_states():
    w = workloads.chain_short(C=2, N=3 * T + 5)
    y, ck = tfx.chain(_gpu(w.x), w.stages, return_ckpt=True)
    ck = _cpu(ck)
    fir_out = O.fir(w.x, w.stages[0][1])
    sec = w.stages[1][1]
    ref = O.sos(fir_out, sec)
    for t in (1, 2, 3):
        t1 = min(fir_out.shape[1], (t + 1) * T)
        got = _resume_from_ckpt(fir_out, sec, ck[:, t], t * T, t1)
        assert_close(got, ref[:, t * T:t1], TOL_IIR_F32, "chain resume at tile %d" % t)


@pytest.mark.slow
def test_chain_mid_full_size():
    w = workloads.chain_mid()
    y = _cpu(tfx.chain(_gpu(w.x), w.stages))
    assert_close(y, O.chain(w.x, w.stages), TOL_IIR_F32, "chain_mid full")


# ----------------------------------------------------------------- errors

def test_alias_rejected():
    x = _gpu(_x(2, 1000, (124,)))
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    sec = _gpu(_sections(1, (125,)))
    st = lib.load().tfx_sos(x.data_ptr(), x.data_ptr() + 400, 2, 1000, 1000, 1000, sec.data_ptr(), 1,
                            None, None, None, ws.data_ptr(), ws.numel(), None)
    assert lib.STATUS_NAMES[st] == "TFX_E_ALIAS"


def test_workspace_too_small_rejected():
    x = _gpu(_x(2, 1000, (126,)))
    y = torch.empty_like(x)
    ws = torch.empty(256, dtype=torch.uint8, device=DEV)
    sec = _gpu(_sections(1, (127,)))
    st = lib.load().tfx_sos(x.data_ptr(), y.data_ptr(), 2, 1000, 1000, 1000, sec.data_ptr(), 1,
                            None, None, None, ws.data_ptr(), ws.numel(), None)
    assert lib.STATUS_NAMES[st] == "TFX_E_WORKSPACE"
    assert b"too small" in lib.load().tfx_last_error()


def test_cpu_tensor_rejected():
    with pytest.raises(TypeError):
        tfx.sos(torch.zeros(2, 10), np.zeros((1, 5), np.float32))


def test_chain_run_replays_on_prepared_workspace():
    # one prepare, many runs: the epoch-tagged look-back must re-arm itself
    from paper_2504_08624_amd.functional import _stages
    C, N = 3, 5 * T + 7
    w = workloads.chain_short(C=C, N=N)
    x2 = _x(C, N, (130,))
    kept, desc = _stages(w.stages, torch.device(DEV))
    arr = lib.stage_array(desc)
    L = lib.load()
    nb = lib.size_out()
    lib.call("tfx_chain_workspace_size", C, N, arr, len(desc), 0, nb)
    ws = torch.empty(nb.value, dtype=torch.uint8, device=DEV)
    sp = torch.cuda.current_stream().cuda_stream
    lib.check(L.tfx_chain_prepare(C, N, arr, len(desc), 0, ws.data_ptr(), ws.numel(), sp), "prepare")
    refs = [O.chain(w.x, w.stages), O.chain(x2, w.stages)]
    xs = [_gpu(w.x), _gpu(x2)]
    for i in range(7):
        y = torch.empty_like(xs[i % 2])
        lib.check(L.tfx_chain_run(xs[i % 2].data_ptr(), y.data_ptr(), C, N, N, N, arr, len(desc), 0, None,
                                  ws.data_ptr(), ws.numel(), sp), "run")
        assert_close(_cpu(y), refs[i % 2], TOL_IIR_F32, "replay %d" % i)
    hdr = _cpu(ws[:16].view(torch.int32))
    assert hdr[1] == 0 and hdr[2] == 8  # epoch advanced once per run, no spin timeouts


# ------------------------------------------- cascade lengths of the table form

@pytest.mark.parametrize("S", [1, 2, 3, 4, 5, 6, 7, 8])
def test_chain_fft_every_cascade_length(S):
    """FFT FIR then S sections: up to six sections the cascade's second phase
    is the zero-input-response table form, seven and eight take the
    matrix-core form; both against the oracle, over several tiles and a
    ragged tail, with poles up to radius 0.994."""
    x = _x(3, 4 * T + 17, (90, S))
    h = design.fir_lowpass(255, 5000.0, 48000.0).astype(np.float32)
    # peaking sections across the band (gains near one: a well-conditioned
    # cascade, so fp32 rounding stays at its own size in the output)
    g = signals.rng(91, S)
    sec = np.concatenate([design.peaking(f, q, gd, 48000.0) for f, q, gd in
                          zip(np.geomspace(300.0, 12000.0, S), g.uniform(0.7, 4.0, S), g.uniform(-9.0, 9.0, S))])
    sec = sec.astype(np.float32)
    assert 0.975 < design.max_pole_radius(sec) < 0.999  # below the FP64-carry threshold
    y = _cpu(tfx.chain(_gpu(x), [("fir", _gpu(h)), ("sos", _gpu(sec))]))
    assert_close(y, O.chain(x, [("fir", h), ("sos", sec)]), TOL_IIR_F32, "FFT FIR + %d sections" % S)


@pytest.mark.parametrize("S", [3, 5])
def test_sos_state_in_through_the_table_form(S):
    """A nonzero state entering the first tile reaches every later sample
    through the zero-input response; no final state is asked for."""
    x = _x(2, 3 * T + 5, (92, S))
    sec = _sections(S, (93, S), r_hi=0.995)
    st = signals.rng(94, S).standard_normal((2, S, 2)).astype(np.float32)
    y = _cpu(tfx.sos(_gpu(x), _gpu(sec), state_in=_gpu(st)))
    assert_close(y, O.sos(x, sec, state_in=st), TOL_IIR_F32, "state_in, %d sections" % S)


@pytest.mark.parametrize("S", [7, 8])
@pytest.mark.parametrize("fir", ["none", "direct", "fft", "bf16"])
def test_chain_matrix_core_cascade_every_fir_form(S, fir):
    """Cascades of seven and eight sections run on the matrix cores behind
    every FIR form: odd channel count (a half-empty channel pair), several
    tiles and a ragged tail, a state entering the first tile, and the tile
    checkpoints, against the oracle."""
    C, N = 3, 5 * T + 1234
    x = _x(C, N, (140, S))
    g = signals.rng(141, S)
    sec = np.concatenate([design.peaking(f, q, gd, 48000.0) for f, q, gd in
                          zip(np.geomspace(200.0, 15000.0, S), g.uniform(0.7, 6.0, S), g.uniform(-9.0, 9.0, S))])
    sec = sec.astype(np.float32)
    si = (0.01 * signals.rng(142, S).standard_normal((C, S, 2))).astype(np.float32)
    stages, tol, kw = [], TOL_IIR_F32, {}
    if fir == "direct":
        stages = [("fir", design.fir_lowpass(17, 9000.0, 48000.0).astype(np.float32))]
    elif fir == "fft":
        stages = [("fir", design.fir_lowpass(255, 5000.0, 48000.0).astype(np.float32))]
    elif fir == "bf16":
        stages = [("fir", design.fir_lowpass(33, 9000.0, 48000.0).astype(np.float32))]
        tol, kw = TOL_FIR_LOWP, {"compute": "bf16"}
    xg = _gpu(x)
    st = [(k, _gpu(c)) for k, c in stages] + [("sos", _gpu(sec))]
    y, ck = tfx.chain(xg, st, return_ckpt=True, **kw)
    ref = O.chain(x, stages + [("sos", sec)])
    assert_close(_cpu(y), ref, tol, "%s FIR + %d sections" % (fir, S))
    # checkpoints: the state entering every section at every tile start
    f = O.chain(x, stages) if stages else x.astype(np.float64)
    ckc = _cpu(ck)
    for t in (1, 3, 5):
        _, s_ref = O.sos(f[:, :t * T], sec, return_state=True)
        assert_close(ckc[:, t].reshape(C, -1), s_ref.reshape(C, -1), 10 * tol, "checkpoint tile %d" % t)
    if fir == "none":
        # a state entering the first tile
        y2 = _cpu(tfx.sos(xg, _gpu(sec), state_in=_gpu(si)))
        assert_close(y2, O.sos(x, sec, state_in=si), TOL_IIR_F32, "state_in, %d sections" % S)

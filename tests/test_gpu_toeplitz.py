"""GPU parity of the matrix-core block-Toeplitz FIR (bf16 / fp16 operands,
fp32 accumulation; split-bf16 with three products) against the FP64 oracle.

Tolerances (per-channel relative RMS): 1e-2 for bf16 and fp16 operands; the
split-bf16 mode represents each operand to about 2^-17 relative and drops
only the lo*lo product, so it is held to 1e-4.
"""
import numpy as np
import pytest
import torch

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import design, lib, signals, workloads
from oracle import oracle as O
from tests.metrics import TOL_FIR_LOWP, assert_close, channel_errors

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
T = 3072
TOL_SPLIT = 1e-4
TOL = {"bf16": TOL_FIR_LOWP, "f16": TOL_FIR_LOWP, "bf16x3": TOL_SPLIT}
TOL_SAME = 1e-5  # same arithmetic up to the look-back's combination order


def _x(C, N, key, sigma=0.1):
    return signals.to_f32(np.stack([signals.white(N, (*key, c), sigma) for c in range(C)]).reshape(C, N))


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("compute", ["bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("M", [1, 2, 31, 32, 33, 101, 1023, 6200])
@pytest.mark.parametrize("C,N", [(1, 1), (2, 1000), (3, 16384 + 33), (1, 40000)])
def test_toeplitz_parity(compute, M, C, N):
    print("toeplitz %s M=%d C=%d N=%d" % (compute, M, C, N), flush=True)
    x = _x(C, N, (401, M, C, N))
    # random taps: no near-zero leading tap, so even N = 1 has a meaningful output
    h = (np.random.default_rng(M + 17).standard_normal(M) / np.sqrt(M)).astype(np.float32)
    y = _cpu(tfx.fir(_gpu(x), _gpu(h), compute=compute))
    assert_close(y, O.fir(x, h), TOL[compute], "toeplitz %s M=%d C=%d N=%d" % (compute, M, C, N))


def test_toeplitz_lags_beyond_one_lds_stage():
    # 8191 taps = 257 frame lags: two LDS stages of lags
    w = workloads.fir_long(C=2, N=50_000)
    h = w.stages[0][1]
    ref = O.fir(w.x, h)
    for compute in ("bf16", "f16", "bf16x3"):
        y = _cpu(tfx.fir(_gpu(w.x), _gpu(h), compute=compute))
        assert_close(y, ref, TOL[compute], "fir_long %s" % compute)


def test_toeplitz_accuracy_order():
    # split-bf16 beats fp16, which beats bf16 (mantissas of 8, 11, ~16 bits)
    x = _x(2, 20000, (402,))
    h = design.fir_lowpass(255, 4000.0, 48000.0).astype(np.float32)
    ref = O.fir(x, h)
    err = {c: channel_errors(_cpu(tfx.fir(_gpu(x), _gpu(h), compute=c)), ref).max()
           for c in ("bf16", "f16", "bf16x3")}
    assert err["bf16x3"] < err["f16"] < err["bf16"], err


def test_toeplitz_strided_rows_and_unaligned():
    C, N = 3, 20000
    x = _x(C, N, (403,))
    h = design.fir_lowpass(77, 5000.0, 48000.0).astype(np.float32)
    xb = torch.zeros((C, N + 5), dtype=torch.float32, device=DEV)
    xb[:, 1:N + 1] = _gpu(x)  # rows start 4 bytes past a 16-byte boundary
    y = _cpu(tfx.fir(xb[:, 1:N + 1], _gpu(h), compute="bf16"))
    assert_close(y, O.fir(x, h), TOL_FIR_LOWP, "toeplitz strided")


def test_toeplitz_deterministic():
    x = _gpu(_x(2, 30000, (404,)))
    h = _gpu(design.fir_lowpass(513, 3000.0, 48000.0).astype(np.float32))
    a = tfx.fir(x, h, compute="bf16")
    b = tfx.fir(x, h, compute="bf16")
    assert torch.equal(a, b)


@pytest.mark.parametrize("compute", ["bf16", "bf16x3"])
def test_chain_with_matrix_core_fir(compute):
    # low-precision FIR part, then the fp32 cascade in place
    w = workloads.chain_mid(C=3, N=5 * T + 11)
    st = [(k, _gpu(c)) for k, c in w.stages]
    y = _cpu(tfx.chain(_gpu(w.x), st, compute=compute))
    assert_close(y, O.chain(w.x, w.stages), TOL[compute], "chain_mid %s" % compute)


def _sections(S, key, r_lo=0.5, r_hi=0.99):
    rng = np.random.default_rng(list(key))
    rows = []
    for _ in range(S):
        r, th = rng.uniform(r_lo, r_hi), rng.uniform(0.05, 3.0)
        z = rng.uniform(0.3, 1.2)
        rows.append([1.0, -2 * z * np.cos(th * 0.7), z * z, -2 * r * np.cos(th), r * r])
    return np.asarray(rows, np.float32)


@pytest.mark.parametrize("compute", ["bf16", "f16"])
@pytest.mark.parametrize("M", [1, 33, 1023, 2100])
@pytest.mark.parametrize("C,N,S", [(1, 1, 2), (2, 100, 3), (3, 5 * T + 11, 6), (2, 2 * T + 5, 10)])
def test_chain_fused_matrix_core_fir_matches_two_passes(compute, M, C, N, S):
    """With a cascade behind it, the bf16 / fp16 matrix-core FIR runs inside
    the chain kernel; its output must match the stand-alone matrix-core FIR
    followed by the fp32 cascade (the same products in the same order and the
    same cascade code; only the decoupled look-back, which combines a
    predecessor's aggregate or its inclusive prefix depending on which is
    out first, may round differently), and the oracle at the bf16/fp16 bar.
    M = 2100 needs two operand passes (65 lags); S = 10 takes the per-section
    look-back."""
    print("fused tz chain %s M=%d C=%d N=%d S=%d" % (compute, M, C, N, S), flush=True)
    x = _x(C, N, (410, M, C, N))
    # random taps: no near-zero leading tap, so even N = 1 has a meaningful output
    h = (np.random.default_rng(M + 23).standard_normal(M) / np.sqrt(M)).astype(np.float32)
    sec = _sections(S, (411, M, S))
    xg, hg, sg = _gpu(x), _gpu(h), _gpu(sec)
    y, ck = tfx.chain(xg, [("fir", hg), ("sos", sg)], compute=compute, return_ckpt=True)
    f = tfx.fir(xg, hg, compute=compute)
    y2, ck2 = tfx.sos(f, sg, return_ckpt=True)
    assert_close(_cpu(y), _cpu(y2).astype(np.float64), TOL_SAME, "fused vs two passes")
    assert_close(_cpu(ck).reshape(C, -1), _cpu(ck2).reshape(C, -1).astype(np.float64), TOL_SAME, "checkpoints")
    ref = O.chain(x, [("fir", h), ("sos", sec)])
    assert_close(_cpu(y), ref, TOL[compute], "fused chain %s M=%d" % (compute, M))


def test_chain_fused_matrix_core_fir_high_q_and_strided():
    """A section with pole radius above 0.999 (the FP64-carry kernel variant)
    and rows with a stride (no 16-byte alignment) through the fused path."""
    C, N = 3, 4 * T + 7
    x = _x(C, N + 3, (412,))
    h = design.fir_lowpass(255, 5000.0, 48000.0).astype(np.float32)
    sec = np.concatenate([_sections(2, (413,)), np.array([[1.0, 0.0, -1.0, -2 * 0.9995 * np.cos(0.01), 0.9995 ** 2]],
                                                           np.float32)])
    xb = _gpu(x)
    xs = xb[:, 1:N + 1]
    y = tfx.chain(xs, [("fir", _gpu(h)), ("sos", _gpu(sec))], compute="bf16")
    y2 = tfx.sos(tfx.fir(xs, _gpu(h), compute="bf16"), _gpu(sec))
    assert_close(_cpu(y), _cpu(y2).astype(np.float64), TOL_SAME, "fused vs two passes, high-Q")
    assert_close(_cpu(y), O.chain(x[:, 1:N + 1], [("fir", h), ("sos", sec)]), TOL_FIR_LOWP, "fused high-Q")


def test_low_precision_rejects_fp32_only_algorithms():
    x = _gpu(_x(1, 100, (405,)))
    with pytest.raises(lib.TfxError, match="UNSUPPORTED"):
        tfx.fir(x, np.ones(8, np.float32), compute="bf16", algo="fft")
    with pytest.raises(lib.TfxError, match="UNSUPPORTED"):
        tfx.fir(x, np.ones(8, np.float32), compute="f32", algo="toeplitz")

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


def test_low_precision_rejects_fp32_only_algorithms():
    x = _gpu(_x(1, 100, (405,)))
    with pytest.raises(lib.TfxError, match="UNSUPPORTED"):
        tfx.fir(x, np.ones(8, np.float32), compute="bf16", algo="fft")
    with pytest.raises(lib.TfxError, match="UNSUPPORTED"):
        tfx.fir(x, np.ones(8, np.float32), compute="f32", algo="toeplitz")

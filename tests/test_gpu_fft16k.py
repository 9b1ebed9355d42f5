"""GPU parity of the overlap-save FIR with one 16384-point FFT per block of
8192 outputs (filters of 1026..8193 taps; the automatic choice in that
range), through the C ABI, against the FP64 oracle at the FP32 FIR tolerance
(1e-5): several blocks and a ragged tail, odd channel counts, the longest
filter the form takes, the adjoint correlation (input gradient) and tap
gradient, a cascade behind it, streaming blocks carrying the FIR history,
and sampled outputs of the 64 x 5,760,000 long-filter workload at full size.
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
B = 8192  # outputs per block


def _x(C, N, key, sigma=0.1):
    return signals.to_f32(np.stack([signals.white(N, (*key, c), sigma) for c in range(C)]).reshape(C, N))


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _taps(M, seed):
    return (np.random.default_rng(seed).standard_normal(M) / np.sqrt(M)).astype(np.float32)


@pytest.mark.parametrize("M", [1026, 2049, 4097, 8191, 8193])
@pytest.mark.parametrize("C,N", [(1, 1), (2, 100), (3, B - 1), (1, B), (2, B + 1), (3, 3 * B + 17), (4, 50_000)])
def test_fir_fft16k_parity(M, C, N):
    print("fft16k M=%d C=%d N=%d" % (M, C, N), flush=True)
    x = _x(C, N, (601, M, C, N))
    h = _taps(M, M + 601)
    y = _cpu(tfx.fir(_gpu(x), _gpu(h), algo="fft16k"))
    assert_close(y, O.fir(x, h), TOL_FIR_F32, "fft16k M=%d C=%d N=%d" % (M, C, N))


def test_fir_fft16k_is_the_automatic_choice():
    C, N, M = 2, 2 * B + 5, 3000
    x = _gpu(_x(C, N, (602,)))
    h = _gpu(_taps(M, 602))
    assert torch.equal(tfx.fir(x, h), tfx.fir(x, h, algo="fft16k"))


def test_fir_fft16k_impulse_and_refusal():
    h = np.random.default_rng(603).standard_normal(5000).astype(np.float32)
    x = np.zeros((1, 20_000), np.float32)
    x[0, 0] = 1.0
    x[0, 12_000] = 1.0  # an impulse in the third block, reaching into the fourth
    y = _cpu(tfx.fir(_gpu(x), _gpu(h), algo="fft16k"))[0]
    ref = np.zeros(20_000)
    ref[:5000] += h
    ref[12_000:17_000] += h
    assert np.max(np.abs(y - ref)) < 1e-6 * np.abs(h).max()
    with pytest.raises(lib.TfxError) as ei:  # more taps than the form takes
        tfx.fir(_gpu(x), _gpu(np.ones(8194, np.float32)), algo="fft16k")
    assert ei.value.status == 2


def test_fir_fft16k_strided_rows():
    C, N, M = 3, 2 * B + 333, 2500
    x = _x(C, N, (604,))
    h = _taps(M, 604)
    xb = torch.zeros((C, N + 29), dtype=torch.float32, device=DEV)
    xb[:, :N] = _gpu(x)
    y = _cpu(tfx.fir(xb[:, :N], _gpu(h), algo="fft16k"))
    assert_close(y, O.fir(x, h), TOL_FIR_F32, "fft16k strided")


@pytest.mark.parametrize("M", [1500, 8191])
def test_fir_fft16k_backward(M):
    """Input gradient by the correlation form of the same kernel (block at
    the tile, conjugated spectrum); tap gradient by the FFT cross-correlation
    kernels."""
    print("fft16k backward M=%d" % M, flush=True)
    C, N = 3, 3 * B + 101
    x = _x(C, N, (605, M))
    g = _x(C, N, (606, M), 1.0)
    h = design.fir_lowpass(M, 4000.0, 48000.0).astype(np.float32)
    gx, gh = tfx.fir_backward(_gpu(x), _gpu(g), _gpu(h), algo="fft16k")
    rgx, rgh = O.fir_backward(g, x, h)
    assert_close(_cpu(gx), rgx, TOL_FIR_F32, "gx")
    e = np.linalg.norm(_cpu(gh).astype(np.float64) - rgh) / np.linalg.norm(rgh)
    print("fft16k backward M=%d: gx ok, gh rel err %.3e" % (M, e), flush=True)
    assert e <= 1e-4


def test_chain_fft16k_with_cascade_and_autograd():
    C, N, M = 2, 4 * B + 7, 2049
    x = _x(C, N, (607,))
    h = design.fir_lowpass(M, 3000.0, 48000.0).astype(np.float32)
    sec = design.random_sections(signals.rng(608), 3, 0.5, 0.95).astype(np.float32)
    stages = [("fir", h), ("sos", sec)]
    y = _cpu(tfx.chain(_gpu(x), stages))
    assert_close(y, O.chain(x, stages), TOL_IIR_F32, "fft16k FIR | 3 SOS")
    g = _x(C, N, (609,), 1.0)
    xg = _gpu(x).requires_grad_(True)
    hg = _gpu(h).requires_grad_(True)
    sg = _gpu(sec).requires_grad_(True)
    tfx.chain(xg, [("fir", hg), ("sos", sg)]).backward(_gpu(g))
    rgx, (rgh, rgs) = O.chain_backward(g, x, stages)
    assert_close(_cpu(xg.grad), rgx, TOL_IIR_F32, "dL/dx")
    for a, b, what in ((hg.grad, rgh, "dL/dh"), (sg.grad, rgs, "dL/dsos")):
        e = np.linalg.norm(_cpu(a).astype(np.float64).ravel() - np.ravel(b)) / np.linalg.norm(b)
        assert e <= 1e-4, "%s rel err %.3e" % (what, e)


@pytest.mark.parametrize("blk", [1000, 8192, 20_000])
def test_stream_fft16k_history(blk):
    C, M = 3, 4000
    N = 3 * blk + 17 if blk < 20_000 else 2 * blk
    x = _x(C, N, (610, blk))
    h = _taps(M, 610)
    sec = design.random_sections(signals.rng(611), 2, 0.5, 0.9).astype(np.float32)
    stages = [("fir", h), ("sos", sec)]
    sm = tfx.ChainStream([(k, _gpu(c)) for k, c in stages], C, blk)
    xs = _gpu(x)
    ys = [sm.process(xs[:, i:i + blk].contiguous()) for i in range(0, N, blk)]
    y = _cpu(torch.cat(ys, dim=1))
    assert_close(y, O.chain(x, stages), TOL_IIR_F32, "stream fft16k blocks of %d" % blk)


@pytest.mark.slow
def test_fir_long_full_size_sampled():
    """The long-filter workload at full size (64 x 5,760,000, 8191 taps) in
    the launch the benchmark times: 4 channels (both halves of two pairs and
    the last channel) on 300 outputs each, spread over the signal and
    including the first and last samples, against the oracle computed output
    by output."""
    w = workloads.fir_long()
    h = w.stages[0][1]
    x = _gpu(w.x)
    y = tfx.fir(x, _gpu(h))
    torch.cuda.synchronize()
    N = w.x.shape[1]
    pos = np.unique(np.concatenate([np.linspace(0, N - 1, 296).astype(np.int64), [1, 8191, 8192, N - 2]]))
    chans = [0, 1, 40, 63]
    got = y[chans][:, torch.from_numpy(pos).to(DEV)].cpu().numpy()
    ref = O.fir_at(w.x[chans], h, pos)
    e = channel_errors(got, ref)
    print("fir_long full size, sampled: max per-channel rel err %.3e" % e.max(), flush=True)
    assert e.max() <= TOL_FIR_F32

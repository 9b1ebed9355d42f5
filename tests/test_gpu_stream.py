"""Streaming (block-by-block) chains: filtering a signal block by block with
ChainStream (tfx_chain_stream: carried FIR input history and cascade
registers) must give the same signal as filtering it in one piece, for every
FIR form (direct, FFT, partitioned FFT, matrix-core fused and stand-alone),
block lengths from 0 and 1 sample to the prepared maximum, and FIR histories
longer than the blocks."""
import numpy as np
import pytest
import torch

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import design, lib, signals
from oracle import oracle as O
from tests.metrics import TOL_FIR_F32, TOL_FIR_LOWP, TOL_IIR_F32, assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
T = 3072


def _x(C, N, key):
    return signals.to_f32(np.stack([signals.white(N, (*key, c), 0.1) for c in range(C)]).reshape(C, N))


def _cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _sections(S, key):
    rng = np.random.default_rng(list(key))
    rows = []
    for _ in range(S):
        r, th = rng.uniform(0.5, 0.99), rng.uniform(0.05, 3.0)
        rows.append([1.0, -1.2 * np.cos(th), 0.5, -2 * r * np.cos(th), r * r])
    return np.asarray(rows, np.float32)


def _blocks(total, sizes, seed):
    rng = np.random.default_rng(seed)
    out, n = [], 0
    while n < total:
        b = min(int(rng.choice(sizes)), total - n)
        out.append(b)
        n += b
    return out


CASES = {
    "fft1023+sos6": ([("fir", 1023), ("sos", 6)], "f32", TOL_IIR_F32),
    "direct17+sos2": ([("fir", 17), ("sos", 2)], "f32", TOL_IIR_F32),
    "parts2100": ([("fir", 2100)], "f32", TOL_FIR_F32),
    "fir255+fir31+sos3": ([("fir", 255), ("fir", 31), ("sos", 3)], "f32", TOL_IIR_F32),
    "sos10": ([("sos", 10)], "f32", TOL_IIR_F32),
    "bf16 255+sos2": ([("fir", 255), ("sos", 2)], "bf16", TOL_FIR_LOWP),
    "bf16 fir 300": ([("fir", 300)], "bf16", TOL_FIR_LOWP),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("sizes,nmax", [((1, 7, 64, 300), 300), ((0, 1000, 3071, 3072, 3073, 7000), 7000)])
def test_stream_matches_one_piece(case, sizes, nmax):
    spec, compute, tol = CASES[case]
    print("stream %s sizes %s" % (case, sizes), flush=True)
    C, N = 3, 24000 if nmax > 1000 else 2400
    x = _x(C, N, (600, len(case), nmax))
    stages = []
    for i, (k, n) in enumerate(spec):
        if k == "fir":
            h = np.random.default_rng(n + i).standard_normal(n) / np.sqrt(n)
            stages.append(("fir", h.astype(np.float32)))
        else:
            stages.append(("sos", _sections(n, (601, n, i))))
    st = [(k, torch.from_numpy(c).to(DEV)) for k, c in stages]
    xs = torch.from_numpy(x).to(DEV)
    stream = tfx.ChainStream(st, C, nmax, compute=compute)
    outs, n0 = [], 0
    for b in _blocks(N, sizes, 602):
        outs.append(_cpu(stream.process(xs[:, n0:n0 + b].contiguous())))
        n0 += b
    y = np.concatenate(outs, axis=1)
    assert y.shape == (C, N)
    ref = O.chain(x, stages)
    assert_close(y, ref, tol, "stream %s" % case)
    one = _cpu(tfx.chain(xs, st, compute=compute))
    assert_close(y, one.astype(np.float64), max(tol, 1e-5), "stream vs one piece %s" % case)


def test_stream_reset_starts_a_new_stream():
    C, N = 2, 5000
    x = _x(C, N, (603,))
    h = design.fir_lowpass(101, 4000.0, 48000.0).astype(np.float32)
    sec = _sections(2, (604,))
    st = [("fir", torch.from_numpy(h).to(DEV)), ("sos", torch.from_numpy(sec).to(DEV))]
    stream = tfx.ChainStream(st, C, 2000)
    xs = torch.from_numpy(x).to(DEV)
    a = _cpu(stream.process(xs[:, :2000].contiguous()))
    stream.process(xs[:, 2000:4000].contiguous())
    stream.reset()
    b = _cpu(stream.process(xs[:, :2000].contiguous()))
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-6 * np.abs(a).max())


def test_stream_rejects_blocks_longer_than_prepared():
    st = [("sos", torch.from_numpy(_sections(1, (605,))).to(DEV))]
    stream = tfx.ChainStream(st, 1, 100)
    with pytest.raises(lib.TfxError, match="INVALID_ARG"):
        stream.process(torch.zeros(1, 101, device=DEV))

"""GPU parity of the batched real FFT (tfx_rfft / tfx_irfft through the C
ABI) against the FP64 oracle (the DFT sums written out): every power-of-two
size 16..4096, an odd number of rows, contiguous rows (two rows share a
complex FFT) and strided rows (one row per channel), the round trip, and
sampled rows of a 46-million-sample batch.  Tolerance 1e-5 relative RMS per
row (an fp32 radix-16 FFT of up to 2^12 points rounds about sqrt(12) times
per value)."""
import numpy as np
import pytest
import torch

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import lib, signals
from oracle import fft as F
from tests.metrics import assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = 1e-5


def _rows(B, n, key):
    return signals.to_f32(np.stack([signals.white(n, (*key, b), 1.0) for b in range(B)]).reshape(B, n))


def _cplx(a):
    a = np.asarray(a)
    return np.concatenate([a.real, a.imag], axis=-1)


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
@pytest.mark.parametrize("B", [1, 7])
def test_rfft_irfft_parity(n, B):
    x = _rows(B, n, (801, n, B))
    X = tfx.rfft(torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    ref = F.rfft(x)
    assert X.shape == (B, n // 2 + 1)
    assert_close(_cplx(X.cpu().numpy()), _cplx(ref), TOL, "rfft n=%d B=%d" % (n, B))
    # the inverse on the oracle's spectrum (rounded to complex64), and the round trip
    S = torch.from_numpy(ref.astype(np.complex64)).to(DEV)
    y = tfx.irfft(S, n)
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), F.irfft(ref.astype(np.complex64), n), TOL, "irfft n=%d B=%d" % (n, B))
    rt = tfx.irfft(X, n)
    torch.cuda.synchronize()
    assert_close(rt.cpu().numpy(), x, TOL, "round trip n=%d" % n)


@pytest.mark.parametrize("n", [16, 1024])
def test_rfft_strided_rows_and_batch_dims(n):
    B = 5
    x = _rows(B, n, (802, n))
    buf = torch.zeros((B, n + 24), dtype=torch.float32, device=DEV)
    buf[:, :n] = torch.from_numpy(x).to(DEV)
    X = tfx.rfft(buf[:, :n])                       # row stride n + 24: one row per channel
    torch.cuda.synchronize()
    assert_close(_cplx(X.cpu().numpy()), _cplx(F.rfft(x)), TOL, "strided rfft n=%d" % n)
    X3 = tfx.rfft(torch.from_numpy(np.stack([x, 2 * x])).to(DEV))   # [2, B, n]
    torch.cuda.synchronize()
    assert X3.shape == (2, B, n // 2 + 1)
    assert_close(_cplx(X3[1].cpu().numpy()), _cplx(2 * F.rfft(x)), TOL, "batched dims n=%d" % n)


def test_irfft_ignores_imaginary_parts_of_end_bins():
    n = 256
    g = np.random.default_rng(803)
    S = (g.standard_normal((3, n // 2 + 1)) + 1j * g.standard_normal((3, n // 2 + 1))).astype(np.complex64)
    y = tfx.irfft(torch.from_numpy(S).to(DEV), n)
    torch.cuda.synchronize()
    assert_close(y.cpu().numpy(), F.irfft(S, n), TOL, "end-bin imaginary parts")


def test_fft_size_refused_and_empty_batch():
    with pytest.raises(lib.TfxError) as ei:
        tfx.rfft(torch.zeros((2, 48), device=DEV))
    assert ei.value.status == 2
    X = tfx.rfft(torch.zeros((0, 64), device=DEV))
    assert X.shape == (0, 33)


def test_rfft_large_batch_sampled_rows():
    """8 x 5,760,000 samples as 11,250 rows of 4096: sampled rows against
    the oracle."""
    n = 4096
    x = torch.from_numpy(_rows(8, 5_760_000, (804,))).to(DEV).reshape(-1, n)
    X = tfx.rfft(x)
    torch.cuda.synchronize()
    picks = [0, 1, 2, 5000, 11248, 11249]
    got = X[picks].cpu().numpy()
    ref = F.rfft(x[picks].cpu().numpy())
    assert_close(_cplx(got), _cplx(ref), TOL, "rfft large batch")

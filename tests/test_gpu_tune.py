"""The FIR tuner on the GPU (tfx_fir_autotune through the C ABI): every form
it can pick matches the oracle at its stated accuracy on the tuned shape;
the pick is admissible for the tolerance; an automatic fp32 call of the
tuned shape then runs the picked form (bit-identical output); the cache file
records it; a capturing stream is refused."""
import numpy as np
import pytest
import torch

import paper_2504_08624_amd as tfx
from paper_2504_08624_amd import lib, signals
from oracle import oracle as O
from tests.metrics import assert_close

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
STATED = {("direct", "f32"): 1e-5, ("fft", "f32"): 1e-5, ("fft16k", "f32"): 1e-5, ("toeplitz", "bf16x3"): 1e-4,
          ("toeplitz", "f16"): 1e-2, ("toeplitz", "bf16"): 1e-2}


def _x(C, N, key, sigma=0.1):
    return signals.to_f32(np.stack([signals.white(N, (*key, c), sigma) for c in range(C)]).reshape(C, N))


@pytest.mark.parametrize("M", [31, 1023, 4000])
def test_every_candidate_form_matches_the_oracle(M):
    C, N = 3, 40_000
    x = _x(C, N, (701, M))
    h = (np.random.default_rng(M + 701).standard_normal(M) / np.sqrt(M)).astype(np.float32)
    ref = O.fir(x, h)
    xg, hg = torch.from_numpy(x).to(DEV), torch.from_numpy(h).to(DEV)
    for (algo, comp), tol in STATED.items():
        if algo == "fft16k" and M > 8193:
            continue
        y = tfx.fir(xg, hg, compute=comp, algo=algo)
        torch.cuda.synchronize()
        assert_close(y.cpu().numpy(), ref, tol, "M=%d %s/%s" % (M, algo, comp))


@pytest.mark.parametrize("tol", [1e-5, 1e-4, 1e-2])
def test_autotune_pick_is_admissible_and_used(tol, tmp_path):
    C, N, M = 4, 3 * 8192 + 100, 2047
    x = torch.from_numpy(_x(C, N, (702,))).to(DEV)
    h = torch.from_numpy((np.random.default_rng(702).standard_normal(M) / np.sqrt(M)).astype(np.float32)).to(DEV)
    path = tmp_path / "tune.txt"
    tfx.set_tuning_cache(path)
    try:
        algo, comp, ms = tfx.fir_autotune(x, h, tol=tol, reps=2)
    finally:
        tfx.set_tuning_cache(None)
    print("tol %g: picked %s/%s, %.3f ms" % (tol, algo, comp, ms), flush=True)
    assert STATED[(algo, comp)] <= tol and ms > 0
    assert tfx.fir_tuned(C, N, M, tol) == (algo, comp)
    text = path.read_text()
    assert (" %d %d " % (M, C)) in text and "gfx950" in text
    if comp == "f32":  # an automatic fp32 call of this shape now runs the picked form
        assert torch.equal(tfx.fir(x, h), tfx.fir(x, h, algo=algo))


def test_autotune_refuses_capture():
    C, N, M = 2, 10_000, 300
    x = torch.from_numpy(_x(C, N, (703,))).to(DEV)
    h = torch.ones(M, device=DEV) / M
    y = torch.empty_like(x)
    nb = lib.size_out()
    lib.call("tfx_fir_autotune_workspace_size", C, N, M, 1e-5, nb)
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=DEV)
    a, c, ms = lib.ctypes.c_int32(0), lib.ctypes.c_int32(0), lib.ctypes.c_float(0)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    z = torch.zeros(4, device=DEV)
    with torch.cuda.graph(g, stream=s):
        z.add_(1.0)
        st = lib.load().tfx_fir_autotune(x.data_ptr(), y.data_ptr(), C, N, N, N, h.data_ptr(), M, 1e-5, 1,
                                         ws.data_ptr(), nb.value, s.cuda_stream, a, c, ms)
    assert lib.STATUS_NAMES[st] == "TFX_E_CAPTURE"
    g.replay()
    torch.cuda.synchronize()
    assert float(z[0]) == 1.0

"""tfx_chain_noalloc: tfx_chain on the library's own device scratch array.

The GPU test calls the no-allocation entry point through the C ABI twice in a
row (the second call with fewer channels and samples, so the array holds the
first call's contents when the second starts) and compares each output with
tfx_chain's on a caller-owned workspace and with the FP64 oracle, at the
chain tolerance (per-channel relative RMS 1e-4).  The host test checks that a
call whose workspace exceeds the array is refused before anything runs.
"""
import ctypes

import numpy as np
import pytest

from paper_2504_08624_amd import lib, workloads
from oracle import oracle as O
from tests.metrics import TOL_IIR_F32, assert_close

SCRATCH = 16 << 20


def _status_of(L, name, *args):
    return getattr(L, name)(*args)


def test_noalloc_refuses_oversize_workspace():
    L = lib.load()
    # 64 channels x 2^27 samples x 8 sections: look-back records alone need
    # far more than the scratch array; refused on the host (no device call)
    arr = lib.stage_array([(lib.STAGE_SOS, 8, 256)])
    nb = lib.size_out()
    lib.call("tfx_chain_workspace_size", 64, 1 << 27, arr, 1, 0, nb)
    assert nb.value > SCRATCH
    st = L.tfx_chain_noalloc(256, 512, 64, 1 << 27, 1 << 27, 1 << 27, arr, 1, 0, None, None, None)
    assert st == 3, st  # TFX_E_WORKSPACE
    assert b"scratch" in L.tfx_last_error()


@pytest.mark.gpu
def test_noalloc_matches_tfx_chain_twice():
    import torch
    from paper_2504_08624_amd import functional as F

    dev = torch.device("cuda:0")
    L = lib.load()
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    for C, N in [(5, 9 * 3072 + 5), (2, 4001)]:
        print("tfx_chain_noalloc: chain_mid filters (1023-tap FIR | 6 SOS), C=%d N=%d" % (C, N), flush=True)
        w = workloads.chain_mid(C=C, N=N)
        x = torch.from_numpy(w.x).to(dev)
        kept, desc = F._stages(w.stages, dev)
        arr = lib.stage_array(desc)
        need = lib.size_out()
        lib.call("tfx_chain_workspace_size", C, N, arr, len(desc), 0, need)
        assert need.value <= SCRATCH
        y = torch.full_like(x, float("nan"))
        stream = torch.cuda.current_stream(dev).cuda_stream
        lib.call("tfx_chain_noalloc", x.data_ptr(), y.data_ptr(), C, N, N, N, arr, len(desc), 0, None,
                 flags.data_ptr(), stream)
        ref_gpu = F.chain(x, [(k, t) for (k, _), t in zip(w.stages, kept)])
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        other = ref_gpu.cpu().numpy()
        print("  max |noalloc - tfx_chain| = %.3e" % float(np.abs(got - other).max()), flush=True)
        assert_close(got, other.astype(np.float64), TOL_IIR_F32, "noalloc vs tfx_chain C=%d N=%d" % (C, N))
        assert_close(got, O.chain(w.x, w.stages), TOL_IIR_F32, "noalloc vs oracle C=%d N=%d" % (C, N))
        assert int(flags.item()) == 0, "scratch status word 0x%x" % int(flags.item())

"""Error metric used by every parity test.

Per-channel relative RMS error  e_c = ||y[c] - ref[c]||_2 / ||ref[c]||_2 ;
a channel whose reference is all zero is judged on its absolute RMS against
the global reference RMS.  Tolerances (FP32 FIR 1e-5, FP32 IIR and chains
1e-4, BF16/FP16 FIR 1e-2) are stated where each test uses them.
"""
import numpy as np

TOL_FIR_F32 = 1e-5
TOL_IIR_F32 = 1e-4
TOL_FIR_LOWP = 1e-2


def channel_errors(y, ref):
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    assert y.shape == ref.shape, (y.shape, ref.shape)
    grms = np.sqrt(np.mean(ref * ref)) if ref.size else 0.0
    errs = []
    for yc, rc in zip(y, ref):
        den = np.linalg.norm(rc)
        num = np.linalg.norm(yc - rc)
        if den > 0:
            errs.append(num / den)
        else:
            errs.append((num / np.sqrt(max(rc.size, 1))) / grms if grms > 0 else num)
    return np.array(errs)


def assert_close(y, ref, tol, what=""):
    e = channel_errors(y, ref)
    assert np.all(np.isfinite(e)) and e.max() <= tol, "%s: max per-channel rel err %.3e > %.1e" % (
        what, e.max() if e.size else 0.0, tol)
    return float(e.max()) if e.size else 0.0

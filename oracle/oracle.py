"""FP64 CPU oracle for the FIR / IIR-SOS filter chain.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module.  The GPU library and its
Python binding never import it, and this module imports nothing from them.

The arithmetic lives in ``tfx_oracle.c`` (plain double-precision loops, one
channel at a time, the textbook definitions the paper's Sec. 3 names: causal
FIR convolution and the coefficient-driven recursive filter in transposed
direct form II, stages applied in pipe order).  This module loads it with
ctypes, promotes inputs exactly to float64, and composes stages into chains in
the order written (Sec. 3, the pipe example).

Conventions shared with the GPU path (they are the interface, not code):
  * signals are row-major [C, N];
  * an SOS stage is an [S, 5] array of rows [b0, b1, b2, a1, a2] (a0 == 1);
  * SOS state is [C, S, 2] = the two TDF-II delay registers (s1, s2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tfx_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64


def build(force: bool = False) -> str:
    """Compile tfx_oracle.c with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_fir.argtypes = [_dp, _dp, _i64, _i64, _dp, _i64]
            lib.oracle_fir_at.argtypes = [_dp, _i64, _i64, _dp, _i64, _i64p, _i64, _dp]
            lib.oracle_sos.argtypes = [_dp, _dp, _i64, _i64, _dp, _i64, _dp, _dp]
            lib.oracle_fir_backward.argtypes = [_dp, _dp, _dp, _i64, _i64, _i64, _dp, _dp]
            lib.oracle_sos_backward.argtypes = [_dp, _dp, _dp, _i64, _i64, _i64, _dp, _dp]
            for f in ("oracle_fir", "oracle_fir_at", "oracle_sos",
                      "oracle_fir_backward", "oracle_sos_backward"):
                getattr(lib, f).restype = None
            lib.oracle_last_seconds.restype = ctypes.c_double
            lib.oracle_last_seconds.argtypes = []
            lib.oracle_threads.restype = ctypes.c_int
            lib.oracle_threads.argtypes = []
            _lib = lib
    return _lib


def last_seconds() -> float:
    """Steady-clock seconds of the filtering loops of the last fir / fir_at /
    sos call (C side, excluding the float64 promotion)."""
    return float(_load().oracle_last_seconds())


def threads() -> int:
    """Threads the oracle's loops over channels may use."""
    return int(_load().oracle_threads())


def _d(a) -> np.ndarray:
    """Exact promotion to a C-contiguous float64 array."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _as2d(x):
    x = _d(x)
    if x.ndim == 1:
        return x[None, :], True
    if x.ndim != 2:
        raise ValueError("signal must be [N] or [C, N]")
    return x, False


def fir(x, h) -> np.ndarray:
    """y[c, n] = sum_{k<=min(M-1, n)} h[k] x[c, n-k]."""
    x2, squeeze = _as2d(x)
    h = _d(h).ravel()
    if h.size < 1:
        raise ValueError("FIR needs at least one tap")
    C, N = x2.shape
    y = np.empty_like(x2)
    if N:
        _load().oracle_fir(_p(x2), _p(y), C, N, _p(h), h.size)
    return y[0] if squeeze else y


def fir_at(x, h, positions) -> np.ndarray:
    """FIR outputs y[c, positions[p]] only; returns [C, P]."""
    x2, _ = _as2d(x)
    h = _d(h).ravel()
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.int64))
    C, N = x2.shape
    if pos.size and (pos.min() < 0 or pos.max() >= N):
        raise ValueError("position out of range")
    out = np.empty((C, pos.size), dtype=np.float64)
    if pos.size:
        _load().oracle_fir_at(_p(x2), C, N, _p(h), h.size,
                              pos.ctypes.data_as(_i64p), pos.size, _p(out))
    return out


def sos(x, coeffs, state_in=None, return_state=False):
    """Cascade of TDF-II sections, rows [b0 b1 b2 a1 a2], in array order."""
    x2, squeeze = _as2d(x)
    co = _d(coeffs).reshape(-1, 5)
    S = co.shape[0]
    C, N = x2.shape
    y = np.empty_like(x2)
    si = None
    if state_in is not None:
        si = _d(state_in).reshape(C, S, 2)
    so = np.zeros((C, S, 2), dtype=np.float64)
    if S == 0:
        y[...] = x2
        if si is not None:
            so[...] = si
    else:
        _load().oracle_sos(_p(x2), _p(y), C, N, _p(co), S,
                           _p(si) if si is not None else None, _p(so))
    y = y[0] if squeeze else y
    if return_state:
        return y, (so[0] if squeeze else so)
    return y


def chain(x, stages):
    """Apply stages left to right (pipe order).  stages: list of
    ("fir", taps) or ("sos", [S, 5] rows)."""
    y, squeeze = _as2d(x)
    for kind, coef in stages:
        if kind == "fir":
            y = fir(y, coef)
        elif kind == "sos":
            y = sos(y, coef)
        else:
            raise ValueError("unknown stage kind %r" % (kind,))
    return y[0] if squeeze else y


def fir_backward(g, x, h):
    """Returns (gx [C, N], gh [M]) of the FIR for upstream gradient g."""
    g2, squeeze = _as2d(g)
    x2, _ = _as2d(x)
    h = _d(h).ravel()
    C, N = g2.shape
    gx = np.zeros_like(g2)
    gh = np.zeros(h.size, dtype=np.float64)
    if N:
        _load().oracle_fir_backward(_p(g2), _p(x2), _p(h), h.size, C, N, _p(gx), _p(gh))
    return (gx[0] if squeeze else gx), gh


def sos_backward(g, x, coeffs):
    """Returns (gx [C, N], gsos [S, 5]) of the cascade (zero initial state)."""
    g2, squeeze = _as2d(g)
    x2, _ = _as2d(x)
    co = _d(coeffs).reshape(-1, 5)
    S = co.shape[0]
    C, N = g2.shape
    gx = np.array(g2, copy=True)
    gs = np.zeros((S, 5), dtype=np.float64)
    if N and S:
        _load().oracle_sos_backward(_p(g2), _p(x2), _p(co), S, C, N, _p(gx), _p(gs))
    return (gx[0] if squeeze else gx), gs


def chain_backward(g, x, stages):
    """Adjoint of chain(): returns (gx, [grad of each stage's coefficients]).
    The forward signals are recomputed stage by stage and kept."""
    x2, squeeze = _as2d(x)
    inputs = [x2]
    for kind, coef in stages:
        inputs.append(chain(inputs[-1], [(kind, coef)]))
    gcur, _ = _as2d(g)
    grads = [None] * len(stages)
    for i in range(len(stages) - 1, -1, -1):
        kind, coef = stages[i]
        if kind == "fir":
            gcur, grads[i] = fir_backward(gcur, inputs[i], coef)
        else:
            gcur, grads[i] = sos_backward(gcur, inputs[i], coef)
    return (gcur[0] if squeeze else gcur), grads


def sos_batched(clips):
    """Ragged batch: clips is a list of (x [C_i, N_i], sos_i [S_i, 5]);
    each clip is filtered by its own cascade.  Returns a list of outputs."""
    return [sos(x, co) for x, co in clips]

"""Torch-facing entry points: fir, sos, chain and their adjoints.

PyTorch supplies device memory (``torch.empty``) and the current HIP stream;
the filtering runs in libtfx.so through the C ABI (``lib.py``).  Inputs must
be float32 HIP tensors shaped [N] or [C, N]; there is no CPU path.

When autograd is recording and the signal or a coefficient tensor requires a
gradient, the calls go through ``torch.autograd.Function`` wrappers whose
backward runs the library's adjoint kernels (the forward keeps only the
tile-boundary checkpoints of the IIR states, not per-sample signals).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import design, lib


def _signal(x: torch.Tensor):
    if not isinstance(x, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if x.device.type != "cuda":
        raise TypeError("tfx runs on the GPU only; got a tensor on %s" % x.device)
    if x.dtype != torch.float32:
        raise TypeError("tfx signals are float32, got %s" % x.dtype)
    squeeze = x.dim() == 1
    x2 = x.unsqueeze(0) if squeeze else x
    if x2.dim() != 2:
        raise ValueError("signal must be [N] or [C, N]")
    C, N = x2.shape
    if x2.stride(1) != 1 or (C > 1 and x2.stride(0) < N):
        x2 = x2.contiguous()
    ld = x2.stride(0) if C > 1 else max(N, 1)
    return x2, squeeze, ld


def _coef(c, device) -> torch.Tensor:
    t = torch.as_tensor(c, dtype=torch.float32)
    return t.to(device).contiguous()


def _stream(device):
    return ctypes_ptr(torch.cuda.current_stream(device).cuda_stream)


def ctypes_ptr(v):
    return int(v) if v else None


def _workspace(nbytes: int, device):
    if nbytes <= 0:
        return None, 0
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
    return ws, int(nbytes)


# One device-side status word per device.  After every call that used a
# workspace, the workspace's status word (set by a kernel whose look-back wait
# gave up) is folded into it by tfx_workspace_status on the same stream, so
# nothing synchronises; device_status() reads it.
_status_words = {}


def _status_word(device) -> torch.Tensor:
    device = torch.device(device)
    key = device.index if device.index is not None else torch.cuda.current_device()
    w = _status_words.get(key)
    if w is None:
        w = torch.zeros(1, dtype=torch.int32, device=torch.device("cuda", key))
        _status_words[key] = w
    return w


def _track(ws, wsb: int, device):
    if ws is None or wsb < 256:
        return
    lib.call("tfx_workspace_status", _ptr(ws), wsb, _status_word(device).data_ptr(), 1, _stream(device))


def device_status(device=None, clear: bool = True) -> int:
    """Synchronises the device and returns the OR of the status words of
    every workspace used by the calls of this module since the last clear
    (0 = clean; lib.DEV_LOOKBACK_TIMEOUT = a look-back wait gave up, so the
    output of some call is wrong)."""
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    w = _status_word(device)
    torch.cuda.synchronize(device)
    v = int(w.item())
    if clear and v:
        w.zero_()
    return v


def check_device_status(device=None):
    """Raises lib.TfxError(TFX_E_DEVICE) if a kernel flagged a workspace
    since the last check (clears the flag)."""
    v = device_status(device, clear=True)
    if v:
        raise lib.TfxError(lib.TFX_E_DEVICE, "device status",
                           "workspace status word 0x%x (look-back wait gave up: some output is wrong)" % v)


def _ptr(t):
    return t.data_ptr() if t is not None else None


def tile_length() -> int:
    return int(lib.load().tfx_sos_tile_length())


def _fir_raw(x: torch.Tensor, h, compute: str = "f32", algo: str = "auto") -> torch.Tensor:
    x2, squeeze, ld = _signal(x)
    C, N = x2.shape
    h = _coef(h, x.device).reshape(-1)
    y = torch.empty((C, N), dtype=torch.float32, device=x.device)
    nb = lib.size_out()
    lib.call("tfx_fir_workspace_size", C, N, h.numel(), lib.COMPUTE[compute], lib.FIR_ALGO[algo], nb)
    ws, wsb = _workspace(nb.value, x.device)
    lib.call("tfx_fir", _ptr(x2), _ptr(y), C, N, ld, max(N, 1), _ptr(h), h.numel(),
             lib.COMPUTE[compute], lib.FIR_ALGO[algo], _ptr(ws), wsb, _stream(x.device))
    _track(ws, wsb, x.device)
    return y[0] if squeeze else y


_ALGO_NAMES = {v: k for k, v in lib.FIR_ALGO.items()}
_COMPUTE_NAMES = {v: k for k, v in lib.COMPUTE.items()}


def fir_autotune(x: torch.Tensor, h, tol: float = 1e-5, reps: int = 3):
    """Times every FIR form whose stated accuracy is within ``tol`` on this
    signal and these taps (tfx_fir_autotune) and returns (algo, compute, ms)
    of the fastest; an fp32 ``fir(x, h)`` of this shape then uses it.
    Synchronises the device."""
    x2, squeeze, ld = _signal(x)
    C, N = x2.shape
    h = _coef(h, x.device).reshape(-1)
    y = torch.empty((C, N), dtype=torch.float32, device=x.device)
    nb = lib.size_out()
    lib.call("tfx_fir_autotune_workspace_size", C, N, h.numel(), float(tol), nb)
    ws, wsb = _workspace(nb.value, x.device)
    a, c, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0.0)
    lib.call("tfx_fir_autotune", _ptr(x2), _ptr(y), C, N, ld, max(N, 1), _ptr(h), h.numel(), float(tol), int(reps),
             _ptr(ws), wsb, _stream(x.device), a, c, ms)
    _track(ws, wsb, x.device)
    return _ALGO_NAMES[a.value], _COMPUTE_NAMES[c.value], float(ms.value)


def set_tuning_cache(path):
    """Makes the FIR tuning cache persistent in a text file (None: memory only)."""
    lib.call("tfx_set_tuning_cache", None if path is None else str(path).encode())


def fir_tuned(C: int, N: int, M: int, tol: float = 1e-5):
    """(algo, compute) recorded by fir_autotune for this shape, or ("auto", "f32")."""
    a, c = ctypes.c_int32(0), ctypes.c_int32(0)
    lib.call("tfx_fir_tuned", int(C), int(N), int(M), float(tol), a, c)
    return _ALGO_NAMES[a.value], _COMPUTE_NAMES[c.value]


def _sos_raw(x: torch.Tensor, sections, state_in=None, return_state: bool = False,
             return_ckpt: bool = False):
    x2, squeeze, ld = _signal(x)
    C, N = x2.shape
    co = _coef(sections, x.device).reshape(-1, 5)
    S = co.shape[0]
    y = torch.empty((C, N), dtype=torch.float32, device=x.device)
    si = None
    if state_in is not None:
        si = _coef(state_in, x.device).reshape(C, S, 2)
    so = torch.empty((C, S, 2), dtype=torch.float32, device=x.device) if return_state else None
    ck = None
    if return_ckpt:
        nt = (N + tile_length() - 1) // tile_length()
        ck = torch.empty((C, nt, S, 2), dtype=torch.float32, device=x.device)
    nb = lib.size_out()
    lib.call("tfx_sos_workspace_size", C, N, S, nb)
    ws, wsb = _workspace(nb.value, x.device)
    lib.call("tfx_sos", _ptr(x2), _ptr(y), C, N, ld, max(N, 1), _ptr(co), S, _ptr(si), _ptr(so),
             _ptr(ck), _ptr(ws), wsb, _stream(x.device))
    _track(ws, wsb, x.device)
    y = y[0] if squeeze else y
    out = [y]
    if return_state:
        out.append(so[0] if squeeze else so)
    if return_ckpt:
        out.append(ck)
    return out[0] if len(out) == 1 else tuple(out)


def _stages(stages, device):
    kept, desc = [], []
    for kind, coef in stages:
        if kind == "fir":
            t = _coef(coef, device).reshape(-1)
            desc.append((lib.STAGE_FIR, t.numel(), t.data_ptr()))
        elif kind == "sos":
            t = _coef(coef, device).reshape(-1, 5)
            desc.append((lib.STAGE_SOS, t.shape[0], t.data_ptr()))
        else:
            raise ValueError("unknown stage kind %r" % (kind,))
        kept.append(t)
    return kept, desc


def _chain_raw(x: torch.Tensor, stages, compute: str = "f32", return_ckpt: bool = False):
    x2, squeeze, ld = _signal(x)
    C, N = x2.shape
    kept, desc = _stages(stages, x.device)
    arr = lib.stage_array(desc)
    S = sum(n for k, n, _ in desc if k == lib.STAGE_SOS)
    y = torch.empty((C, N), dtype=torch.float32, device=x.device)
    ck = None
    if return_ckpt:
        nt = (N + tile_length() - 1) // tile_length()
        ck = torch.empty((C, nt, S, 2), dtype=torch.float32, device=x.device)
    nb = lib.size_out()
    lib.call("tfx_chain_workspace_size", C, N, arr, len(desc), lib.COMPUTE[compute], nb)
    ws, wsb = _workspace(nb.value, x.device)
    lib.call("tfx_chain", _ptr(x2), _ptr(y), C, N, ld, max(N, 1), arr, len(desc),
             lib.COMPUTE[compute], _ptr(ck), _ptr(ws), wsb, _stream(x.device))
    _track(ws, wsb, x.device)
    del kept
    y = y[0] if squeeze else y
    return (y, ck) if return_ckpt else y


# ------------------------------------------------------------------ adjoint

def fir_backward(x: torch.Tensor, gy: torch.Tensor, h, compute: str = "f32", algo: str = "auto",
                 need_taps: bool = True):
    """(dL/dx, dL/dh) of y = fir(x, h) given gy = dL/dy."""
    x2, squeeze, ld = _signal(x)
    g2, _, ldg = _signal(gy)
    C, N = x2.shape
    if tuple(g2.shape) != (C, N):
        raise ValueError("gy must have the shape of x")
    h = _coef(h, x.device).reshape(-1)
    gx = torch.empty((C, N), dtype=torch.float32, device=x.device)
    gh = torch.empty_like(h) if need_taps else None
    nb = lib.size_out()
    lib.call("tfx_fir_backward_workspace_size", C, N, h.numel(), lib.COMPUTE[compute], lib.FIR_ALGO[algo], nb)
    ws, wsb = _workspace(nb.value, x.device)
    lib.call("tfx_fir_backward", _ptr(x2), _ptr(g2), _ptr(gx), C, N, ld, ldg, max(N, 1), _ptr(h), h.numel(),
             _ptr(gh), lib.COMPUTE[compute], lib.FIR_ALGO[algo], _ptr(ws), wsb, _stream(x.device))
    _track(ws, wsb, x.device)
    return (gx[0] if squeeze else gx), gh


def sos_backward(x: torch.Tensor, gy: torch.Tensor, sections, ckpt: torch.Tensor, need_coef: bool = True):
    """(dL/dx, dL/dsections) of y = sos(x, sections, state_in) given gy and
    the forward's checkpoints (``sos(..., return_ckpt=True)``)."""
    x2, squeeze, ld = _signal(x)
    g2, _, ldg = _signal(gy)
    C, N = x2.shape
    if tuple(g2.shape) != (C, N):
        raise ValueError("gy must have the shape of x")
    co = _coef(sections, x.device).reshape(-1, 5)
    S = co.shape[0]
    gx = torch.empty((C, N), dtype=torch.float32, device=x.device)
    gs = torch.empty_like(co) if need_coef else None
    ck = ckpt.contiguous() if ckpt is not None else None
    nb = lib.size_out()
    lib.call("tfx_sos_backward_workspace_size", C, N, S, nb)
    ws, wsb = _workspace(nb.value, x.device)
    lib.call("tfx_sos_backward", _ptr(x2), _ptr(g2), _ptr(gx), C, N, ld, ldg, max(N, 1), _ptr(co), S, _ptr(ck),
             _ptr(gs), _ptr(ws), wsb, _stream(x.device))
    _track(ws, wsb, x.device)
    return (gx[0] if squeeze else gx), gs


def chain_backward(x: torch.Tensor, gy: torch.Tensor, stages, ckpt, compute: str = "f32",
                   need_coef: bool = True):
    """(dL/dx, [dL/dcoef of every stage]) of y = chain(x, stages) given gy
    and the forward's checkpoints (``chain(..., return_ckpt=True)``; None when
    the chain has no SOS stage)."""
    x2, squeeze, ld = _signal(x)
    g2, _, ldg = _signal(gy)
    C, N = x2.shape
    if tuple(g2.shape) != (C, N):
        raise ValueError("gy must have the shape of x")
    kept, desc = _stages(stages, x.device)
    arr = lib.stage_array(desc)
    gx = torch.empty((C, N), dtype=torch.float32, device=x.device)
    grads = [torch.empty_like(t) for t in kept] if need_coef else [None] * len(kept)
    parr = lib.pointer_array([_ptr(g) for g in grads])
    ck = ckpt.contiguous() if ckpt is not None else None
    nb = lib.size_out()
    lib.call("tfx_chain_backward_workspace_size", C, N, arr, len(desc), lib.COMPUTE[compute], nb)
    ws, wsb = _workspace(nb.value, x.device)
    lib.call("tfx_chain_backward", _ptr(x2), _ptr(g2), _ptr(gx), C, N, ld, ldg, max(N, 1), arr, len(desc),
             lib.COMPUTE[compute], _ptr(ck), parr, _ptr(ws), wsb, _stream(x.device))
    _track(ws, wsb, x.device)
    del kept
    return (gx[0] if squeeze else gx), grads


class ChainStream:
    """Block-by-block filtering of a stream with a fixed chain: every call to
    ``process`` filters the next block as the continuation of the previous
    ones (FIR input history and cascade registers carried on the device).
    The device tables are prepared once for blocks of up to ``max_block``
    samples; each block is then one ``tfx_chain_stream`` call."""

    def __init__(self, stages, channels: int, max_block: int, compute: str = "f32", device="cuda:0"):
        self.device = torch.device(device)
        self.C, self.n_max, self.compute = int(channels), int(max_block), compute
        self._kept, desc = _stages(stages, self.device)
        self._arr = lib.stage_array(desc)
        self._ns = len(desc)
        firs = [n for k, n, _ in desc if k == lib.STAGE_FIR]
        self.M = (firs[0] + sum(n - 1 for n in firs[1:])) if firs else 0
        self.S = sum(n for k, n, _ in desc if k == lib.STAGE_SOS)
        nb = lib.size_out()
        lib.call("tfx_chain_workspace_size", self.C, self.n_max, self._arr, self._ns, lib.COMPUTE[compute], nb)
        self._ws, self._wsb = _workspace(nb.value, self.device)
        lib.call("tfx_chain_prepare", self.C, self.n_max, self._arr, self._ns, lib.COMPUTE[compute],
                 _ptr(self._ws), self._wsb, _stream(self.device))
        H = max(self.M - 1, 0)
        self._hist = [torch.zeros((self.C, H), dtype=torch.float32, device=self.device) for _ in range(2)]
        self._state = [torch.zeros((self.C, self.S, 2), dtype=torch.float32, device=self.device) for _ in range(2)]
        self._cur = 0

    def reset(self):
        """Start of a new stream: zero history and registers."""
        for t in self._hist + self._state:
            t.zero_()

    def process(self, x: torch.Tensor) -> torch.Tensor:
        x2, squeeze, ld = _signal(x)
        C, N = x2.shape
        if C != self.C:
            raise ValueError("the stream has %d channels" % self.C)
        y = torch.empty((C, N), dtype=torch.float32, device=x.device)
        i, o = self._cur, 1 - self._cur
        lib.call("tfx_chain_stream", _ptr(x2), _ptr(y), C, N, ld, max(N, 1), self._arr, self._ns,
                 lib.COMPUTE[self.compute], self.n_max, _ptr(self._hist[i]), _ptr(self._hist[o]),
                 _ptr(self._state[i]), _ptr(self._state[o]), _ptr(self._ws), self._wsb, _stream(x.device))
        _track(self._ws, self._wsb, x.device)
        self._cur = o
        return y[0] if squeeze else y


class _ChainFn(torch.autograd.Function):
    """y = chain(x, stages) with the library's adjoint as backward."""

    @staticmethod
    def forward(ctx, kinds, compute, x, *coefs):
        stages = list(zip(kinds, coefs))
        has_sos = any(k == "sos" for k in kinds)
        if has_sos:
            y, ck = _chain_raw(x, stages, compute, return_ckpt=True)
        else:
            y, ck = _chain_raw(x, stages, compute), None
        ctx.kinds, ctx.compute = kinds, compute
        ctx.save_for_backward(x, ck if ck is not None else torch.empty(0, device=x.device), *coefs)
        ctx.has_ck = ck is not None
        return y

    @staticmethod
    def backward(ctx, gy):
        x, ck, *coefs = ctx.saved_tensors
        need_coef = any(ctx.needs_input_grad[3:])
        gx, grads = chain_backward(x, gy.contiguous(), list(zip(ctx.kinds, coefs)), ck if ctx.has_ck else None,
                                   ctx.compute, need_coef)
        out = [None, None, gx if ctx.needs_input_grad[2] else None]
        for c, g, need in zip(coefs, grads, ctx.needs_input_grad[3:]):
            out.append(g.reshape(c.shape) if (need and g is not None) else None)
        return tuple(out)


def _wants_grad(x, coefs):
    if not torch.is_grad_enabled():
        return False
    return bool(getattr(x, "requires_grad", False)) or any(
        isinstance(c, torch.Tensor) and c.requires_grad for c in coefs)


def _as_param(c, device, shape_fn):
    if isinstance(c, torch.Tensor) and c.requires_grad:
        if c.dtype != torch.float32 or c.device != device:
            raise TypeError("trainable coefficients must be float32 tensors on the signal's device")
        return c
    return shape_fn(_coef(c, device))


def chain(x: torch.Tensor, stages, compute: str = "f32", return_ckpt: bool = False):
    """Apply ("fir", taps) / ("sos", sections) stages left to right in one
    fused launch (all FIR stages merged and applied first, all sections
    concatenated behind them).  Differentiable in x and every coefficient
    tensor when autograd records (``return_ckpt`` is then not available)."""
    coefs = [c for _, c in stages]
    if _wants_grad(x, coefs):
        if return_ckpt:
            raise ValueError("return_ckpt is for explicit adjoint calls, not autograd")
        if compute != "f32" and any(k == "fir" for k, _ in stages):
            # refused before the forward runs, not at loss.backward()
            raise ValueError("the adjoint computes in fp32 only: a differentiable chain with a FIR stage needs "
                             "compute='f32' (got %r)" % (compute,))
        kinds = tuple(k for k, _ in stages)
        for k in kinds:
            if k not in ("fir", "sos"):
                raise ValueError("unknown stage kind %r" % (k,))
        ts = [_as_param(c, x.device, (lambda t: t.reshape(-1)) if k == "fir" else (lambda t: t.reshape(-1, 5)))
              for k, c in stages]
        return _ChainFn.apply(kinds, compute, x, *ts)
    return _chain_raw(x, stages, compute, return_ckpt)


def fir(x: torch.Tensor, h, compute: str = "f32", algo: str = "auto") -> torch.Tensor:
    """y[c, n] = sum_k h[k] x[c, n-k] (causal, zero history, same length).
    Differentiable in x and h when autograd records."""
    if _wants_grad(x, [h]):
        if algo not in ("auto",):
            raise ValueError("the differentiable FIR uses the automatic algorithm choice")
        return chain(x, [("fir", h)], compute)
    return _fir_raw(x, h, compute, algo)


def sos(x: torch.Tensor, sections, state_in=None, return_state: bool = False,
        return_ckpt: bool = False):
    """Cascade of second-order sections, rows [b0 b1 b2 a1 a2] (a0 == 1).

    state_in: optional [C, S, 2] TDF-II registers.  Returns y, plus the final
    state [C, S, 2] if ``return_state`` and the tile checkpoints
    [C, ceil(N/T), S, 2] if ``return_ckpt``.  Differentiable in x and the
    sections (zero initial state) when autograd records."""
    if _wants_grad(x, [sections]):
        if state_in is not None or return_state or return_ckpt:
            raise ValueError("the differentiable SOS takes no state and returns only y")
        return chain(x, [("sos", sections)])
    return _sos_raw(x, sections, state_in, return_state, return_ckpt)


def lfilter(x: torch.Tensor, b, a, compute: str = "f32") -> torch.Tensor:
    """Direct-form IIR y = (b(z^-1) / a(z^-1)) x, zero initial state.  The
    polynomials are factored into second-order sections in FP64 on the host
    (roots paired nearest-zero-to-pole) and run as one fused chain; a
    denominator of length 1 is a plain FIR.  An unstable denominator (a pole
    on or outside the unit circle) is an error.  Differentiable in x."""
    bb = np.atleast_1d(np.asarray(b, dtype=np.float64))
    aa = np.trim_zeros(np.atleast_1d(np.asarray(a, dtype=np.float64)), "b")
    if aa.size == 0 or aa[0] == 0.0:
        raise ValueError("a[0] must be nonzero")
    if aa.size == 1:
        return chain(x, [("fir", (bb / aa[0]).astype(np.float32))], compute)
    rows = design.tf2sos(bb, aa)
    if design.max_pole_radius(rows) >= 1.0:
        raise ValueError("the denominator has a pole on or outside the unit circle")
    return chain(x, [("sos", rows.astype(np.float32))], compute)


# ------------------------------------------------------------------ batched

class SosBatch:
    """A ragged batch of clips, each [C_i, N_i] with its own cascade [S_i, 5],
    filtered by one kernel launch.

    ``SosBatch(xs, sections)`` allocates the outputs and the workspace and
    prepares the batch (descriptor table and section tables on the device);
    ``run()`` then filters every clip with one launch on the current stream
    and may be captured in a CUDA/HIP graph; ``tune()`` times every launch
    configuration on this batch and keeps the fastest.  The inputs, the
    coefficient tensors and the outputs stay owned by this object."""

    def __init__(self, xs, sections, config=None):
        if len(xs) != len(sections):
            raise ValueError("one cascade per clip")
        self.device = xs[0].device if xs else torch.device("cuda", torch.cuda.current_device())
        self.xs, self.lds, self.secs, self.ys = [], [], [], []
        for x, sec in zip(xs, sections):
            x2, _, ld = _signal(x)
            self.xs.append(x2)
            self.lds.append(ld)
            self.secs.append(_coef(sec, self.device).reshape(-1, 5))
            self.ys.append(torch.empty(x2.shape, dtype=torch.float32, device=self.device))
        n = len(self.xs)
        self.clips = (lib.Clip * max(1, n))()
        for i, (x2, ld, sec, y) in enumerate(zip(self.xs, self.lds, self.secs, self.ys)):
            c = self.clips[i]
            c.x, c.y = _ptr(x2), _ptr(y)
            c.C, c.N = x2.shape
            c.ldx, c.ldy = ld, max(x2.shape[1], 1)
            c.sos, c.S, c.reserved = _ptr(sec), sec.shape[0], 0
        self.n = n
        nb = lib.size_out()
        lib.call("tfx_sos_batched_workspace_size", self.clips, n, nb)
        self.ws, self.wsb = _workspace(nb.value, self.device)
        self.config = lib.BatchConfig(0, 0)
        if config:
            self.config.chunk, self.config.order = int(config.get("chunk", 0)), int(config.get("order", 0))
        self.prepare()

    def prepare(self):
        lib.call("tfx_sos_batched_prepare", self.clips, self.n, self.config, _ptr(self.ws), self.wsb,
                 _stream(self.device))

    def run(self):
        lib.call("tfx_sos_batched_run", self.clips, self.n, self.config, _ptr(self.ws), self.wsb,
                 _stream(self.device))
        _track(self.ws, self.wsb, self.device)
        return self.ys

    def tune(self, reps: int = 3):
        best, ms = lib.BatchConfig(0, 0), ctypes.c_float(0.0)
        lib.call("tfx_sos_batched_tune", self.clips, self.n, reps, _ptr(self.ws), self.wsb, _stream(self.device),
                 best, ms)
        _track(self.ws, self.wsb, self.device)
        self.config = best
        return {"chunk": best.chunk, "order": best.order}, float(ms.value)


def sos_batched(xs, sections, config=None):
    """Filter clip i ([C_i, N_i]) by its own cascade sections[i] ([S_i, 5]),
    all clips in one launch; returns the list of outputs."""
    b = SosBatch(xs, sections, config)
    return b.run()

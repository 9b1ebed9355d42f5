"""Torch-facing entry points: fir, sos, chain.

PyTorch supplies device memory (``torch.empty``) and the current HIP stream;
the filtering runs in libtfx.so through the C ABI (``lib.py``).  Inputs must
be float32 HIP tensors shaped [N] or [C, N]; there is no CPU path.
"""
from __future__ import annotations

import torch

from . import lib


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


def _ptr(t):
    return t.data_ptr() if t is not None else None


def tile_length() -> int:
    return int(lib.load().tfx_sos_tile_length())


def fir(x: torch.Tensor, h, compute: str = "f32", algo: str = "auto") -> torch.Tensor:
    """y[c, n] = sum_k h[k] x[c, n-k] (causal, zero history, same length)."""
    x2, squeeze, ld = _signal(x)
    C, N = x2.shape
    h = _coef(h, x.device).reshape(-1)
    y = torch.empty((C, N), dtype=torch.float32, device=x.device)
    nb = lib.size_out()
    lib.call("tfx_fir_workspace_size", C, N, h.numel(), lib.COMPUTE[compute], lib.FIR_ALGO[algo], nb)
    ws, wsb = _workspace(nb.value, x.device)
    lib.call("tfx_fir", _ptr(x2), _ptr(y), C, N, ld, max(N, 1), _ptr(h), h.numel(),
             lib.COMPUTE[compute], lib.FIR_ALGO[algo], _ptr(ws), wsb, _stream(x.device))
    return y[0] if squeeze else y


def sos(x: torch.Tensor, sections, state_in=None, return_state: bool = False,
        return_ckpt: bool = False):
    """Cascade of second-order sections, rows [b0 b1 b2 a1 a2] (a0 == 1).

    state_in: optional [C, S, 2] TDF-II registers.  Returns y, plus the final
    state [C, S, 2] if ``return_state`` and the tile checkpoints
    [C, ceil(N/T), S, 2] if ``return_ckpt``."""
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


def chain(x: torch.Tensor, stages, compute: str = "f32", return_ckpt: bool = False):
    """Apply ("fir", taps) / ("sos", sections) stages left to right in one
    fused launch (all FIR stages merged and applied first, all sections
    concatenated behind them)."""
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
    del kept
    y = y[0] if squeeze else y
    return (y, ck) if return_ckpt else y

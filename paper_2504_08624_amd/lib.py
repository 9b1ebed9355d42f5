"""ctypes binding of libtfx.so (the C ABI declared in include/tfx.h).

Argument marshalling only: every filtering step runs in the HIP kernels of
libtfx.so.  There is no CPU fallback; if the library is missing or cannot be
loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtfx.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tfx.h")

TFX_OK = 0
STATUS_NAMES = {0: "TFX_OK", 1: "TFX_E_INVALID_ARG", 2: "TFX_E_UNSUPPORTED", 3: "TFX_E_WORKSPACE",
                4: "TFX_E_UNSTABLE", 5: "TFX_E_ALIAS", 6: "TFX_E_CAPTURE", 7: "TFX_E_HIP", 8: "TFX_E_DEVICE"}
TFX_E_DEVICE = 8
DEV_LOOKBACK_TIMEOUT = 1
COMPUTE = {"f32": 0, "bf16": 1, "f16": 2, "bf16x3": 3}
FIR_ALGO = {"auto": 0, "direct": 1, "toeplitz": 2, "fft": 3, "fft16k": 4}
STAGE_FIR, STAGE_SOS = 0, 1


class TfxError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        self.status = status
        super().__init__("%s failed: %s: %s" % (func, STATUS_NAMES.get(status, status), message))


class Clip(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("C", ctypes.c_int64), ("N", ctypes.c_int64),
                ("ldx", ctypes.c_int64), ("ldy", ctypes.c_int64), ("sos", ctypes.c_void_p), ("S", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("order", ctypes.c_int32)]


class Stage(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("len", ctypes.c_int32), ("coef", ctypes.c_void_p)]


_vp, _i64, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
_SIGS = {
    "tfx_status_string": (ctypes.c_char_p, [_i32]),
    "tfx_last_error": (ctypes.c_char_p, []),
    "tfx_version": (_i32, []),
    "tfx_sos_tile_length": (_i64, []),
    "tfx_sos_check_stable": (_i32, [_vp, _i32, ctypes.POINTER(_i32)]),
    "tfx_workspace_status": (_i32, [_vp, _sz, _vp, _i32, _vp]),
    "tfx_fir_autotune_workspace_size": (_i32, [_i64, _i64, _i32, ctypes.c_double, ctypes.POINTER(_sz)]),
    "tfx_fir_autotune": (_i32, [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _i32, ctypes.c_double, _i32, _vp, _sz, _vp,
                                ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float)]),
    "tfx_fir_tuned": (_i32, [_i64, _i64, _i32, ctypes.c_double, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "tfx_set_tuning_cache": (_i32, [ctypes.c_char_p]),
    "tfx_fir_workspace_size": (_i32, [_i64, _i64, _i32, _i32, _i32, ctypes.POINTER(_sz)]),
    "tfx_sos_workspace_size": (_i32, [_i64, _i64, _i32, ctypes.POINTER(_sz)]),
    "tfx_chain_workspace_size": (_i32, [_i64, _i64, ctypes.POINTER(Stage), _i32, _i32, ctypes.POINTER(_sz)]),
    "tfx_fir": (_i32, [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _i32, _i32, _i32, _vp, _sz, _vp]),
    "tfx_sos": (_i32, [_vp, _vp, _i64, _i64, _i64, _i64, _vp, _i32, _vp, _vp, _vp, _vp, _sz, _vp]),
    "tfx_chain": (_i32, [_vp, _vp, _i64, _i64, _i64, _i64, ctypes.POINTER(Stage), _i32, _i32, _vp, _vp, _sz,
                         _vp]),
    "tfx_chain_noalloc": (_i32, [_vp, _vp, _i64, _i64, _i64, _i64, ctypes.POINTER(Stage), _i32, _i32, _vp, _vp,
                                 _vp]),
    "tfx_chain_prepare": (_i32, [_i64, _i64, ctypes.POINTER(Stage), _i32, _i32, _vp, _sz, _vp]),
    "tfx_chain_run": (_i32, [_vp, _vp, _i64, _i64, _i64, _i64, ctypes.POINTER(Stage), _i32, _i32, _vp, _vp,
                             _sz, _vp]),
    "tfx_chain_stream": (_i32, [_vp, _vp, _i64, _i64, _i64, _i64, ctypes.POINTER(Stage), _i32, _i32, _i64,
                                _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "tfx_chain_backward_workspace_size": (_i32, [_i64, _i64, ctypes.POINTER(Stage), _i32, _i32,
                                                 ctypes.POINTER(_sz)]),
    "tfx_chain_backward": (_i32, [_vp, _vp, _vp, _i64, _i64, _i64, _i64, _i64, ctypes.POINTER(Stage), _i32,
                                  _i32, _vp, ctypes.POINTER(_vp), _vp, _sz, _vp]),
    "tfx_fir_backward_workspace_size": (_i32, [_i64, _i64, _i32, _i32, _i32, ctypes.POINTER(_sz)]),
    "tfx_fir_backward": (_i32, [_vp, _vp, _vp, _i64, _i64, _i64, _i64, _i64, _vp, _i32, _vp, _i32, _i32, _vp,
                                _sz, _vp]),
    "tfx_sos_batched_workspace_size": (_i32, [ctypes.POINTER(Clip), _i32, ctypes.POINTER(_sz)]),
    "tfx_sos_batched_prepare": (_i32, [ctypes.POINTER(Clip), _i32, ctypes.POINTER(BatchConfig), _vp, _sz, _vp]),
    "tfx_sos_batched_run": (_i32, [ctypes.POINTER(Clip), _i32, ctypes.POINTER(BatchConfig), _vp, _sz, _vp]),
    "tfx_sos_batched": (_i32, [ctypes.POINTER(Clip), _i32, ctypes.POINTER(BatchConfig), _vp, _sz, _vp]),
    "tfx_sos_batched_tune": (_i32, [ctypes.POINTER(Clip), _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(BatchConfig),
                                    ctypes.POINTER(ctypes.c_float)]),
    "tfx_rfft": (_i32, [_vp, _i64, _i32, _i64, _vp, _vp]),
    "tfx_irfft": (_i32, [_vp, _i64, _i32, _vp, _i64, _vp]),
    "tfx_stft_frames": (_i32, [_i64, _i32, _i32, _i32, ctypes.POINTER(_i64)]),
    "tfx_stft": (_i32, [_vp, _i64, _i64, _i64, _i32, _i32, _vp, _i32, _i32, _i32, _vp, _vp]),
    "tfx_istft": (_i32, [_vp, _i64, _i64, _i32, _i32, _vp, _i32, _i32, _i32, _vp, _i64, _i64, _vp]),
    "tfx_sos_backward_workspace_size": (_i32, [_i64, _i64, _i32, ctypes.POINTER(_sz)]),
    "tfx_sos_backward": (_i32, [_vp, _vp, _vp, _i64, _i64, _i64, _i64, _i64, _vp, _i32, _vp, _vp, _vp, _sz,
                                _vp]),
}

_lock = threading.Lock()
_lib = None


def load():
    """Load libtfx.so once; raises if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libtfx.so is not built (%s); run paper_2504_08624_amd.build.build()"
                                   % LIB_PATH)
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(lib, name)
                f.restype = res
                f.argtypes = args
            _lib = lib
    return _lib


def declared_functions():
    """Names of every function the C header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tfx_[a-z0-9_]+)\s*\(", text)))


def check(status: int, func: str):
    if status != TFX_OK:
        msg = load().tfx_last_error().decode()
        raise TfxError(status, func, msg)


def call(name: str, *args):
    f = getattr(load(), name)
    check(f(*args), name)


def size_out():
    return ctypes.c_size_t(0)


def stage_array(stages):
    """stages: list of (kind, length, device pointer) -> ctypes array."""
    arr = (Stage * max(1, len(stages)))()
    for i, (kind, n, ptr) in enumerate(stages):
        arr[i].kind = kind
        arr[i].len = n
        arr[i].coef = ptr
    return arr


def pointer_array(ptrs):
    """list of device pointers (or None) -> ctypes void* array."""
    arr = (ctypes.c_void_p * max(1, len(ptrs)))()
    for i, p in enumerate(ptrs):
        arr[i] = p
    return arr

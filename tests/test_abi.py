"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects bad arguments on the host before any HIP
call is made."""
import ctypes

import pytest

from paper_2504_08624_amd import lib


def test_exports_every_declared_function():
    L = lib.load()
    names = lib.declared_functions()
    assert "tfx_chain" in names and "tfx_sos" in names and "tfx_fir" in names
    for n in names:
        assert hasattr(L, n), n


def test_status_strings_and_version():
    L = lib.load()
    for code, name in lib.STATUS_NAMES.items():
        assert L.tfx_status_string(code).decode() == name
    assert L.tfx_version() >= 100
    assert L.tfx_sos_tile_length() == 3072


def _st(name, *args):
    return lib.STATUS_NAMES[getattr(lib.load(), name)(*args)]


FAKE = 1 << 40  # never dereferenced: every call below fails validation first


def test_sos_argument_validation():
    assert _st("tfx_sos", FAKE, FAKE + (1 << 30), 0, 10, 10, 10, FAKE, 1, None, None, None, None, 0, None) \
        == "TFX_E_INVALID_ARG"                                   # C = 0
    assert _st("tfx_sos", FAKE, FAKE + (1 << 30), 2, 10, 5, 10, FAKE, 1, None, None, None, None, 0, None) \
        == "TFX_E_INVALID_ARG"                                   # ldx < N
    assert _st("tfx_sos", FAKE, FAKE + (1 << 30), 2, 10, 10, 10, None, 1, None, None, None, None, 0, None) \
        == "TFX_E_INVALID_ARG"                                   # sos NULL
    assert _st("tfx_sos", FAKE, FAKE + 8, 2, 10, 10, 10, FAKE, 1, None, None, None, None, 0, None) \
        == "TFX_E_ALIAS"
    assert _st("tfx_sos", FAKE, FAKE + (1 << 30), 2, 10, 10, 10, FAKE, 1, None, None, None, None, 0, None) \
        == "TFX_E_WORKSPACE"
    assert _st("tfx_sos", FAKE, FAKE + (1 << 30), 2, 10, 10, 10, FAKE, 1, None, None, None, FAKE + 8,
               1 << 20, None) == "TFX_E_WORKSPACE"                # misaligned
    assert b"aligned" in lib.load().tfx_last_error()


def test_fir_argument_validation():
    assert _st("tfx_fir", FAKE, FAKE + (1 << 30), 2, 10, 10, 10, FAKE, 0, 0, 0, None, 0, None) == "TFX_E_INVALID_ARG"
    assert _st("tfx_fir", FAKE, FAKE + (1 << 30), 2, 10, 10, 10, FAKE, 70000, 0, 0, None, 0, None) \
        == "TFX_E_INVALID_ARG"
    assert _st("tfx_fir", FAKE, FAKE + (1 << 30), 2, 10, 10, 10, FAKE, 5, 9, 0, None, 0, None) == "TFX_E_INVALID_ARG"


def test_chain_stage_validation():
    bad = lib.stage_array([(7, 3, FAKE)])
    assert _st("tfx_chain", FAKE, FAKE + (1 << 30), 1, 10, 10, 10, bad, 1, 0, None, None, 0, None) \
        == "TFX_E_INVALID_ARG"
    null = lib.stage_array([(lib.STAGE_SOS, 2, None)])
    assert _st("tfx_chain", FAKE, FAKE + (1 << 30), 1, 10, 10, 10, null, 1, 0, None, None, 0, None) \
        == "TFX_E_INVALID_ARG"


def test_workspace_sizes():
    n = ctypes.c_size_t(0)
    assert _st("tfx_sos_workspace_size", 8, 5_760_000, 6, ctypes.byref(n)) == "TFX_OK"
    assert n.value > 0 and n.value % 256 == 0
    z = ctypes.c_size_t(123)
    assert _st("tfx_sos_workspace_size", 8, 100, 0, ctypes.byref(z)) == "TFX_OK" and z.value == 0


def test_host_stability_check():
    import numpy as np
    good = np.array([[1, 0, 0, -1.8, 0.9]], np.float32)
    bad = np.array([[1, 0, 0, -2.0, 1.0]], np.float32)
    s = ctypes.c_int32(-1)
    assert _st("tfx_sos_check_stable", good.ctypes.data, 1, ctypes.byref(s)) == "TFX_OK" and s.value == 1
    assert _st("tfx_sos_check_stable", bad.ctypes.data, 1, ctypes.byref(s)) == "TFX_E_UNSTABLE" and s.value == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(lib, "_lib", None)
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="not built"):
        lib.load()


def test_backward_argument_validation():
    # x, gy, gx at disjoint fake addresses; nothing is launched
    X, G, GX = FAKE, FAKE + (1 << 30), FAKE + (2 << 30)
    many = lib.stage_array([(lib.STAGE_SOS, 17, FAKE)])
    assert _st("tfx_chain_backward", X, G, GX, 1, 10, 10, 10, 10, many, 1, 0, FAKE, None, None, 0, None) \
        == "TFX_E_UNSUPPORTED"                                   # more than 16 sections
    assert b"16" in lib.load().tfx_last_error()
    one = lib.stage_array([(lib.STAGE_SOS, 2, FAKE)])
    assert _st("tfx_chain_backward", X, G, GX, 1, 10, 10, 10, 10, one, 1, 0, None, None, None, 0, None) \
        == "TFX_E_INVALID_ARG"                                   # no checkpoints
    assert _st("tfx_chain_backward", X, G, G + 8, 1, 10, 10, 10, 10, one, 1, 0, FAKE, None, None, 0, None) \
        == "TFX_E_ALIAS"                                         # gx overlaps gy
    assert _st("tfx_chain_backward", X, G, GX, 1, 10, 10, 5, 10, one, 1, 0, FAKE, None, None, 0, None) \
        == "TFX_E_INVALID_ARG"                                   # ldg < N
    assert _st("tfx_chain_backward", X, G, GX, 1, 10, 10, 10, 10, one, 1, 0, FAKE, None, None, 0, None) \
        == "TFX_E_WORKSPACE"
    assert _st("tfx_sos_backward", X, G, GX, 1, 10, 10, 10, 10, FAKE, 2, None, None, None, 0, None) \
        == "TFX_E_INVALID_ARG"                                   # no checkpoints
    assert _st("tfx_fir_backward", X, G, GX, 1, 10, 10, 10, 10, None, 5, None, 0, 0, None, 0, None) \
        == "TFX_E_INVALID_ARG"                                   # taps NULL
    assert _st("tfx_fir_backward", X, G, GX, 1, 10, 10, 10, 10, FAKE, 2000, None, 0, 2, None, 0, None) \
        == "TFX_E_UNSUPPORTED"                                   # Toeplitz with fp32 compute


def test_backward_workspace_sizes():
    n = ctypes.c_size_t(0)
    st = lib.stage_array([(lib.STAGE_FIR, 1023, FAKE), (lib.STAGE_SOS, 6, FAKE)])
    assert _st("tfx_chain_backward_workspace_size", 8, 5_760_000, st, 2, 0, ctypes.byref(n)) == "TFX_OK"
    fwd = ctypes.c_size_t(0)
    assert _st("tfx_chain_workspace_size", 8, 5_760_000, st, 2, 0, ctypes.byref(fwd)) == "TFX_OK"
    # the adjoint keeps the gradient of the FIR output (one signal copy); the
    # FIR output itself is recomputed per tile for an FFT FIR of <= 1025 taps
    assert fwd.value + 8 * 5_760_000 * 4 <= n.value < fwd.value + 2 * 8 * 5_760_000 * 4 and n.value % 256 == 0
    st2 = lib.stage_array([(lib.STAGE_FIR, 17, FAKE), (lib.STAGE_SOS, 6, FAKE)])  # direct FIR: both copies
    assert _st("tfx_chain_backward_workspace_size", 8, 5_760_000, st2, 2, 0, ctypes.byref(n)) == "TFX_OK"
    assert n.value >= 2 * 8 * 5_760_000 * 4
    assert _st("tfx_sos_backward_workspace_size", 2, 1000, 3, ctypes.byref(n)) == "TFX_OK" and n.value > 0
    assert _st("tfx_fir_backward_workspace_size", 2, 1000, 64, 0, 0, ctypes.byref(n)) == "TFX_OK" and n.value > 0


def test_batched_validation_and_sizes():
    L = lib.load()
    clips = (lib.Clip * 2)()
    for i in range(2):
        clips[i].x, clips[i].y = FAKE + (i << 32), FAKE + (i << 32) + (1 << 30)
        clips[i].C, clips[i].N, clips[i].ldx, clips[i].ldy = 3, 10000, 10000, 10000
        clips[i].sos, clips[i].S = FAKE, 2 + i
    n = ctypes.c_size_t(0)
    assert _st("tfx_sos_batched_workspace_size", clips, 2, ctypes.byref(n)) == "TFX_OK" and n.value > 0
    cfg = lib.BatchConfig(20, 0)
    assert _st("tfx_sos_batched_prepare", clips, 2, ctypes.byref(cfg), None, 0, None) == "TFX_E_INVALID_ARG"
    cfg = lib.BatchConfig(16, 0)
    assert _st("tfx_sos_batched_prepare", clips, 2, ctypes.byref(cfg), None, 0, None) == "TFX_E_WORKSPACE"
    clips[1].y = clips[1].x + 8                                    # output overlaps the input
    assert _st("tfx_sos_batched_workspace_size", clips, 2, ctypes.byref(n)) == "TFX_E_ALIAS"
    assert b"clip 1" in L.tfx_last_error()


def test_stream_argument_validation():
    st = lib.stage_array([(lib.STAGE_FIR, 33, FAKE), (lib.STAGE_SOS, 2, FAKE + 4096)])
    ws = 1 << 30
    x, y = FAKE, FAKE + (1 << 30)
    # block longer than the prepared length
    assert _st("tfx_chain_stream", x, y, 2, 100, 100, 100, st, 2, 0, 50, None, None, None, None, FAKE, ws,
               None) == "TFX_E_INVALID_ARG"
    # workspace too small for (C, n_max)
    assert _st("tfx_chain_stream", x, y, 2, 100, 100, 100, st, 2, 0, 1 << 20, None, None, None, None, FAKE, 256,
               None) == "TFX_E_WORKSPACE"
    n = ctypes.c_size_t()
    assert _st("tfx_chain_workspace_size", 2, 200, st, 2, 0, ctypes.byref(n)) == "TFX_OK"
    wsb = n.value
    h = FAKE + (1 << 31)
    # history out overlapping history in (2 ch x 32 floats each)
    assert _st("tfx_chain_stream", x, y, 2, 100, 100, 100, st, 2, 0, 200, h, h + 16, None, None, FAKE, wsb,
               None) == "TFX_E_ALIAS"
    # state out overlapping a signal
    assert _st("tfx_chain_stream", x, y, 2, 100, 100, 100, st, 2, 0, 200, None, None, None, y + 40, FAKE, wsb,
               None) == "TFX_E_ALIAS"


def test_stft_argument_validation():
    x, spec = FAKE, FAKE + (1 << 30)
    T = ctypes.c_int64()
    assert _st("tfx_stft_frames", 1000, 256, 64, 1, ctypes.byref(T)) == "TFX_OK" and T.value == 1 + 1000 // 64
    assert _st("tfx_stft_frames", 1000, 256, 64, 0, ctypes.byref(T)) == "TFX_OK" and T.value == 1 + 744 // 64
    assert _st("tfx_stft_frames", 100, 256, 64, 0, ctypes.byref(T)) == "TFX_OK" and T.value == 0
    # n_fft not a power of two / out of range, hop 0, window longer than the frame
    for n_fft in (400, 8, 8192):
        assert _st("tfx_stft", x, 1, 1000, 1000, n_fft, 64, None, n_fft, 1, 0, spec, None) == "TFX_E_UNSUPPORTED"
    assert _st("tfx_stft", x, 1, 1000, 1000, 256, 0, None, 256, 1, 0, spec, None) == "TFX_E_INVALID_ARG"
    assert _st("tfx_stft", x, 1, 1000, 1000, 256, 64, None, 257, 1, 0, spec, None) == "TFX_E_INVALID_ARG"
    # reflect padding needs more than n_fft/2 samples
    assert _st("tfx_stft", x, 1, 128, 128, 256, 64, None, 256, 1, 0, spec, None) == "TFX_E_INVALID_ARG"
    # spectrum overlapping the signal
    assert _st("tfx_stft", x, 2, 1000, 1000, 256, 64, None, 256, 1, 0, x + 64, None) == "TFX_E_ALIAS"
    # no frames: nothing to do
    assert _st("tfx_stft", x, 1, 100, 100, 256, 64, None, 256, 0, 0, spec, None) == "TFX_OK"


def test_istft_argument_validation():
    spec, y = FAKE, FAKE + (1 << 30)
    assert _st("tfx_istft", spec, 2, 10, 256, 64, None, 256, 1, 0, y, -1, 100, None) == "TFX_E_INVALID_ARG"  # ldy
    assert _st("tfx_istft", spec, 2, 0, 256, 64, None, 256, 1, 0, y, -1, 1000, None) == "TFX_E_INVALID_ARG"  # T
    assert _st("tfx_istft", spec, 2, 10, 256, 0, None, 256, 1, 0, y, -1, 1000, None) == "TFX_E_INVALID_ARG"  # hop
    assert _st("tfx_istft", spec, 2, 10, 256, 64, None, 256, 1, 0, spec + 8, -1, 1000, None) == "TFX_E_ALIAS"
    assert _st("tfx_istft", spec, 2, 10, 300, 64, None, 256, 1, 0, y, -1, 1000, None) == "TFX_E_UNSUPPORTED"
    assert _st("tfx_istft", spec, 2, 10, 256, 64, None, 256, 1, 0, y, 1 << 38, 1 << 38, None) == "TFX_E_UNSUPPORTED"
    # zero-length output: nothing to do
    assert _st("tfx_istft", spec, 2, 10, 256, 64, None, 256, 1, 0, y, 0, 0, None) == "TFX_OK"


def test_workspace_status_arguments():
    # flags NULL is an argument error; a call that needed no workspace (NULL
    # ws or fewer than 256 bytes) has no status word and enqueues nothing
    assert _st("tfx_workspace_status", FAKE, 4096, None, 0, None) == "TFX_E_INVALID_ARG"
    assert _st("tfx_workspace_status", None, 0, FAKE, 0, None) == "TFX_OK"
    assert _st("tfx_workspace_status", FAKE, 128, FAKE, 1, None) == "TFX_OK"
    assert _st("tfx_workspace_status", FAKE + 8, 4096, FAKE, 1, None) == "TFX_E_WORKSPACE"
    assert lib.STATUS_NAMES[lib.TFX_E_DEVICE] == "TFX_E_DEVICE"


def test_tuning_cache_file_drives_the_automatic_choice(tmp_path):
    """An entry of the persistent tuning cache (arch "*": any device) decides
    TFX_FIR_AUTO for its (M, C, log2 N) key: the 777-tap, 5-channel, 2^9..2^10
    sample shape is sent to the direct form (no workspace) instead of the FFT
    (a workspace); the neighbouring tap count keeps the fixed rule.  Lines
    that are malformed or name a form the key does not admit are skipped and
    reported."""
    import paper_2504_08624_amd as tfx
    n = ctypes.c_size_t(0)
    assert _st("tfx_fir_workspace_size", 5, 1000, 777, 0, 0, ctypes.byref(n)) == "TFX_OK" and n.value > 0
    path = tmp_path / "tune.txt"
    path.write_text("# comment\n"
                    "fir * 777 5 9 0 1 0 0.25\n"          # direct, fp32, class 1e-5
                    "fir * 777 5 9 2 2 1 0.10\n"          # Toeplitz bf16 for the 1e-2 class
                    "fir * 9000 5 9 0 4 0 0.5\n"          # the 16384-point form cannot take 9000 taps
                    "fir * 777 5 9 0 2 1 0.1\n"           # bf16 is not admitted at 1e-5
                    "garbage\n")
    L = lib.load()
    assert lib.STATUS_NAMES[L.tfx_set_tuning_cache(str(path).encode())] == "TFX_E_INVALID_ARG"
    assert b"3 malformed" in L.tfx_last_error()
    assert tfx.fir_tuned(5, 1000, 777) == ("direct", "f32")
    assert tfx.fir_tuned(5, 1000, 777, tol=1e-2) == ("toeplitz", "bf16")
    assert tfx.fir_tuned(5, 1000, 778) == ("auto", "f32")
    assert tfx.fir_tuned(5, 5000, 777) == ("auto", "f32")        # another log2 N bucket
    assert _st("tfx_fir_workspace_size", 5, 1000, 777, 0, 0, ctypes.byref(n)) == "TFX_OK" and n.value == 0
    assert _st("tfx_fir_workspace_size", 5, 1000, 778, 0, 0, ctypes.byref(n)) == "TFX_OK" and n.value > 0
    tfx.set_tuning_cache(None)  # memory only from here on; the entries stay


def test_autotune_arguments():
    n16 = ctypes.c_size_t(0)
    n2 = ctypes.c_size_t(0)
    assert _st("tfx_fir_autotune_workspace_size", 8, 100_000, 1023, 1e-5, ctypes.byref(n16)) == "TFX_OK"
    assert _st("tfx_fir_autotune_workspace_size", 8, 100_000, 1023, 1e-2, ctypes.byref(n2)) == "TFX_OK"
    assert n2.value >= n16.value > 0
    assert _st("tfx_fir_autotune_workspace_size", 8, 100_000, 1023, 1e-6, ctypes.byref(n2)) == "TFX_E_UNSUPPORTED"
    a, c, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_float(0)
    assert _st("tfx_fir_autotune", FAKE, FAKE + (1 << 30), 2, 10, 10, 10, FAKE, 5, 1e-6, 1, None, 0, None,
               ctypes.byref(a), ctypes.byref(c), ctypes.byref(ms)) == "TFX_E_UNSUPPORTED"
    assert _st("tfx_fir_autotune", FAKE, FAKE + (1 << 30), 2, 10, 10, 10, FAKE, 5, 1e-5, 0, None, 0, None,
               ctypes.byref(a), ctypes.byref(c), ctypes.byref(ms)) == "TFX_E_INVALID_ARG"   # reps = 0

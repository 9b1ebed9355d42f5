"""MI355X-native multichannel FIR / IIR-SOS filter chains (TorchFX's hot path).

The filtering runs in hand-written HIP kernels for gfx950 behind the C ABI of
libtfx.so (include/tfx.h); this package is its Python binding.  Importing it
loads nothing: the library is loaded on the first call and every call raises
if it is not built (there is no CPU fallback).
"""
from .functional import (ChainStream, SosBatch, chain, chain_backward, check_device_status,  # noqa: F401
                         device_status, fir, fir_autotune, fir_backward, fir_tuned, lfilter, set_tuning_cache, sos,
                         sos_backward, sos_batched, tile_length)
from .filters import (FIR, SOS, AllPass, BandPass, Butterworth, ButterworthBand, Chebyshev1, Chebyshev2,  # noqa: F401
                      DirectForm, Filter, HiShelving, LoShelving, Notch, Peaking, WindowedSincFIR)
from .spectral import irfft, istft, rfft, stft  # noqa: F401
from .wave import Wave  # noqa: F401

__all__ = ["fir", "sos", "chain", "lfilter", "stft", "istft", "rfft", "irfft", "ChainStream", "fir_backward", "sos_backward", "chain_backward", "sos_batched", "SosBatch",
           "tile_length", "device_status", "check_device_status", "fir_autotune", "fir_tuned",
           "set_tuning_cache", "Wave", "Filter", "Butterworth", "Chebyshev1", "Peaking", "HiShelving", "LoShelving",
           "WindowedSincFIR", "FIR", "SOS", "Chebyshev2", "ButterworthBand", "Notch", "AllPass", "BandPass",
           "DirectForm"]

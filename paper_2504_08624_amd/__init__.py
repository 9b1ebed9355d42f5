"""MI355X-native multichannel FIR / IIR-SOS filter chains (TorchFX's hot path).

The filtering runs in hand-written HIP kernels for gfx950 behind the C ABI of
libtfx.so (include/tfx.h); this package is its Python binding.  Importing it
loads nothing: the library is loaded on the first call and every call raises
if it is not built (there is no CPU fallback).
"""
from .functional import (ChainStream, SosBatch, chain, chain_backward, fir, fir_backward, sos,  # noqa: F401
                         sos_backward, sos_batched, tile_length)
from .filters import (FIR, SOS, Butterworth, Chebyshev1, Filter, HiShelving, LoShelving, Peaking,  # noqa: F401
                      WindowedSincFIR)
from .wave import Wave  # noqa: F401

__all__ = ["fir", "sos", "chain", "ChainStream", "fir_backward", "sos_backward", "chain_backward", "sos_batched", "SosBatch",
           "tile_length", "Wave", "Filter", "Butterworth", "Chebyshev1", "Peaking", "HiShelving", "LoShelving",
           "WindowedSincFIR", "FIR", "SOS"]

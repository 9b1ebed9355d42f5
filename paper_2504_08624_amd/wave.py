"""``Wave``: a multichannel signal with its sample rate, and the pipe.

Sec. 3 keeps the samples and the sample rate together and overloads ``|`` as
a pipe, so ``wave | HiShelving(1000) | LoShelving(2000)`` filters the signal
with the filters' sample rate bound from the wave.  Here the pipe is lazy:
piping a filter (or a ``Sequential`` of filters) into a wave only records the
stage, and the recorded stages run as one fused chain (one kernel launch for
the whole cascade, FIR stages merged in front) when the samples are read
(``.y``).  Any other module is applied to the samples at once.  WAV files
are read and written on the host (``from_file``, ``save``).
"""
from __future__ import annotations

from typing import List, Optional

import torch

from .filters import Filter, stages_of
from .functional import chain


class Wave:
    """Samples ``[C, N]`` (a 1-D signal is one channel) at ``fs`` Hz."""

    def __init__(self, y: torch.Tensor, fs: float, _pending: Optional[List[Filter]] = None):
        if not isinstance(y, torch.Tensor):
            y = torch.as_tensor(y, dtype=torch.float32)
        if y.dim() == 1:
            y = y.unsqueeze(0)
        if y.dim() != 2:
            raise ValueError("a Wave holds [channels, samples]")
        if fs <= 0:
            raise ValueError("the sample rate must be positive")
        self._y = y
        self.fs = float(fs)
        self._pending = list(_pending or [])

    @property
    def y(self) -> torch.Tensor:
        """The samples, after every pending stage (one fused launch)."""
        if self._pending:
            self._y = chain(self._y, [f.stage(self._y.device) for f in self._pending])
            self._pending = []
        return self._y

    @property
    def channels(self) -> int:
        return self._y.shape[0]

    def __len__(self) -> int:
        return self._y.shape[1]

    @property
    def duration(self) -> float:
        return len(self) / self.fs

    @property
    def pending(self) -> List[Filter]:
        """Stages recorded by the pipe and not yet run."""
        return list(self._pending)

    def to(self, device) -> "Wave":
        return Wave(self.y.to(device), self.fs)

    @classmethod
    def from_file(cls, path, device=None) -> "Wave":
        """Reads a WAV file (PCM 8/16/32-bit or float) as float32 samples in
        [-1, 1), channels first, with the file's sample rate."""
        import numpy as np
        from scipy.io import wavfile
        fs, data = wavfile.read(path)
        data = np.asarray(data)
        if data.dtype == np.uint8:
            y = (data.astype(np.float32) - 128.0) / 128.0
        elif data.dtype.kind == "i":
            y = data.astype(np.float32) / float(2 ** (8 * data.dtype.itemsize - 1))
        else:
            y = data.astype(np.float32)
        y = y.T if y.ndim == 2 else y[None, :]
        t = torch.from_numpy(np.ascontiguousarray(y))
        return cls(t.to(device) if device is not None else t, float(fs))

    def save(self, path) -> None:
        """Writes the samples (after any pending stages) as a 32-bit float WAV."""
        import numpy as np
        from scipy.io import wavfile
        wavfile.write(path, int(round(self.fs)), np.ascontiguousarray(self.y.detach().cpu().numpy().T))

    def __or__(self, module) -> "Wave":
        stages = stages_of(module, self.fs)
        if stages is not None:
            return Wave(self._y, self.fs, self._pending + stages)
        if isinstance(module, torch.nn.Module) or callable(module):
            return Wave(module(self.y), self.fs)
        raise TypeError("cannot pipe a Wave into %r" % (module,))

    def __repr__(self) -> str:
        return "Wave(%d ch x %d samples @ %g Hz%s)" % (self.channels, len(self), self.fs,
                                                     ", %d pending" % len(self._pending) if self._pending
                                                     else "")

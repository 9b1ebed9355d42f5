"""``Wave``: a multichannel signal with its sample rate, and the pipe.

Sec. 3 keeps the samples and the sample rate together and overloads ``|`` as
a pipe, so ``wave | HiShelving(1000) | LoShelving(2000)`` filters the signal
with the filters' sample rate bound from the wave.  Here the pipe is lazy:
piping a filter (or a ``Sequential`` of filters) into a wave only records the
stage, and the recorded stages run as one fused chain (one kernel launch for
the whole cascade, FIR stages merged in front) when the samples are read
(``.y``).  Any other module is applied to the samples at once.
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

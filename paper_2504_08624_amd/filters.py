"""Filter classes over the fused chain (the object interface of Sec. 3).

Every filter is a ``torch.nn.Module`` holding one stage of the chain: FIR taps
or SOS sections (rows [b0 b1 b2 a1 a2], a0 = 1).  Designed filters
(Butterworth low/high/band-pass/band-stop, Chebyshev types I and II, peaking,
shelving, notch, all-pass, band-pass biquad, windowed-sinc FIR) are
designed in FP64 on the host from their parameters and the sample rate, and
rounded to fp32 once per (sample rate, device).  The sample rate may be given
at construction (``sample_rate=``) or left open and bound lazily by the pipe
of a ``Wave`` (``wave | HiShelving(1000)``), as Sec. 3 describes.

Calling a filter on a tensor runs it through the library (one launch);
``Sequential`` works as usual.  Piping a ``Wave`` through filters, a
``Sequential`` of filters, or a chain of pipes collects the stages and runs
them as one fused chain (see ``wave.Wave``).  ``FIR`` and ``SOS`` hold
explicit coefficients, trainable when ``learnable=True`` (the adjoint of the
library gives their gradients).
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np
import torch
from torch import nn

from . import design
from .functional import chain


class Filter(nn.Module):
    """One stage of a chain.  Subclasses define ``kind`` ("fir" or "sos") and
    either ``_design(fs)`` (designed filters) or ``coefficients(device)``."""

    kind = "sos"

    def __init__(self, sample_rate: Optional[float] = None):
        super().__init__()
        self.sample_rate = None if sample_rate is None else float(sample_rate)
        self._cache = {}

    # ---------------------------------------------------------- sample rate
    def bind(self, fs: float) -> "Filter":
        """Sets the sample rate if it is open; a filter built for another rate
        is an error (its design would be wrong for this signal)."""
        fs = float(fs)
        if self.sample_rate is None:
            self.sample_rate = fs
        elif self.sample_rate != fs:
            raise ValueError("%s was built for %g Hz, the signal is %g Hz" % (type(self).__name__,
                                                                              self.sample_rate, fs))
        return self

    def _design(self, fs: float) -> np.ndarray:
        raise NotImplementedError

    def coefficients(self, device) -> torch.Tensor:
        """fp32 coefficients on ``device`` (designed in FP64 on first use)."""
        if self.sample_rate is None:
            raise ValueError("%s has no sample rate: give sample_rate= or pipe a Wave through it"
                             % type(self).__name__)
        key = (self.sample_rate, str(device))
        t = self._cache.get(key)
        if t is None:
            c = np.asarray(self._design(self.sample_rate), dtype=np.float64)
            t = torch.as_tensor(c.astype(np.float32)).to(device)
            self._cache[key] = t
        return t

    def stage(self, device) -> Tuple[str, torch.Tensor]:
        return self.kind, self.coefficients(device)

    def forward(self, x):
        from .wave import Wave
        if isinstance(x, Wave):
            return x | self
        return chain(x, [self.stage(x.device)])


def stages_of(module, fs: Optional[float]) -> Optional[List[Filter]]:
    """The filters of a Filter or a (nested) Sequential of filters, with the
    sample rate bound; None if the module holds anything else."""
    if isinstance(module, Filter):
        return [module.bind(fs) if fs is not None else module]
    if isinstance(module, nn.Sequential):
        out = []
        for m in module:
            s = stages_of(m, fs)
            if s is None:
                return None
            out.extend(s)
        return out
    return None


# ------------------------------------------------------------------- IIR

class Butterworth(Filter):
    """Butterworth low- or high-pass of even or odd ``order`` (bilinear,
    prewarped), as ceil(order / 2) sections."""

    def __init__(self, cutoff: float, sample_rate: Optional[float] = None, *, order: int = 4,
                 btype: str = "lowpass"):
        super().__init__(sample_rate)
        self.cutoff, self.order, self.btype = float(cutoff), int(order), btype

    def _design(self, fs):
        return design.butterworth(self.order, self.cutoff, fs, self.btype)


class Chebyshev1(Filter):
    """Chebyshev type I low- or high-pass (passband ripple ``ripple_db``)."""

    def __init__(self, cutoff: float, sample_rate: Optional[float] = None, *, order: int = 4,
                 ripple_db: float = 1.0, btype: str = "lowpass"):
        super().__init__(sample_rate)
        self.cutoff, self.order, self.ripple_db, self.btype = float(cutoff), int(order), float(ripple_db), btype

    def _design(self, fs):
        return design.chebyshev1(self.order, self.ripple_db, self.cutoff, fs, self.btype)


class Peaking(Filter):
    """Peaking equaliser at ``center`` Hz (one section)."""

    def __init__(self, center: float, sample_rate: Optional[float] = None, *, q: float = 1.0,
                 gain_db: float = 6.0):
        super().__init__(sample_rate)
        self.center, self.q, self.gain_db = float(center), float(q), float(gain_db)

    def _design(self, fs):
        return design.peaking(self.center, self.q, self.gain_db, fs)


class HiShelving(Filter):
    """High shelf above ``cutoff`` Hz (one section)."""

    def __init__(self, cutoff: float, sample_rate: Optional[float] = None, *, gain_db: float = 6.0,
                 slope: float = 1.0):
        super().__init__(sample_rate)
        self.cutoff, self.gain_db, self.slope = float(cutoff), float(gain_db), float(slope)

    def _design(self, fs):
        return design.shelf(self.cutoff, self.gain_db, fs, "high", self.slope)


class LoShelving(Filter):
    """Low shelf below ``cutoff`` Hz (one section)."""

    def __init__(self, cutoff: float, sample_rate: Optional[float] = None, *, gain_db: float = 6.0,
                 slope: float = 1.0):
        super().__init__(sample_rate)
        self.cutoff, self.gain_db, self.slope = float(cutoff), float(gain_db), float(slope)

    def _design(self, fs):
        return design.shelf(self.cutoff, self.gain_db, fs, "low", self.slope)


class Chebyshev2(Filter):
    """Chebyshev type II low- or high-pass (stopband ``atten_db`` down from
    the stopband edge ``cutoff``)."""

    def __init__(self, cutoff: float, sample_rate: Optional[float] = None, *, order: int = 4,
                 atten_db: float = 40.0, btype: str = "lowpass"):
        super().__init__(sample_rate)
        self.cutoff, self.order, self.atten_db, self.btype = float(cutoff), int(order), float(atten_db), btype

    def _design(self, fs):
        return design.chebyshev2(self.order, self.atten_db, self.cutoff, fs, self.btype)


class ButterworthBand(Filter):
    """Butterworth band-pass or band-stop between ``low`` and ``high`` Hz
    (``order`` is the prototype order: ``order`` sections)."""

    def __init__(self, low: float, high: float, sample_rate: Optional[float] = None, *, order: int = 2,
                 btype: str = "bandpass"):
        super().__init__(sample_rate)
        self.low, self.high, self.order, self.btype = float(low), float(high), int(order), btype

    def _design(self, fs):
        return design.butterworth_band(self.order, self.low, self.high, fs, self.btype)


class Notch(Filter):
    """Second-order notch at ``center`` Hz (one section)."""

    def __init__(self, center: float, sample_rate: Optional[float] = None, *, q: float = 10.0):
        super().__init__(sample_rate)
        self.center, self.q = float(center), float(q)

    def _design(self, fs):
        return design.notch(self.center, self.q, fs)


class AllPass(Filter):
    """Second-order all-pass centred at ``center`` Hz (one section)."""

    def __init__(self, center: float, sample_rate: Optional[float] = None, *, q: float = 0.707):
        super().__init__(sample_rate)
        self.center, self.q = float(center), float(q)

    def _design(self, fs):
        return design.allpass(self.center, self.q, fs)


class BandPass(Filter):
    """Second-order band-pass with unit gain at ``center`` Hz (one section)."""

    def __init__(self, center: float, sample_rate: Optional[float] = None, *, q: float = 0.707):
        super().__init__(sample_rate)
        self.center, self.q = float(center), float(q)

    def _design(self, fs):
        return design.bandpass_biquad(self.center, self.q, fs)


class DirectForm(Filter):
    """Direct-form transfer function b(z^-1) / a(z^-1), factored into
    sections in FP64 (an unstable denominator is an error).  Needs no sample
    rate."""

    def __init__(self, b, a):
        super().__init__(None)
        self.b = np.asarray(b, dtype=np.float64).reshape(-1)
        self.a = np.asarray(a, dtype=np.float64).reshape(-1)
        rows = design.tf2sos(self.b, self.a)
        if design.max_pole_radius(rows) >= 1.0:
            raise ValueError("the denominator has a pole on or outside the unit circle")
        self._rows = rows

    def bind(self, fs):
        return self

    def coefficients(self, device):
        key = str(device)
        t = self._cache.get(key)
        if t is None:
            t = torch.as_tensor(self._rows.astype(np.float32)).to(device)
            self._cache[key] = t
        return t


class SOS(Filter):
    """Explicit sections [S, 5] (rows b0 b1 b2 a1 a2); trainable with
    ``learnable=True``.  Needs no sample rate."""

    def __init__(self, sections, learnable: bool = False):
        super().__init__(None)
        t = torch.as_tensor(np.asarray(sections, dtype=np.float32).reshape(-1, 5))
        if learnable:
            self.sections = nn.Parameter(t)
        else:
            self.register_buffer("sections", t)

    def bind(self, fs):
        return self

    def coefficients(self, device):
        return self.sections if self.sections.device == torch.device(device) else self.sections.to(device)


# ------------------------------------------------------------------- FIR

class FIR(Filter):
    """Explicit taps (y = h * x); trainable with ``learnable=True``.  Needs no
    sample rate."""

    kind = "fir"

    def __init__(self, taps, learnable: bool = False):
        super().__init__(None)
        t = torch.as_tensor(np.asarray(taps, dtype=np.float32).reshape(-1))
        if learnable:
            self.taps = nn.Parameter(t)
        else:
            self.register_buffer("taps", t)

    def bind(self, fs):
        return self

    def coefficients(self, device):
        return self.taps if self.taps.device == torch.device(device) else self.taps.to(device)


class WindowedSincFIR(Filter):
    """Hamming windowed-sinc FIR of ``num_taps`` taps: low-pass at ``cutoff``,
    or band-pass [cutoff, cutoff_hi] when ``cutoff_hi`` is given."""

    kind = "fir"

    def __init__(self, cutoff: float, sample_rate: Optional[float] = None, *, num_taps: int = 101,
                 cutoff_hi: Optional[float] = None):
        super().__init__(sample_rate)
        self.cutoff, self.num_taps = float(cutoff), int(num_taps)
        self.cutoff_hi = None if cutoff_hi is None else float(cutoff_hi)

    def _design(self, fs):
        if self.cutoff_hi is None:
            return design.fir_lowpass(self.num_taps, self.cutoff, fs)
        return design.fir_bandpass(self.num_taps, self.cutoff, self.cutoff_hi, fs)

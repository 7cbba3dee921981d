"""MI355X-native SPIIR filter-bank hot path (Chu et al., arXiv:2011.06787).

The compute lives in ``libspiir.so`` (hand-written HIP for gfx950, C ABI in
``include/spiir.h``); :mod:`.spiir` is its thin ctypes binding.
"""
from . import spiir  # noqa: F401
from .spiir import SpiirBank, SpiirError, peaks, spiir_filter  # noqa: F401

__all__ = ["spiir", "SpiirBank", "SpiirError", "peaks", "spiir_filter"]

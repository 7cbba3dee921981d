"""ctypes binding of libspiir (the C ABI declared in include/spiir.h).

Argument marshalling only: every step of the filter bank runs in the HIP
library.  torch provides device memory and streams.  Loading fails loudly if the
library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspiir.so")

SPIIR_OK = 0
SPIIR_E_INVAL = 1
SPIIR_E_NOMEM = 2
SPIIR_E_HIP = 3
SPIIR_E_STATE = 4
SPIIR_E_UNSUPPORTED = 5

MODE_FP32_SCAN = 0
MODE_BF16_BLOCK = 1

# every function declared in include/spiir.h
EXPORTS = (
    "spiir_opts_default", "spiir_bank_create", "spiir_bank_destroy", "spiir_bank_reset",
    "spiir_bank_get_info", "spiir_filter_chunk", "spiir_peaks", "spiir_last_error",
    "spiir_bank_set_timing", "spiir_bank_kernel_time",
)


class SpiirError(RuntimeError):
    def __init__(self, func: str, status: int, message: str):
        super().__init__(f"{func} failed with status {status}: {message}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [
        ("n_detectors", ctypes.c_int32),
        ("max_chunk", ctypes.c_int32),
        ("max_delay", ctypes.c_int32),
        ("peak_window", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("filters_per_lane", ctypes.c_int32),
        ("time_tile", ctypes.c_int32),
        ("block_len", ctypes.c_int32),
        ("long_pole_abs_a", ctypes.c_double),
    ]


class BankInfo(ctypes.Structure):
    _fields_ = [
        ("n_templates", ctypes.c_int32), ("n_detectors", ctypes.c_int32),
        ("max_chunk", ctypes.c_int32), ("max_delay", ctypes.c_int32),
        ("peak_window", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("n_filters", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
        ("n_slices", ctypes.c_int32), ("filters_per_lane", ctypes.c_int32),
        ("time_tile", ctypes.c_int32), ("scan_waves", ctypes.c_int32),
        ("block_len", ctypes.c_int32), ("n_long_pole", ctypes.c_int32),
        ("scan_wait_timeouts", ctypes.c_int32),
    ]


_lib = None
_P = ctypes.c_void_p


def load():
    """Load libspiir.so; raises if it is missing (build it with ``build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libspiir.so not found at {LIB_PATH}: run paper_2011_06787_amd/build.py "
                           "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    lib.spiir_opts_default.argtypes = [ctypes.POINTER(Opts)]
    lib.spiir_opts_default.restype = None
    lib.spiir_bank_create.argtypes = [ctypes.c_int32, _P, _P, _P, _P, ctypes.POINTER(Opts), _P,
                                      ctypes.POINTER(_P)]
    lib.spiir_bank_destroy.argtypes = [_P]
    lib.spiir_bank_reset.argtypes = [_P, _P]
    lib.spiir_bank_get_info.argtypes = [_P, ctypes.POINTER(BankInfo)]
    lib.spiir_filter_chunk.argtypes = [_P, _P, ctypes.c_int32, _P, _P, _P, _P]
    lib.spiir_peaks.argtypes = [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]
    lib.spiir_bank_set_timing.argtypes = [_P, ctypes.c_int32, ctypes.c_int32]
    lib.spiir_bank_kernel_time.argtypes = [_P, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64)]
    lib.spiir_last_error.argtypes = []
    lib.spiir_last_error.restype = ctypes.c_char_p
    for name in ("spiir_bank_create", "spiir_bank_destroy", "spiir_bank_reset",
                 "spiir_bank_get_info", "spiir_filter_chunk", "spiir_peaks",
                 "spiir_bank_set_timing", "spiir_bank_kernel_time"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().spiir_last_error().decode()


def _check(func: str, status: int):
    if status != SPIIR_OK:
        raise SpiirError(func, status, last_error())


def _stream_ptr(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def default_opts() -> Opts:
    o = Opts()
    load().spiir_opts_default(ctypes.byref(o))
    return o


class SpiirBank:
    """A SPIIR bank resident on the GPU, with per-detector stream state.

    ``offsets`` int32 [T+1], ``a``/``b`` complex64 [F], ``delay`` int32 [F] are host
    arrays (numpy); they are copied at creation.
    """

    def __init__(self, offsets, a, b, delay, *, n_detectors: int = 1, max_chunk: int = 2048,
                 max_delay: int = 0, peak_window: int = 0, mode: int = MODE_FP32_SCAN,
                 filters_per_lane: int = 0, time_tile: int = 0, block_len: int = 0,
                 long_pole_abs_a: float = 0.999, stream=None):
        lib = load()
        self._offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        self._a = np.ascontiguousarray(a, dtype=np.complex64)
        self._b = np.ascontiguousarray(b, dtype=np.complex64)
        self._d = np.ascontiguousarray(delay, dtype=np.int32)
        o = default_opts()
        o.n_detectors, o.max_chunk, o.max_delay = n_detectors, max_chunk, max_delay
        o.peak_window, o.mode, o.filters_per_lane = peak_window, mode, filters_per_lane
        o.time_tile, o.block_len, o.long_pole_abs_a = time_tile, block_len, long_pole_abs_a
        self.opts = o
        h = _P()
        st = lib.spiir_bank_create(int(self._offsets.shape[0] - 1),
                                   self._offsets.ctypes.data, self._a.ctypes.data,
                                   self._b.ctypes.data, self._d.ctypes.data, ctypes.byref(o),
                                   _stream_ptr(stream), ctypes.byref(h))
        _check("spiir_bank_create", st)
        self._h = h
        self.info = self._info()

    @classmethod
    def from_bank(cls, bank, **kw) -> "SpiirBank":
        """From a ``synth.Bank``-like object with offsets, a, b, d."""
        return cls(bank.offsets, bank.a, bank.b, bank.d, **kw)

    def refresh_info(self) -> BankInfo:
        self.info = self._info()
        return self.info

    def _info(self) -> BankInfo:
        info = BankInfo()
        _check("spiir_bank_get_info", load().spiir_bank_get_info(self._h, ctypes.byref(info)))
        return info

    @property
    def n_templates(self) -> int:
        return self.info.n_templates

    @property
    def n_detectors(self) -> int:
        return self.info.n_detectors

    def n_windows(self, n: int) -> int:
        w = self.info.peak_window
        return 1 if w == 0 else n // w

    def reset(self, stream=None):
        _check("spiir_bank_reset", load().spiir_bank_reset(self._h, _stream_ptr(stream)))

    def filter_chunk(self, x, z=None, peak=None, argmax=None, *, want_z: bool = True,
                     want_peaks: bool = True, stream=None):
        """Filter one packet x (cuda float32 [D][n]); returns (z, peak, argmax).

        Outputs are allocated with torch when not given (z complex64 [D][T][n],
        peak float32 [D][T][W], argmax int32 [D][T][W]); unwanted outputs are None.
        """
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        assert x.dim() == 2 and x.shape[0] == self.n_detectors
        n = int(x.shape[1])
        D, T = self.n_detectors, self.n_templates
        if z is None and want_z:
            z = torch.empty((D, T, n), dtype=torch.complex64, device=x.device)
        if peak is None and want_peaks:
            W = self.n_windows(n)
            peak = torch.empty((D, T, W), dtype=torch.float32, device=x.device)
            argmax = torch.empty((D, T, W), dtype=torch.int32, device=x.device)
        st = load().spiir_filter_chunk(self._h, x.data_ptr(), n, _dptr(z), _dptr(peak),
                                       _dptr(argmax), _stream_ptr(stream))
        _check("spiir_filter_chunk", st)
        return z, peak, argmax

    def set_timing(self, enable: bool, capacity: int = 4096):
        """Bracket the main filtering kernel with HIP events (see spiir.h)."""
        _check("spiir_bank_set_timing",
               load().spiir_bank_set_timing(self._h, int(enable), int(capacity)))

    def kernel_time(self) -> Tuple[float, int]:
        """(summed kernel milliseconds, timed launches) since timing was enabled."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check("spiir_bank_kernel_time",
               load().spiir_bank_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def close(self):
        if getattr(self, "_h", None):
            st = load().spiir_bank_destroy(self._h)
            self._h = None
            _check("spiir_bank_destroy", st)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def peaks(z, window: int, peak=None, argmax=None, stream=None) -> Tuple["object", "object"]:
    """Largest |z| per window of each row of z (cuda complex64 [..., n]) and its index."""
    import torch
    assert z.is_cuda and z.dtype == torch.complex64 and z.is_contiguous()
    n = int(z.shape[-1])
    rows = int(np.prod(z.shape[:-1])) if z.dim() > 1 else 1
    n_win = (n + window - 1) // window if window > 0 else 0
    shape = tuple(z.shape[:-1]) + (n_win,)
    if peak is None:
        peak = torch.empty(shape, dtype=torch.float32, device=z.device)
        argmax = torch.empty(shape, dtype=torch.int32, device=z.device)
    st = load().spiir_peaks(z.data_ptr(), rows, n, window, _dptr(peak), _dptr(argmax),
                            _stream_ptr(stream))
    _check("spiir_peaks", st)
    return peak, argmax

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
    "spiir_bank_set_timing", "spiir_bank_kernel_time", "spiir_ckpt_count", "spiir_forward",
    "spiir_backward", "spiir_bank_set_coeffs", "spiir_bank_noise_power", "spiir_triggers",
    "spiir_bank_autocorr", "spiir_xi2", "spiir_coherent", "spiir_triggers_noalloc",
    "spiir_xi2_network", "spiir_bank_trigger_weights",
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
        ("ckpt_stride", ctypes.c_int32),
        ("balance_wgs", ctypes.c_int32),
        ("wait_spins", ctypes.c_int32),
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
        ("scan_wait_timeouts", ctypes.c_int32), ("balance_waves", ctypes.c_int32),
        ("block_mfma_flop_per_column", ctypes.c_int64),
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
    lib.spiir_ckpt_count.argtypes = [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    lib.spiir_forward.argtypes = [_P, _P, ctypes.c_int32, _P, _P, _P]
    lib.spiir_backward.argtypes = [_P, _P, ctypes.c_int32, _P, _P, _P, _P, _P]
    lib.spiir_bank_set_coeffs.argtypes = [_P, _P, _P, _P]
    lib.spiir_bank_noise_power.argtypes = [_P, _P]
    lib.spiir_triggers.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                   ctypes.c_float, ctypes.c_int32, _P, _P, _P, _P]
    lib.spiir_triggers_noalloc.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                           ctypes.c_float, ctypes.c_int32, _P, _P, _P]
    lib.spiir_bank_autocorr.argtypes = [_P, ctypes.c_int32, _P, _P]
    lib.spiir_bank_trigger_weights.argtypes = [_P, _P, _P]
    lib.spiir_xi2.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                              _P, ctypes.c_int32, _P, _P]
    lib.spiir_xi2_network.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                      ctypes.c_int32, _P, ctypes.c_int32, _P, ctypes.c_int32, _P,
                                      _P, _P]
    lib.spiir_coherent.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                   ctypes.c_int32, _P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P,
                                   _P, _P, _P]
    lib.spiir_last_error.argtypes = []
    lib.spiir_last_error.restype = ctypes.c_char_p
    for name in ("spiir_bank_create", "spiir_bank_destroy", "spiir_bank_reset",
                 "spiir_bank_get_info", "spiir_filter_chunk", "spiir_peaks",
                 "spiir_bank_set_timing", "spiir_bank_kernel_time", "spiir_ckpt_count",
                 "spiir_forward", "spiir_backward", "spiir_bank_set_coeffs",
                 "spiir_bank_noise_power", "spiir_triggers", "spiir_triggers_noalloc",
                 "spiir_bank_autocorr", "spiir_xi2", "spiir_coherent", "spiir_xi2_network",
                 "spiir_bank_trigger_weights"):
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
                 long_pole_abs_a: float = 0.999, ckpt_stride: int = 0, balance_wgs: int = 0,
                 wait_spins: int = 0, stream=None):
        lib = load()
        self._offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        self._a = np.ascontiguousarray(a, dtype=np.complex64)
        self._b = np.ascontiguousarray(b, dtype=np.complex64)
        self._d = np.ascontiguousarray(delay, dtype=np.int32)
        o = default_opts()
        o.n_detectors, o.max_chunk, o.max_delay = n_detectors, max_chunk, max_delay
        o.peak_window, o.mode, o.filters_per_lane = peak_window, mode, filters_per_lane
        o.time_tile, o.block_len, o.long_pole_abs_a = time_tile, block_len, long_pole_abs_a
        o.ckpt_stride, o.balance_wgs, o.wait_spins = ckpt_stride, balance_wgs, wait_spins
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

    # ---- differentiation (FP32 scan mode) ----
    def ckpt_count(self, n: int) -> int:
        cnt = ctypes.c_int64()
        _check("spiir_ckpt_count", load().spiir_ckpt_count(self._h, int(n), ctypes.byref(cnt)))
        return cnt.value

    def forward(self, x, z=None, ckpt=None, stream=None):
        """Whole-signal forward from zero state; returns (z, checkpoints)."""
        import torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.dim() == 2
        n = int(x.shape[1])
        if z is None:
            z = torch.empty((self.n_detectors, self.n_templates, n), dtype=torch.complex64,
                            device=x.device)
        if ckpt is None:
            ckpt = torch.empty(self.ckpt_count(n), dtype=torch.complex64, device=x.device)
        _check("spiir_forward", load().spiir_forward(self._h, x.data_ptr(), n, z.data_ptr(),
                                                       ckpt.data_ptr(), _stream_ptr(stream)))
        return z, ckpt

    def backward(self, x, grad_z, ckpt, grad_a=None, grad_b=None, stream=None):
        """Gradients (complex64 [F], original filter order) of a loss with dL/dz = grad_z."""
        import torch
        assert grad_z.dtype == torch.complex64 and grad_z.is_contiguous()
        n = int(x.shape[1])
        F = int(self._offsets[-1])
        if grad_a is None:
            grad_a = torch.empty(F, dtype=torch.complex64, device=x.device)
            grad_b = torch.empty(F, dtype=torch.complex64, device=x.device)
        _check("spiir_backward", load().spiir_backward(
            self._h, x.data_ptr(), n, grad_z.data_ptr(), ckpt.data_ptr(), grad_a.data_ptr(),
            grad_b.data_ptr(), _stream_ptr(stream)))
        return grad_a, grad_b

    def set_coeffs(self, a, b, stream=None):
        """Load coefficients from cuda complex64 tensors [F] (original filter order)."""
        import torch
        assert a.dtype == torch.complex64 and b.dtype == torch.complex64
        a = a.contiguous(); b = b.contiguous()
        _check("spiir_bank_set_coeffs", load().spiir_bank_set_coeffs(
            self._h, a.data_ptr(), b.data_ptr(), _stream_ptr(stream)))

    def noise_power(self) -> np.ndarray:
        """E|z_t|^2 per template for unit-variance white input (FP64, host)."""
        out = np.empty(self.n_templates, dtype=np.float64)
        _check("spiir_bank_noise_power", load().spiir_bank_noise_power(self._h, out.ctypes.data))
        return out

    def trigger_weights(self, stream=None):
        """2 / E|z_t|^2 per template (cuda float32 [T]), computed on the GPU from the
        bank's current coefficients (Sec. II.C.1 normalisation)."""
        import torch
        w = torch.empty(self.n_templates, dtype=torch.float32, device="cuda")
        _check("spiir_bank_trigger_weights",
               load().spiir_bank_trigger_weights(self._h, w.data_ptr(), _stream_ptr(stream)))
        return w

    def autocorr(self, nj: int = 175, stream=None):
        """R_t[j], j = 0..nj, of each template's impulse response (Sec. II.C.1): cuda
        complex128 [T][nj+1], computed in closed form on the GPU (synchronous)."""
        import torch
        R = torch.empty((self.n_templates, nj + 1), dtype=torch.complex128, device="cuda")
        _check("spiir_bank_autocorr",
               load().spiir_bank_autocorr(self._h, int(nj), R.data_ptr(), _stream_ptr(stream)))
        return R

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


def _make_autograd():
    import torch

    class SpiirFilterFn(torch.autograd.Function):
        """z = SPIIR bank(a, b) applied to x from zero state, differentiable in a and b.

        The backward pass is the library's reverse-time adjoint scan
        (``spiir_backward``) with checkpointed states.
        """

        @staticmethod
        def forward(ctx, a, b, x, bank):
            bank.set_coeffs(a.detach(), b.detach())
            z, ckpt = bank.forward(x)
            ctx.save_for_backward(a.detach(), b.detach(), x, ckpt)
            ctx.bank = bank
            return z

        @staticmethod
        def backward(ctx, grad_z):
            a, b, x, ckpt = ctx.saved_tensors
            bank = ctx.bank
            bank.set_coeffs(a, b)
            ga, gb = bank.backward(x, grad_z.contiguous(), ckpt)
            return ga, gb, None, None

    return SpiirFilterFn


_autograd_fn = None


def spiir_filter(a, b, x, bank: SpiirBank):
    """Differentiable SNR series z[D][T][n] of the bank with coefficients (a, b)."""
    global _autograd_fn
    if _autograd_fn is None:
        _autograd_fn = _make_autograd()
    return _autograd_fn.apply(a, b, x, bank)


def triggers(z, weight, threshold: float = 4.0, window: int = 2048, work=None, stream=None):
    """Single-detector candidates (Sec. II.C.1) from z (cuda complex64 [D][T][n]).

    ``weight`` cuda float32 [T] (2 / E|z_t|^2).  Returns (snr, index), each [D][T][W].
    """
    import torch
    assert z.is_cuda and z.dtype == torch.complex64 and z.is_contiguous() and z.dim() == 3
    D, T, n = (int(v) for v in z.shape)
    W = (n + window - 1) // window
    if work is None:
        work = torch.empty((D, T, W), dtype=torch.int64, device=z.device)
    snr = torch.empty((D, T, W), dtype=torch.float32, device=z.device)
    idx = torch.empty((D, T, W), dtype=torch.int32, device=z.device)
    _check("spiir_triggers", load().spiir_triggers(z.data_ptr(), D, T, n, weight.data_ptr(),
                                                   float(threshold), int(window), work.data_ptr(),
                                                   snr.data_ptr(), idx.data_ptr(), _stream_ptr(stream)))
    return snr, idx


def triggers_noalloc(z, weight, threshold: float = 4.0, window: int = 2048, out=None,
                     stream=None):
    """``triggers`` through the entry point that allocates nothing: the key slots are
    the library's per-device workspace.  ``out`` = (snr, index) preallocated
    [D][T][W] tensors, else they are allocated here (by torch, outside the call)."""
    import torch
    assert z.is_cuda and z.dtype == torch.complex64 and z.is_contiguous() and z.dim() == 3
    D, T, n = (int(v) for v in z.shape)
    W = (n + window - 1) // window
    if out is None:
        out = (torch.empty((D, T, W), dtype=torch.float32, device=z.device),
               torch.empty((D, T, W), dtype=torch.int32, device=z.device))
    snr, idx = out
    assert snr.dtype == torch.float32 and idx.dtype == torch.int32
    assert snr.is_contiguous() and idx.is_contiguous() and snr.numel() >= D * T * W
    assert idx.numel() >= D * T * W
    _check("spiir_triggers_noalloc",
           load().spiir_triggers_noalloc(z.data_ptr(), D, T, n, weight.data_ptr(), float(threshold),
                                         int(window), snr.data_ptr(), idx.data_ptr(),
                                         _stream_ptr(stream)))
    return snr, idx


def xi2(z, index, R, nj: int, stream=None):
    """Signal-consistency statistic (Sec. II.C.1) at candidate samples.

    ``z`` cuda complex64 [D][T][n]; ``index`` cuda int32 [D][T][W] (candidate samples,
    -1 = none, e.g. from ``triggers``); ``R`` cuda complex128 [T][nj+1] from
    ``SpiirBank.autocorr(nj)``.  Returns cuda float32 [D][T][W], NaN where undefined.
    """
    import torch
    assert z.is_cuda and z.dtype == torch.complex64 and z.is_contiguous() and z.dim() == 3
    assert index.dtype == torch.int32 and index.is_contiguous() and index.dim() == 3
    assert R.dtype == torch.complex128 and R.is_contiguous() and R.shape[-1] == nj + 1
    D, T, n = (int(v) for v in z.shape)
    assert index.shape[0] == D and index.shape[1] == T and R.shape[0] == T
    W = int(index.shape[2])
    out = torch.empty((D, T, W), dtype=torch.float32, device=z.device)
    _check("spiir_xi2", load().spiir_xi2(z.data_ptr(), D, T, n, index.data_ptr(), W, R.data_ptr(),
                                         int(nj), out.data_ptr(), _stream_ptr(stream)))
    return out


def xi2_network(z, index, pix, tau, R, nj: int, stream=None):
    """xi^2 of every detector at coherent candidates and their mean xi^2_C (Sec. II.C.1).

    ``z`` cuda complex64 [D][T][n]; ``index``, ``pix`` cuda int32 [D][T][W] (candidate
    samples and their sky directions, -1 = none); ``tau`` cuda int32 [P][D]; ``R`` cuda
    complex128 [T][nj+1].  Returns (xi2_det [D][T][W][D], xi2_c [D][T][W]) float32.
    """
    import torch
    assert z.is_cuda and z.dtype == torch.complex64 and z.is_contiguous() and z.dim() == 3
    D, T, n = (int(v) for v in z.shape)
    W = int(index.shape[2])
    for a, dt in ((index, torch.int32), (pix, torch.int32), (tau, torch.int32)):
        assert a.is_cuda and a.dtype == dt and a.is_contiguous()
    assert tuple(index.shape) == (D, T, W) and tuple(pix.shape) == (D, T, W)
    assert tau.dim() == 2 and tau.shape[1] == D
    assert R.dtype == torch.complex128 and R.is_contiguous() and tuple(R.shape) == (T, nj + 1)
    per = torch.empty((D, T, W, D), dtype=torch.float32, device=z.device)
    mean = torch.empty((D, T, W), dtype=torch.float32, device=z.device)
    _check("spiir_xi2_network", load().spiir_xi2_network(
        z.data_ptr(), D, T, n, index.data_ptr(), pix.data_ptr(), W, tau.data_ptr(),
        int(tau.shape[0]), R.data_ptr(), int(nj), per.data_ptr(), mean.data_ptr(),
        _stream_ptr(stream)))
    return per, mean


def coherent(z, index, U, tau, shifts, stream=None):
    """Coherent and null SNR^2 (Sec. II.C.1) of candidates over sky directions.

    ``z`` cuda complex64 [D][T][n]; ``index`` cuda int32 [D][T][W]; ``U`` cuda float32
    [P][D][D]; ``tau`` cuda int32 [P][D]; ``shifts`` cuda int32 [K][D].  Returns
    (rho_C^2, direction, rho_N^2), each [D][T][W][K].
    """
    import torch
    assert z.is_cuda and z.dtype == torch.complex64 and z.is_contiguous() and z.dim() == 3
    D, T, n = (int(v) for v in z.shape)
    W = int(index.shape[2])
    P, K = int(U.shape[0]), int(shifts.shape[0])
    for a, dt in ((index, torch.int32), (U, torch.float32), (tau, torch.int32), (shifts, torch.int32)):
        assert a.is_cuda and a.dtype == dt and a.is_contiguous()
    assert tuple(U.shape) == (P, D, D) and tuple(tau.shape) == (P, D) and shifts.shape[1] == D
    snr2 = torch.empty((D, T, W, K), dtype=torch.float32, device=z.device)
    null2 = torch.empty_like(snr2)
    pix = torch.empty((D, T, W, K), dtype=torch.int32, device=z.device)
    _check("spiir_coherent", load().spiir_coherent(z.data_ptr(), D, T, n, index.data_ptr(), W,
                                                   U.data_ptr(), tau.data_ptr(), P,
                                                   shifts.data_ptr(), K, snr2.data_ptr(),
                                                   pix.data_ptr(), null2.data_ptr(),
                                                   _stream_ptr(stream)))
    return snr2, pix, null2

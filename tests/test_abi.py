"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects invalid arguments on the host before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2011_06787_amd import spiir

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(spiir_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = spiir.load()
    decl = declared_functions()
    assert decl, "no declarations found"
    for name in sorted(decl):
        assert hasattr(lib, name), name
    assert decl == set(spiir.EXPORTS)


def test_opts_default():
    o = spiir.default_opts()
    assert o.n_detectors == 1 and o.max_chunk == 2048 and o.mode == spiir.MODE_FP32_SCAN
    assert o.filters_per_lane == 4 and o.block_len == 128 and o.long_pole_abs_a == 0.999


def _create(offsets, a, b, d, **kw):
    lib = spiir.load()
    o = spiir.default_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    offsets = np.ascontiguousarray(offsets, np.int32)
    a = np.ascontiguousarray(a, np.complex64)
    b = np.ascontiguousarray(b, np.complex64)
    d = np.ascontiguousarray(d, np.int32)
    h = ctypes.c_void_p()
    st = lib.spiir_bank_create(len(offsets) - 1, offsets.ctypes.data, a.ctypes.data, b.ctypes.data,
                               d.ctypes.data, ctypes.byref(o), None, ctypes.byref(h))
    return st, h


GOOD = dict(offsets=[0, 2], a=[0.5 + 0.1j, 0.9j], b=[1 + 0j, 0.5j], d=[0, 3])


@pytest.mark.parametrize("change, expect", [
    (dict(a=[1.0 + 0j, 0.9j]), spiir.SPIIR_E_INVAL),            # |a| = 1
    (dict(a=[0.8 + 0.7j, 0.9j]), spiir.SPIIR_E_INVAL),          # |a| > 1
    (dict(a=[np.nan, 0.9j]), spiir.SPIIR_E_INVAL),              # non-finite
    (dict(b=[np.inf, 0.5j]), spiir.SPIIR_E_INVAL),
    (dict(d=[-1, 3]), spiir.SPIIR_E_INVAL),                     # negative delay
    (dict(offsets=[1, 2]), spiir.SPIIR_E_INVAL),                # offsets[0] != 0
    (dict(offsets=[0, 2, 1]), spiir.SPIIR_E_INVAL),             # decreasing
    (dict(max_delay=2), spiir.SPIIR_E_INVAL),                   # delay 3 > max_delay
    (dict(max_delay=9000), spiir.SPIIR_E_INVAL),                # above the supported range
    (dict(n_detectors=0), spiir.SPIIR_E_INVAL),
    (dict(max_chunk=0), spiir.SPIIR_E_INVAL),
    (dict(filters_per_lane=3), spiir.SPIIR_E_INVAL),
    (dict(time_tile=24), spiir.SPIIR_E_INVAL),                  # not a multiple of 16
    (dict(time_tile=8192), spiir.SPIIR_E_INVAL),
    (dict(balance_wgs=9), spiir.SPIIR_E_INVAL),
    (dict(balance_wgs=-1), spiir.SPIIR_E_INVAL),
    (dict(mode=7), spiir.SPIIR_E_INVAL),
    (dict(mode=1, block_len=96), spiir.SPIIR_E_INVAL),          # unsupported block length
    (dict(mode=1, max_chunk=1000), spiir.SPIIR_E_INVAL),        # not a multiple of L
    (dict(peak_window=4096), spiir.SPIIR_E_INVAL),              # larger than max_chunk
])
def test_create_rejects_invalid_arguments(change, expect):
    args = dict(GOOD)
    opt_keys = {"max_delay", "n_detectors", "max_chunk", "filters_per_lane", "mode", "peak_window",
                "time_tile", "block_len", "balance_wgs"}
    opts = {k: v for k, v in change.items() if k in opt_keys}
    args.update({k: v for k, v in change.items() if k not in opt_keys})
    offsets = args["offsets"]
    if offsets == [0, 2, 1]:
        args["a"] = args["a"][:2]
    st, h = _create(args["offsets"], args["a"], args["b"], args["d"], **opts)
    assert st == expect, spiir.last_error()
    assert not h.value
    assert spiir.last_error() != ""


def test_null_and_shape_errors_without_gpu():
    lib = spiir.load()
    assert lib.spiir_bank_create(1, None, None, None, None, None, None,
                                 ctypes.byref(ctypes.c_void_p())) == spiir.SPIIR_E_INVAL
    assert lib.spiir_filter_chunk(None, None, 16, None, None, None, None) == spiir.SPIIR_E_INVAL
    assert lib.spiir_bank_reset(None, None) == spiir.SPIIR_E_INVAL
    assert lib.spiir_bank_destroy(None) == spiir.SPIIR_OK
    assert lib.spiir_peaks(None, 4, 16, 0, None, None, None) == spiir.SPIIR_E_INVAL   # window 0
    assert lib.spiir_peaks(None, 4, 16, 8, None, None, None) == spiir.SPIIR_E_INVAL   # NULL buffers
    assert lib.spiir_bank_autocorr(None, 10, None, None) == spiir.SPIIR_E_INVAL
    assert lib.spiir_xi2(None, 1, 2, 100, None, 1, None, 0, None, None) == spiir.SPIIR_E_INVAL  # nj 0
    assert lib.spiir_xi2(None, 1, 2, 100, None, 1, None, 5, None, None) == spiir.SPIIR_E_INVAL  # NULLs
    assert lib.spiir_xi2(None, 0, 2, 100, None, 1, None, 5, None, None) == spiir.SPIIR_OK      # empty
    args = (None, 1, None, None, 4, None, 1, None, None, None, None)
    assert lib.spiir_coherent(None, 1, 2, 100, *args) == spiir.SPIIR_E_INVAL    # one detector
    assert lib.spiir_coherent(None, 9, 2, 100, *args) == spiir.SPIIR_E_INVAL    # too many
    assert lib.spiir_coherent(None, 3, 2, 100, *args) == spiir.SPIIR_E_INVAL    # NULL buffers
    f = lib.spiir_xi2_network
    assert f(None, 0, 2, 100, None, None, 1, None, 4, None, 5, None, None, None) == spiir.SPIIR_E_INVAL  # n_det 0
    assert f(None, 9, 2, 100, None, None, 1, None, 4, None, 5, None, None, None) == spiir.SPIIR_E_INVAL  # 9 detectors
    assert f(None, 3, 2, 100, None, None, 1, None, 4, None, 0, None, None, None) == spiir.SPIIR_E_INVAL  # nj 0
    assert f(None, 3, 2, 100, None, None, 1, None, 4, None, 5, None, None, None) == spiir.SPIIR_E_INVAL  # NULLs
    assert f(None, 3, 0, 100, None, None, 1, None, 4, None, 5, None, None, None) == spiir.SPIIR_OK      # empty
    assert lib.spiir_peaks(None, 0, 16, 8, None, None, None) == spiir.SPIIR_OK        # empty no-op
    assert lib.spiir_peaks(None, -1, 16, 8, None, None, None) == spiir.SPIIR_E_INVAL


def test_product_path_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(spiir, "_lib", None)
    monkeypatch.setattr(spiir, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="libspiir.so not found"):
        spiir.load()


def test_triggers_noalloc_rejects_oversize_and_bad_arguments_without_gpu():
    # the workspace holds 2^20 key slots: one more is refused before anything is enqueued
    lib = spiir.load()
    f = lib.spiir_triggers_noalloc
    dummy = ctypes.c_void_p(16)   # never dereferenced: every case fails on the host
    assert f(dummy, 2, 1 << 19, 2049, dummy, 4.0, 2048, dummy, dummy, None) == spiir.SPIIR_E_INVAL
    assert "workspace" in spiir.last_error()
    assert f(dummy, 1, (1 << 20) + 1, 16, dummy, 4.0, 16, dummy, dummy, None) == spiir.SPIIR_E_INVAL
    assert f(dummy, 1, 2, 100, dummy, 4.0, 0, dummy, dummy, None) == spiir.SPIIR_E_INVAL   # window 0
    assert f(dummy, 1, 2, 100, dummy, -1.0, 8, dummy, dummy, None) == spiir.SPIIR_E_INVAL  # threshold
    assert f(None, 1, 2, 100, None, 4.0, 8, None, None, None) == spiir.SPIIR_E_INVAL      # NULLs
    assert f(None, 0, 2, 100, None, 4.0, 8, None, None, None) == spiir.SPIIR_OK           # empty

"""FP64 CPU oracle for the SPIIR filter-bank hot path (test infrastructure).

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg use this package.  The HIP library never imports, links or calls it, and it
never calls the HIP library: the two share nothing but the seeded inputs of
``synth``.

What it computes (each function cites the passage it follows):

* ``filter``         Eq. zk (Section II.B.1), read as a sum of independent
                     first-order complex IIR filters, in FP64.
* ``filter_stream``  the same, in consecutive chunks with state and input
                     history carried (data arrives in packets, Section II.A).
* ``peaks``          largest |z| per template per window and its index
                     (trigger selection, Section II.C.1), FP64.
* ``peaks_f32``      the same decision taken in float32 on a complex64 series.
* ``grad``           gradient of a real loss w.r.t. a_k, b_k by forward-mode
                     sensitivities.
* ``overlap_grad``   overlap (Eq. overlap) between the summed impulse response
                     and a target, and its closed-form gradient.

Complex gradients follow the convention dL/dRe + i dL/dIm.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spiir_oracle.c")
_LIB = os.path.join(_HERE, "libspiir_oracle.so")
_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F64 = ctypes.c_double


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.spo_filter.argtypes = [_I32, _P, _P, _P, _P, _I32, _I64, _P, _I64, _P, _P, _P]
        lib.spo_peaks.argtypes = [_I64, _I64, _I64, _P, _P, _P, _P]
        lib.spo_grad.argtypes = [_I32, _P, _P, _P, _P, _I32, _I64, _P, _P, _P, _P]
        lib.spo_overlap_grad.argtypes = [_I32, _P, _P, _P, _P, _I64, _P, _I32, _F64, _P, _P, _P]
        for f in (lib.spo_filter, lib.spo_peaks, lib.spo_grad, lib.spo_overlap_grad):
            f.restype = ctypes.c_int
        lib.spo_noise_power.argtypes = [_I32, _P, _P, _P, _P, _P]
        lib.spo_autocorr.argtypes = [_I32, _P, _P, _P, _P, _I32, _P]
        lib.spo_noise_power.restype = ctypes.c_int
        lib.spo_threads.argtypes = []
        lib.spo_set_threads.argtypes = [_I32]
        lib.spo_set_threads.restype = None
        lib.spo_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(arr: Optional[np.ndarray]):
    return None if arr is None else arr.ctypes.data_as(ctypes.c_void_p)


def _bank_arrays(bank):
    """CSR offsets, complex128 a and b (exact promotion), int32 delays."""
    offsets = np.ascontiguousarray(bank.offsets, dtype=np.int32)
    a = np.ascontiguousarray(bank.a, dtype=np.complex128)
    b = np.ascontiguousarray(bank.b, dtype=np.complex128)
    d = np.ascontiguousarray(bank.d, dtype=np.int32)
    return offsets, a, b, d


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments (status {rc})")


def filter(bank, x: np.ndarray, hist: Optional[np.ndarray] = None,
           state: Optional[np.ndarray] = None) -> np.ndarray:
    """complex128 z[D][T][n] for real input x[D][n] (Eq. zk, Section II.B.1).

    ``hist`` ([D][H]) holds the H samples just before x (zero before that);
    ``state`` (complex128 [D][F]) holds y_k before x and is updated in place to
    y_k at the last sample.  Both default to a stream starting at x.  Inputs
    are promoted to float64 (exactly, for float32 data).
    """
    offsets, a, b, d = _bank_arrays(bank)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    n_det, n = x.shape
    hist_len = 0
    if hist is not None:
        hist = np.ascontiguousarray(np.atleast_2d(hist), dtype=np.float64)
        assert hist.shape[0] == n_det
        hist_len = hist.shape[1]
    if state is not None:
        assert state.dtype == np.complex128 and state.flags.c_contiguous
        assert state.shape == (n_det, bank.n_filters)
    z = np.empty((n_det, bank.n_templates, n), dtype=np.complex128)
    rc = _load().spo_filter(bank.n_templates, _ptr(offsets), _ptr(a), _ptr(b), _ptr(d), n_det, n,
                            _ptr(x), hist_len, _ptr(hist), _ptr(state), _ptr(z))
    _check(rc, "filter")
    return z


def filter_stream(bank, x: np.ndarray, chunk: int) -> np.ndarray:
    """``filter`` over x[D][N] in consecutive chunks with carried state/history."""
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    n_det, n_total = x.shape
    hist_len = max(bank.max_delay, 1)
    hist = np.zeros((n_det, hist_len), dtype=np.float64)
    state = np.zeros((n_det, bank.n_filters), dtype=np.complex128)
    out = np.empty((n_det, bank.n_templates, n_total), dtype=np.complex128)
    for lo in range(0, n_total, chunk):
        hi = min(lo + chunk, n_total)
        out[:, :, lo:hi] = filter(bank, x[:, lo:hi], hist=hist, state=state)
        hist = np.concatenate([hist, x[:, lo:hi]], axis=1)[:, -hist_len:].copy()
    return out


def peaks(z: np.ndarray, window: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Per row of z[..., n] and window: (max |z|, argmax in window, top-2 margin), FP64.

    Ties in |z|^2 go to the lowest index.  Margin is (p1 - p2)/p1 over |z|.
    """
    z = np.ascontiguousarray(z, dtype=np.complex128)
    lead, n = z.shape[:-1], z.shape[-1]
    rows = int(np.prod(lead)) if lead else 1
    n_win = (n + window - 1) // window
    peak = np.empty(rows * n_win, dtype=np.float64)
    arg = np.empty(rows * n_win, dtype=np.int32)
    margin = np.empty(rows * n_win, dtype=np.float64)
    rc = _load().spo_peaks(rows, n, window, _ptr(z), _ptr(peak), _ptr(arg), _ptr(margin))
    _check(rc, "peaks")
    shape = tuple(lead) + (n_win,)
    return peak.reshape(shape), arg.reshape(shape), margin.reshape(shape)


def peaks_f32(z: np.ndarray, window: int) -> Tuple[np.ndarray, np.ndarray]:
    """Peak decision taken in float32 on a complex64 series.

    |z|^2 = re*re + im*im with each product and the sum rounded to float32 (no
    fused multiply-add); the largest per window, lowest index on ties; the peak
    value is the float32 square root of the winning |z|^2.
    """
    z = np.ascontiguousarray(z, dtype=np.complex64)
    lead, n = z.shape[:-1], z.shape[-1]
    n_win = (n + window - 1) // window
    re = z.real.astype(np.float32)
    im = z.imag.astype(np.float32)
    p = (re * re).astype(np.float32) + (im * im).astype(np.float32)
    pad = n_win * window - n
    if pad:
        p = np.concatenate([p, np.full(tuple(lead) + (pad,), -np.inf, np.float32)], axis=-1)
    p = p.reshape(tuple(lead) + (n_win, window))
    arg = np.argmax(p, axis=-1).astype(np.int32)          # first occurrence on ties
    best = np.take_along_axis(p, arg[..., None].astype(np.int64), axis=-1)[..., 0]
    return np.sqrt(best).astype(np.float32), arg


def grad(bank, x: np.ndarray, gz: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """(grad_a, grad_b) complex128 [F] of a loss with dL/dz = gz[D][T][n].

    The forward pass starts from zero state and zero history.
    """
    offsets, a, b, d = _bank_arrays(bank)
    x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
    n_det, n = x.shape
    gz = np.ascontiguousarray(gz, dtype=np.complex128).reshape(n_det, bank.n_templates, n)
    ga = np.empty(bank.n_filters, dtype=np.complex128)
    gb = np.empty(bank.n_filters, dtype=np.complex128)
    rc = _load().spo_grad(bank.n_templates, _ptr(offsets), _ptr(a), _ptr(b), _ptr(d), n_det, n,
                          _ptr(x), _ptr(gz), _ptr(ga), _ptr(gb))
    _check(rc, "grad")
    return ga, gb


def overlap_grad(bank, target: np.ndarray, mode: int = 0, scale: Optional[float] = None):
    """(overlap[T], grad_a[F], grad_b[F]) for loss = scale * sum_t (1 - O_t).

    ``target`` is complex [T][n]; the impulse response is taken over the same
    n samples.  ``mode`` 0 uses |<g, u>| (phase-maximised), 1 uses Re<g, u>.
    ``scale`` defaults to 1/T (the mean over templates).
    """
    offsets, a, b, d = _bank_arrays(bank)
    target = np.ascontiguousarray(target, dtype=np.complex128)
    n_t, n = target.shape
    assert n_t == bank.n_templates
    if scale is None:
        scale = 1.0 / max(n_t, 1)
    ov = np.empty(n_t, dtype=np.float64)
    ga = np.empty(bank.n_filters, dtype=np.complex128)
    gb = np.empty(bank.n_filters, dtype=np.complex128)
    rc = _load().spo_overlap_grad(bank.n_templates, _ptr(offsets), _ptr(a), _ptr(b), _ptr(d), n,
                                  _ptr(target), int(mode), float(scale), _ptr(ov), _ptr(ga),
                                  _ptr(gb))
    _check(rc, "overlap_grad")
    return ov, ga, gb


def noise_power(bank) -> np.ndarray:
    """E|z_t|^2 for unit-variance white input (closed form, FP64), per template."""
    offsets, a, b, d = _bank_arrays(bank)
    out = np.empty(bank.n_templates, dtype=np.float64)
    rc = _load().spo_noise_power(bank.n_templates, _ptr(offsets), _ptr(a), _ptr(b), _ptr(d), _ptr(out))
    _check(rc, "noise_power")
    return out


def triggers(z: np.ndarray, weight: np.ndarray, threshold: float, window: int):
    """Trigger selection of Section II.C.1 on z[D][T][n] (complex64), decided in float32.

    rho2_t[n] = (re*re + im*im) * weight_t, each product and the sum rounded to
    float32 (weight_t = 2 / E|z_t|^2 normalises each quadrature to unit variance).
    For each sample the template with the largest rho2 (lowest index on ties) is a
    candidate if rho2 > threshold^2; per template and window of ``window`` samples the
    candidate with the largest rho2 (lowest sample on ties) is kept.  Returns
    (snr[D][T][W] float32, 0 where none; index[D][T][W] int32 sample in the packet,
    -1 where none), snr = sqrt(rho2) in float32.
    """
    z = np.ascontiguousarray(z, dtype=np.complex64)
    D, T, n = z.shape
    W = (n + window - 1) // window
    re = z.real.astype(np.float32)
    im = z.imag.astype(np.float32)
    w = np.asarray(weight, dtype=np.float32)
    p = ((re * re).astype(np.float32) + (im * im).astype(np.float32)).astype(np.float32)
    r2 = (p * w[None, :, None]).astype(np.float32)
    thr2 = np.float32(threshold) * np.float32(threshold)
    snr = np.zeros((D, T, W), dtype=np.float32)
    idx = np.full((D, T, W), -1, dtype=np.int32)
    for det in range(D):
        tstar = np.argmax(r2[det], axis=0)               # lowest template on ties
        best = r2[det][tstar, np.arange(n)]
        for i in np.nonzero(best > thr2)[0]:
            t, wdx = int(tstar[i]), int(i) // window
            if best[i] > (snr[det, t, wdx] if idx[det, t, wdx] >= 0 else np.float32(-1)):
                snr[det, t, wdx] = best[i]
                idx[det, t, wdx] = int(i)
    got = idx >= 0
    snr[got] = np.sqrt(snr[got]).astype(np.float32)
    return snr, idx


def autocorr(bank, nj: int) -> np.ndarray:
    """R_t[j] = sum_m u_t[m+j] conj(u_t[m]), j = 0..nj, of each template's impulse
    response u_t (closed form, FP64): the correlation of a template with itself used
    by the signal-consistency statistic of Section II.C.1.  complex128 [T][nj+1]."""
    offsets, a, b, d = _bank_arrays(bank)
    out = np.empty((bank.n_templates, nj + 1), dtype=np.complex128)
    rc = _load().spo_autocorr(bank.n_templates, _ptr(offsets), _ptr(a), _ptr(b), _ptr(d), int(nj),
                              _ptr(out))
    _check(rc, "autocorr")
    return out


def xi2(z: np.ndarray, index: np.ndarray, R: np.ndarray, nj: int) -> np.ndarray:
    """The signal-consistency statistic of Section II.C.1 at candidate samples.

    For row (detector, template) and candidate sample c = index[d, t, w] (-1 = none):
      xi2 = sum_{j=-nj..nj} |v[c+j] - v[c] A[j]|^2 / sum_{j=-nj..nj} (2 - 2|A[j]|^2)
    with A[j] = R_t[j] / R_t[0] (A[-j] = conj(A[j])) and v = z * sqrt(2 / R_t[0]), the SNR
    normalised to unit variance per quadrature for unit white input (so that a
    noise-only series gives a reduced chi-square of mean 1).  NaN where there is no
    candidate or c +- nj leaves the series.  z: complex [D][T][n]; R: [T][>= nj+1].
    Plain FP64 loops.
    """
    z = np.asarray(z, dtype=np.complex128)
    D, T, n = z.shape
    out = np.full(index.shape, np.nan, dtype=np.float64)
    for t in range(T):
        r0 = R[t, 0].real
        A = np.concatenate([np.conj(R[t, nj:0:-1]), R[t, :nj + 1]]) / r0     # j = -nj..nj
        den = np.sum(2.0 - 2.0 * np.abs(A) ** 2)
        scale = np.sqrt(2.0 / r0)
        for det in range(D):
            for w in range(index.shape[2]):
                c = int(index[det, t, w])
                if c < 0 or c - nj < 0 or c + nj >= n:
                    continue
                v = z[det, t, c - nj:c + nj + 1] * scale
                out[det, t, w] = np.sum(np.abs(v - v[nj] * A) ** 2) / den
    return out


def xi2_network(z: np.ndarray, index: np.ndarray, pix: np.ndarray, tau: np.ndarray,
                R: np.ndarray, nj: int):
    """xi^2 of every detector at a coherent candidate and their mean xi^2_C (Section
    II.C.1: xi^2_C = (1/N_d) sum_I xi_I^2).

    For the candidate of detector I, template t, window w at sample c = index[I, t, w]
    with sky direction p = pix[I, t, w] (the coherent stage's best direction), detector J
    is read at its arrival time in that direction, s_J = c + tau[p, J] - tau[p, I], and
      xi_J^2 = sum_{j=-nj..nj} |v_J[s_J+j] - v_J[s_J] A[j]|^2 / sum_{j=-nj..nj} (2 - 2|A[j]|^2)
    with A[j] = R_t[j] / R_t[0] (A[-j] = conj(A[j])) and v_J = z[J, t] * sqrt(2 / R_t[0]).
    Returns (xi2_det float64 [D][T][W][D] (last axis J), xi2_c float64 [D][T][W]); NaN
    where there is no candidate (c < 0 or p < 0) or some s_J +- nj leaves [0, n).
    Plain FP64 loops.
    """
    z = np.asarray(z, dtype=np.complex128)
    D, T, n = z.shape
    W = index.shape[2]
    per = np.full((D, T, W, D), np.nan)
    mean = np.full((D, T, W), np.nan)
    for t in range(T):
        r0 = R[t, 0].real
        A = np.concatenate([np.conj(R[t, nj:0:-1]), R[t, :nj + 1]]) / r0     # j = -nj..nj
        den = np.sum(2.0 - 2.0 * np.abs(A) ** 2)
        scale = np.sqrt(2.0 / r0)
        for I in range(D):
            for w in range(W):
                c, p = int(index[I, t, w]), int(pix[I, t, w])
                if c < 0 or p < 0:
                    continue
                s = [c + int(tau[p, J]) - int(tau[p, I]) for J in range(D)]
                if min(s) - nj < 0 or max(s) + nj >= n:
                    continue
                vals = []
                for J in range(D):
                    v = z[J, t, s[J] - nj:s[J] + nj + 1] * scale
                    vals.append(np.sum(np.abs(v - v[nj] * A) ** 2) / den)
                per[I, t, w, :] = vals
                mean[I, t, w] = sum(vals) / D
    return per, mean


def coherent_map(z: np.ndarray, index: np.ndarray, U: np.ndarray, tau: np.ndarray,
                 shifts: np.ndarray):
    """Coherent and null SNR^2 of every candidate at every sky direction and time shift
    (Section II.C.1, Eq. llr_form, and the null statistic of the appendix), FP64 loops.

    The z_I of Eq. llr_form form a vector (the per-detector inner products of the
    appendix); a diagonal matrix there would drop the phase coherence.  For the
    candidate of detector I, template t, window w at sample c = index[I, t, w], shift k
    and direction p, detector J contributes v_J = z[J, t, s_J] with
        s_J = c + tau[p, J] - tau[p, I] + shifts[k, (J - I) mod D] - shifts[k, 0]
    (background events shift the other detectors' series relative to the candidate's
    detector, column r of the shift table being the detector r places after it),
    and with U = U[p]:
        rho_C^2 = sum_{i < 2} |sum_J U[J, i] v_J|^2      (projection on the signal plane)
        rho_N^2 = sum_{i >= 2} |sum_J U[J, i] v_J|^2     (projection on the null space).
    Returns (rho_C^2, rho_N^2) as float64 [D][T][W][K][P], NaN where there is no
    candidate or some s_J (any p) falls outside [0, n).
    """
    z = np.asarray(z, dtype=np.complex128)
    U = np.asarray(U, dtype=np.float64)
    D, T, n = z.shape
    W, K, P = index.shape[2], shifts.shape[0], U.shape[0]
    rc = np.full((D, T, W, K, P), np.nan)
    rn = np.full((D, T, W, K, P), np.nan)
    for I in range(D):
        for t in range(T):
            for w in range(W):
                c = int(index[I, t, w])
                if c < 0:
                    continue
                rel = [(J - I) % D for J in range(D)]
                for k in range(K):
                    sk = np.array([shifts[k, r] - shifts[k, 0] for r in rel])
                    s = c + (tau - tau[:, I:I + 1]) + sk[None, :]  # [P][D]
                    if s.min() < 0 or s.max() >= n:
                        continue
                    for p in range(P):
                        v = np.array([z[J, t, s[p, J]] for J in range(D)])
                        proj = U[p].T @ v
                        rc[I, t, w, k, p] = np.sum(np.abs(proj[:2]) ** 2)
                        rn[I, t, w, k, p] = np.sum(np.abs(proj[2:]) ** 2)
    return rc, rn


def coherent(z, index, U, tau, shifts):
    """Per candidate and time shift: the largest rho_C^2 over the sky directions, its
    direction (lowest on ties) and rho_N^2 there.  float64 / int32 [D][T][W][K];
    NaN / -1 where coherent_map is undefined."""
    rc, rn = coherent_map(z, index, U, tau, shifts)
    ok = ~np.isnan(rc[..., 0])
    pix = np.full(ok.shape, -1, dtype=np.int32)
    best = np.full(ok.shape, np.nan)
    null = np.full(ok.shape, np.nan)
    arg = np.argmax(np.where(np.isnan(rc), -np.inf, rc), axis=-1)
    pix[ok] = arg[ok]
    best[ok] = np.take_along_axis(rc, arg[..., None], axis=-1)[..., 0][ok]
    null[ok] = np.take_along_axis(rn, arg[..., None], axis=-1)[..., 0][ok]
    return best, pix, null


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().spo_threads())


def set_threads(n: int) -> None:
    """Number of OpenMP threads for the oracle's parallel loops from now on."""
    _load().spo_set_threads(int(n))


def rel_err(z_test: np.ndarray, z_ref: np.ndarray) -> np.ndarray:
    """Per-series relative L2 error ||z_test - z_ref|| / ||z_ref|| over the last axis."""
    zt = np.asarray(z_test, dtype=np.complex128)
    zr = np.asarray(z_ref, dtype=np.complex128)
    num = np.sqrt(np.sum(np.abs(zt - zr) ** 2, axis=-1))
    den = np.sqrt(np.sum(np.abs(zr) ** 2, axis=-1))
    return num / np.where(den > 0, den, 1.0)

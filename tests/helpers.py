"""Comparison helpers shared by the GPU parity tests (numpy + oracle only)."""
import numpy as np

import oracle


def check_peaks(gpu_peak, gpu_arg, z_gpu, z_ref, window):
    """Check GPU peaks/argmax against the FP64 oracle series z_ref.

    Where the oracle's gap between the best and second-best |z| in a window
    exceeds twice the largest |z_gpu - z_ref| in that window (so that the error
    cannot reorder them), the GPU index must equal the oracle's.  Elsewhere the
    GPU index must point at a sample whose oracle |z| is within that error band
    of the oracle maximum.  Returns (n_windows, n_ambiguous, max peak rel. error).
    """
    p_ref, a_ref, margin = oracle.peaks(z_ref, window)
    lead, n = z_ref.shape[:-1], z_ref.shape[-1]
    n_win = p_ref.shape[-1]
    pad = n_win * window - n
    diff = np.abs(np.asarray(z_gpu, np.complex128) - z_ref)
    zabs = np.abs(z_ref)
    if pad:
        diff = np.concatenate([diff, np.zeros(lead + (pad,))], axis=-1)
        zabs = np.concatenate([zabs, np.zeros(lead + (pad,))], axis=-1)
    err = diff.reshape(lead + (n_win, window)).max(axis=-1)
    zabs = zabs.reshape(lead + (n_win, window))
    gap = margin * p_ref                       # p1 - p2 in |z| units
    slack = 2.0 * err + 4.0 * np.finfo(np.float32).eps * p_ref
    strict = gap > slack
    gpu_arg = np.asarray(gpu_arg)
    assert np.array_equal(gpu_arg[strict], a_ref[strict]), "argmax differs where the margin is clear"
    chosen = np.take_along_axis(zabs, gpu_arg[..., None].astype(np.int64), axis=-1)[..., 0]
    assert np.all(chosen[~strict] >= p_ref[~strict] - slack[~strict]), "ambiguous argmax not near-max"
    rel = np.abs(np.asarray(gpu_peak, np.float64) - p_ref) / np.maximum(p_ref, 1e-300)
    return int(strict.size), int((~strict).sum()), float(rel.max())


def threshold_fixture():
    """Samples whose normalised SNR^2 equals threshold^2 = 16 exactly in float32, and one
    just above.  The paper keeps SNRs *over* the threshold (Sec. II.C.1), so only the
    sample above may become a candidate.  Expected values are written out by hand."""
    D, T, n, window = 1, 3, 40, 10
    z = np.zeros((D, T, n), np.complex64)
    w = np.array([1.0, 2.0, 0.25], np.float32)
    z[0, 0, 3] = 4 + 0j                   # 16 * 1
    z[0, 1, 14] = 2 + 2j                  # (4 + 4) * 2
    z[0, 2, 25] = 8 + 0j                  # 64 * 0.25
    above = np.float32(np.nextafter(np.float32(4.0), np.float32(5.0)))
    z[0, 0, 36] = above + 0j              # (4 + ulp)^2 rounds above 16
    exp_idx = np.full((D, T, 4), -1, np.int32)
    exp_idx[0, 0, 3] = 36
    exp_snr = np.zeros((D, T, 4), np.float32)
    exp_snr[0, 0, 3] = np.sqrt(np.float32(above * above))
    return z, w, window, exp_idx, exp_snr

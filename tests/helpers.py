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

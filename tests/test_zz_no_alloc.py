"""The entry point that allocates nothing (spiir_triggers_noalloc) against the one that
takes a caller's workspace (spiir_triggers): same kernels, so the same candidates bit for
bit, on two calls in a row, the second smaller than the first (the shared workspace keeps
the first call's keys, which the second must clear)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _series(rng, D, T, n, amp=1.0):
    z = ((rng.standard_normal((D, T, n)) + 1j * rng.standard_normal((D, T, n))) * amp)
    return z.astype(np.complex64)


def test_noalloc_triggers_match_workspace_entry_point_twice(gpu):
    import torch
    rng = np.random.default_rng(77)
    cases = [(3, 64, 6000, 512), (2, 9, 1500, 256)]   # second call: fewer slots, other shape
    for D, T, n, window in cases:
        print(f"no-alloc triggers: D={D} T={T} n={n} window={window}", flush=True)
        # amplitude 1: some windows keep a candidate, others none (checked on the CPU
        # with the oracle for these seeds: 647 / 1657 and 27 / 81)
        z = torch.from_numpy(_series(rng, D, T, n)).cuda()
        w = torch.from_numpy(rng.uniform(0.5, 1.5, size=T).astype(np.float32)).cuda()
        W = (n + window - 1) // window
        snr = torch.full((D, T, W), -5.0, dtype=torch.float32, device="cuda")
        idx = torch.full((D, T, W), -7, dtype=torch.int32, device="cuda")
        gpu.triggers_noalloc(z, w, 4.0, window, out=(snr, idx))
        snr_ref, idx_ref = gpu.triggers(z, w, 4.0, window)
        torch.cuda.synchronize()
        assert np.array_equal(idx.cpu().numpy(), idx_ref.cpu().numpy())
        assert np.array_equal(snr.cpu().numpy(), snr_ref.cpu().numpy())
        assert (idx_ref >= 0).sum().item() > 0 and (idx_ref < 0).sum().item() > 0


def test_noalloc_triggers_on_a_side_stream_at_the_size_limit(gpu):
    # exactly the workspace's 2^20 slots (1 detector, 1024 templates, 1024 windows of 2),
    # then a small call: both equal the workspace entry point's result
    import torch
    rng = np.random.default_rng(78)
    s = torch.cuda.Stream()
    for D, T, n, window in [(1, 1024, 2048, 2), (1, 5, 300, 100)]:
        print(f"no-alloc triggers (side stream): D={D} T={T} n={n} window={window}", flush=True)
        z = torch.from_numpy(_series(rng, D, T, n, 1.8)).cuda()
        w = torch.from_numpy(rng.uniform(0.5, 1.5, size=T).astype(np.float32)).cuda()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            snr, idx = gpu.triggers_noalloc(z, w, 3.0, window, stream=s)
        s.synchronize()
        snr_ref, idx_ref = gpu.triggers(z, w, 3.0, window)
        torch.cuda.synchronize()
        assert np.array_equal(idx.cpu().numpy(), idx_ref.cpu().numpy())
        assert np.array_equal(snr.cpu().numpy(), snr_ref.cpu().numpy())

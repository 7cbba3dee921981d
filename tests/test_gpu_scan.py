"""GPU parity of the FP32 scan path against the FP64 oracle (through the C ABI).

Tolerance: the relative SNR error per (detector, template), ||z_gpu - z_ref|| /
||z_ref|| over the stream, must be at most 1e-4 for the FP32 scan.
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_peaks

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4


def run_stream(gpu, bank, x, chunk, *, peak_window=0, filters_per_lane=0, max_delay=0,
               want_z=True, time_tile=0, balance_wgs=0):
    import torch
    D, N = x.shape
    zs, pk, am = [], [], []
    with gpu.SpiirBank.from_bank(bank, n_detectors=D, max_chunk=chunk, peak_window=peak_window,
                                 filters_per_lane=filters_per_lane, max_delay=max_delay,
                                 time_tile=time_tile, balance_wgs=balance_wgs) as sb:
        fits = chunk + sb.info.max_delay + 16 <= 12288
        assert (sb.info.balance_waves > 0) == (time_tile <= 0 and balance_wgs > 0 and fits)
        xd = torch.from_numpy(x).cuda()
        for lo in range(0, N, chunk):
            xc = xd[:, lo:lo + chunk].contiguous()
            z, p, a = sb.filter_chunk(xc, want_z=want_z)
            if want_z:
                zs.append(z.cpu().numpy())
            pk.append(p.cpu().numpy()); am.append(a.cpu().numpy())
        torch.cuda.synchronize()
        assert sb.refresh_info().scan_wait_timeouts == 0
    z = np.concatenate(zs, axis=-1) if want_z else None
    return z, pk, am


def test_tiny_workload_whole_and_chunked(gpu):
    w = synth.tiny()
    x = w.input()
    z_ref = oracle.filter(w.bank, x)
    for chunk in (16384, 2048):
        z, pk, am = run_stream(gpu, w.bank, x, chunk)
        err = oracle.rel_err(z, z_ref)
        print(f"chunk {chunk}: max rel err {err.max():.3e}")
        assert err.max() <= TOL_FP32
        # per-chunk peaks (one window per packet)
        for c, lo in enumerate(range(0, x.shape[1], chunk)):
            check_peaks(pk[c], am[c], z[..., lo:lo + chunk], z_ref[..., lo:lo + chunk], chunk)


@pytest.mark.parametrize("time_tile, balance_wgs", [(0, 0), (0, 3), (256, 0), (16, 0)])
@pytest.mark.parametrize("chunk", [1, 7, 100, 512, 1000])
def test_chunk_sizes_agree_with_oracle(gpu, chunk, time_tile, balance_wgs):
    rng = np.random.default_rng(100 + chunk)
    bank = synth.draw_filters(rng, np.array([70, 130, 5]))
    n = 3000 if chunk > 1 else 400
    x = rng.standard_normal((2, n)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, _, _ = run_stream(gpu, bank, x, chunk, time_tile=time_tile, balance_wgs=balance_wgs)
    assert oracle.rel_err(z, z_ref).max() <= TOL_FP32


@pytest.mark.parametrize("time_tile, balance_wgs", [(16, 0), (256, 0), (4096, 0), (-1, 0),
                                                  (0, 1), (-1, 2), (0, 4), (0, 8)])
def test_schedules_on_a_larger_bank(gpu, time_tile, balance_wgs):
    # many slices and tiles: the persistent queue's dependency chains, and the slice
    # queue with few and with many resident workgroups per compute unit
    rng = np.random.default_rng(150)
    bank = synth.draw_filters(rng, rng.integers(50, 900, size=96))
    x = rng.standard_normal((3, 6144)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, pk, am = run_stream(gpu, bank, x, 2048, time_tile=time_tile, balance_wgs=balance_wgs)
    assert oracle.rel_err(z, z_ref).max() <= TOL_FP32


@pytest.mark.parametrize("time_tile, balance_wgs", [(0, 0), (0, 2), (256, 0)])
@pytest.mark.parametrize("fpl", [1, 2, 4, 8])
def test_filters_per_lane_and_slice_boundaries(gpu, fpl, time_tile, balance_wgs):
    # template sizes around the slot/slice boundaries: 64*fpl filters per slice
    counts = np.array([1, 63, 64, 65, 64 * fpl, 64 * fpl + 1, 3 * 64 * fpl - 7, 0, 2])
    rng = np.random.default_rng(200 + fpl)
    bank = synth.draw_filters(rng, counts)
    x = rng.standard_normal((1, 2500)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, pk, am = run_stream(gpu, bank, x, 2500, filters_per_lane=fpl, peak_window=500,
                           time_tile=time_tile, balance_wgs=balance_wgs)
    err = oracle.rel_err(z, z_ref)
    nz = np.linalg.norm(z_ref, axis=-1) > 0
    assert err[nz].max() <= TOL_FP32
    assert np.all(z[:, 7] == 0)             # template with no filters
    check_peaks(pk[0], am[0], z, z_ref, 500)


@pytest.mark.parametrize("time_tile, balance_wgs", [(0, 0), (0, 2), (256, 0)])
def test_bank_without_filters(gpu, time_tile, balance_wgs):
    # every template empty (F = 0): the SNR is zero and each window's peak is 0 at its
    # first sample, as the oracle's float32 decision gives (lowest index on ties)
    rng = np.random.default_rng(310)
    bank = synth.draw_filters(rng, np.array([0, 0, 0]))
    assert bank.n_filters == 0
    x = rng.standard_normal((2, 700)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, pk, am = run_stream(gpu, bank, x, 300, peak_window=100, time_tile=time_tile,
                           balance_wgs=balance_wgs)
    assert z.shape == z_ref.shape and np.all(z == 0) and np.all(z_ref == 0)
    for c, lo in enumerate(range(0, 700, 300)):
        p_ref, a_ref = oracle.peaks_f32(z_ref[..., lo:lo + 300].astype(np.complex64), 100)
        assert np.array_equal(pk[c], p_ref) and np.array_equal(am[c], a_ref)


def test_delay_extremes_and_history(gpu):
    # delays 0 and exactly max_delay; history longer than the chunk; max_delay > largest delay
    rng = np.random.default_rng(300)
    bank = synth.draw_filters(rng, np.array([40, 40]), max_delay=2047)
    bank.d[:5] = 0
    bank.d[5:10] = 2047
    x = rng.standard_normal((1, 6000)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    for chunk, md, tt, q in ((512, 0, 0, 0), (300, 4000, 256, 0), (6000, 0, 0, 0), (6000, 0, 512, 0),
                             (300, 8191, 64, 0), (300, 8191, 0, 2), (4000, 8191, 0, 2)):
        z, _, _ = run_stream(gpu, bank, x, chunk, max_delay=md, time_tile=tt, balance_wgs=q)
        assert oracle.rel_err(z, z_ref).max() <= TOL_FP32


def test_zero_delay_bank_has_no_history(gpu):
    rng = np.random.default_rng(301)
    bank = synth.draw_filters(rng, np.array([64, 10]), max_delay=0)
    x = rng.standard_normal((1, 1500)).astype(np.float32)
    z, _, _ = run_stream(gpu, bank, x, 256)
    assert oracle.rel_err(z, oracle.filter(bank, x)).max() <= TOL_FP32


def test_three_detectors(gpu):
    rng = np.random.default_rng(400)
    bank = synth.draw_filters(rng, rng.integers(20, 300, size=12))
    x = rng.standard_normal((3, 4096)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, pk, am = run_stream(gpu, bank, x, 512)
    assert oracle.rel_err(z, z_ref).max() <= TOL_FP32
    for c in range(8):
        check_peaks(pk[c], am[c], z[..., c * 512:(c + 1) * 512], z_ref[..., c * 512:(c + 1) * 512], 512)


def test_reset_restarts_the_stream(gpu):
    import torch
    rng = np.random.default_rng(500)
    bank = synth.draw_filters(rng, np.array([100, 50]))
    x = torch.from_numpy(rng.standard_normal((1, 1024)).astype(np.float32)).cuda()
    with gpu.SpiirBank.from_bank(bank, max_chunk=1024) as sb:
        z1, p1, a1 = sb.filter_chunk(x)
        z1 = z1.clone()
        sb.filter_chunk(x)
        sb.reset()
        z3, p3, a3 = sb.filter_chunk(x)
        assert torch.equal(z1, z3)


def test_deterministic_repeat(gpu):
    import torch
    w = synth.tiny()
    x = torch.from_numpy(w.input()).cuda()
    outs = []
    for _ in range(2):
        with gpu.SpiirBank.from_bank(w.bank, max_chunk=16384) as sb:
            outs.append([t.clone() for t in sb.filter_chunk(x)])
    for u, v in zip(*outs):
        assert torch.equal(u, v)


def test_fused_peaks_equal_standalone_peaks(gpu):
    import torch
    rng = np.random.default_rng(600)
    bank = synth.draw_filters(rng, np.array([300, 200, 90]))
    x = torch.from_numpy(rng.standard_normal((2, 2048)).astype(np.float32)).cuda()
    with gpu.SpiirBank.from_bank(bank, n_detectors=2, max_chunk=2048, peak_window=256) as sb:
        z, p, a = sb.filter_chunk(x)
        p2, a2 = gpu.peaks(z, 256)
        assert torch.equal(p, p2) and torch.equal(a, a2)


def test_outputs_optional(gpu):
    import torch
    rng = np.random.default_rng(700)
    bank = synth.draw_filters(rng, np.array([64, 64]))
    x = torch.from_numpy(rng.standard_normal((1, 512)).astype(np.float32)).cuda()
    with gpu.SpiirBank.from_bank(bank, max_chunk=512) as a_bank, \
            gpu.SpiirBank.from_bank(bank, max_chunk=512) as b_bank:
        za, _, _ = a_bank.filter_chunk(x, want_peaks=False)
        _, pb, ab = b_bank.filter_chunk(x, want_z=False)
        _, pa, aa = a_bank.filter_chunk(x)      # second packet
        _, pb2, ab2 = b_bank.filter_chunk(x)
        assert torch.equal(pa, pb2) and torch.equal(aa, ab2)
        p0, a0 = gpu.peaks(za, 512)
        assert torch.equal(p0, pb) and torch.equal(a0, ab)


def test_invalid_calls_on_gpu(gpu):
    import torch
    rng = np.random.default_rng(800)
    bank = synth.draw_filters(rng, np.array([10]))
    with gpu.SpiirBank.from_bank(bank, max_chunk=256, peak_window=64) as sb:
        with pytest.raises(gpu.SpiirError):
            sb.filter_chunk(torch.zeros((1, 300), device="cuda"))       # n > max_chunk
        with pytest.raises(gpu.SpiirError):
            sb.filter_chunk(torch.zeros((1, 100), device="cuda"))       # not a multiple of window
        z, p, a = sb.filter_chunk(torch.zeros((1, 128), device="cuda"))
        assert torch.all(z == 0) and torch.all(a == 0)


@pytest.mark.parametrize("rows, n, window", [(5, 1000, 128), (1, 7, 7), (3, 4096, 4096), (2, 300, 1)])
def test_standalone_peaks_bit_exact(gpu, rows, n, window):
    import torch
    rng = np.random.default_rng(rows * 7 + n)
    z = (rng.standard_normal((rows, n)) + 1j * rng.standard_normal((rows, n))).astype(np.complex64)
    if n > 20:
        z[0, 3] = z[0, 11] = 50 + 50j            # exact tie: lowest index wins
    p, a = gpu.peaks(torch.from_numpy(z).cuda(), window)
    pr, ar = oracle.peaks_f32(z, window)
    assert np.array_equal(a.cpu().numpy(), ar)
    assert np.array_equal(p.cpu().numpy(), pr)


def test_realistic_bank_full_size_sampled(gpu):
    """The 1024-template realistic bank in 1-s packets in the benchmark's launch
    configuration (default filters per lane, balanced schedule with 2 workgroups per
    compute unit), checked on a seeded sample of templates over 8 s, with the first
    and last templates always included."""
    w = synth.realistic()
    n = 8 * 2048
    x = w.input()[:, :n]
    z, pk, am = run_stream(gpu, w.bank, x, 2048, balance_wgs=2)
    pick = sorted(set([0, w.bank.n_templates - 1]) |
                  set(np.random.default_rng(9).choice(w.bank.n_templates, 14, replace=False).tolist()))
    sub = w.bank.subset(pick)
    z_ref = oracle.filter(sub, x)
    err = oracle.rel_err(z[:, pick], z_ref)
    print(f"realistic sampled: max rel err {err.max():.3e} median {np.median(err):.3e}")
    assert err.max() <= TOL_FP32
    for c in range(8):
        check_peaks(pk[c][:, pick], am[c][:, pick], z[:, pick, c * 2048:(c + 1) * 2048],
                    z_ref[..., c * 2048:(c + 1) * 2048], 2048)


def test_wait_timeout_is_reported_until_reset(gpu):
    """A state hand-off wait that hits its bound, forced from the host with a bound of one
    poll on the persistent scan (its tile-1 items start while the tile-0 items they need
    are still running): every wave still finishes, the bank counts the timeouts, the next
    filter_chunk returns SPIIR_E_STATE without enqueueing anything, and a reset clears
    the count and the status."""
    import torch
    w = synth.realistic(n_templates=64, seconds=2)
    x = torch.from_numpy(w.input()).cuda()
    with gpu.SpiirBank.from_bank(w.bank, max_chunk=2048, time_tile=256, wait_spins=1) as sb:
        sb.filter_chunk(x[:, :2048].contiguous(), want_peaks=False)
        torch.cuda.synchronize()
        assert sb.refresh_info().scan_wait_timeouts > 0
        with pytest.raises(gpu.SpiirError) as exc:
            sb.filter_chunk(x[:, 2048:].contiguous(), want_peaks=False)
        assert exc.value.status == gpu.SPIIR_E_STATE
        sb.reset()
        assert sb.refresh_info().scan_wait_timeouts == 0
        sb.filter_chunk(x[:, 2048:].contiguous(), want_peaks=False)   # accepted again
        torch.cuda.synchronize()

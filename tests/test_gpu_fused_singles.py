"""Single-slice templates in the FP32 scan (through the C ABI).

A template whose filters fit one slice is its own SNR series: every schedule writes
it straight into z, and the balanced schedule also finds its peaks (Section II.C.1,
one candidate per template per window) at the end of each wave's part of the slice,
handing a window that a cut splits to the wave that continues it; the slice-sum
kernel then visits only the other templates.  Checked here:

* z of the balanced schedule equals z of the one-wave-per-slice schedule bit for bit
  (the same arithmetic in the same order), and the oracle within 1e-4;
* the peaks equal the standalone peak search of that z bit for bit (the same
  decision), with z requested or not, for one window per packet, windows of whole
  sub-tiles, and windows that are not (those leave the peaks to the slice-sum kernel);
* an exact tie in |z| goes to the lowest index, in every window.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-4


def mixed_bank(seed):
    """Templates of one slice, several slices and none (4 filters per lane: 256 per
    slice), and two pass-through templates (one filter, a = 0, b = 1, d = 0: z = x)."""
    rng = np.random.default_rng(seed)
    counts = np.array([30, 0, 200, 64, 1, 257, 600, 128, 513, 90, 256, 1, 700, 255, 17, 1])
    bank = synth.draw_filters(rng, counts, max_delay=600)
    for t in (4, 11):
        k = int(bank.offsets[t])
        bank.a[k], bank.b[k], bank.d[k] = 0.0, 1.0, 0
    return bank


def packets(seed, D, n, count):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((D, n * count)).astype(np.float32)
    # exact ties for the pass-through templates: |x| = 7 at two samples of every
    # 16-sample sub-tile pair, the lower one first
    for c in range(count):
        for j in range(0, n - 40, 40):
            x[:, c * n + j + 3] = 7.0
            x[:, c * n + j + 21] = -7.0
    return x


@pytest.mark.parametrize("n, window", [(2048, 0), (2048, 256), (2048, 16), (1000, 0),
                                       (2000, 100), (777, 0)])
def test_balanced_singles_match_static_schedule_and_peaks(gpu, n, window):
    import torch
    D, count = 2, 3
    bank = mixed_bank(40 + n)
    x_host = packets(50 + n, D, n, count)
    x = torch.from_numpy(x_host).cuda()
    kw = dict(n_detectors=D, max_chunk=n, peak_window=window, filters_per_lane=4)
    zs = []
    with gpu.SpiirBank.from_bank(bank, balance_wgs=2, **kw) as bal, \
            gpu.SpiirBank.from_bank(bank, balance_wgs=0, **kw) as sta, \
            gpu.SpiirBank.from_bank(bank, balance_wgs=2, **kw) as pko:
        assert bal.info.balance_waves > 0 and sta.info.balance_waves == 0
        for c in range(count):
            xc = x[:, c * n:(c + 1) * n].contiguous()
            z, p, a = bal.filter_chunk(xc)
            zr, pr, ar = sta.filter_chunk(xc)
            _, po, ao = pko.filter_chunk(xc, want_z=False)     # peaks only
            assert torch.equal(z, zr)
            p2, a2 = gpu.peaks(z, window if window > 0 else n)
            assert torch.equal(p, p2) and torch.equal(a, a2)
            assert torch.equal(pr, p2) and torch.equal(ar, a2)
            assert torch.equal(po, p2) and torch.equal(ao, a2)
            # the pass-through templates: the tie goes to the first sample of |x| = 7
            for t in (4, 11):
                w = window if window > 0 else n
                for k in range(n // w if window > 0 else 1):
                    seg = np.abs(x_host[:, c * n + k * w: c * n + (k + 1) * w])
                    first = np.argmax(seg == seg.max(axis=1, keepdims=True), axis=1)
                    assert np.array_equal(a[:, t, k].cpu().numpy(), first)
            zs.append(z.cpu().numpy())
        torch.cuda.synchronize()
        assert bal.refresh_info().scan_wait_timeouts == 0
    z_all = np.concatenate(zs, axis=-1)
    err = oracle.rel_err(z_all, oracle.filter(bank, x_host))
    print(f"n {n} window {window}: max rel err {err.max():.3e}")
    assert err.max() <= TOL_FP32


@pytest.mark.parametrize("fpl, balance_wgs", [(8, 3), (2, 4), (1, 4)])
def test_balanced_singles_other_slice_widths(gpu, fpl, balance_wgs):
    """8, 2 and 1 filters per lane (512, 128 and 64 filters per slice): other single-slice
    sets."""
    import torch
    D, n = 3, 512
    bank = mixed_bank(70 + fpl)
    x = torch.from_numpy(packets(80 + fpl, D, n, 1)).cuda()
    kw = dict(n_detectors=D, max_chunk=n, filters_per_lane=fpl)
    with gpu.SpiirBank.from_bank(bank, balance_wgs=balance_wgs, **kw) as bal, \
            gpu.SpiirBank.from_bank(bank, balance_wgs=0, **kw) as sta:
        assert bal.info.balance_waves > 0
        z, p, a = bal.filter_chunk(x)
        zr, pr, ar = sta.filter_chunk(x)
        assert torch.equal(z, zr) and torch.equal(p, pr) and torch.equal(a, ar)


def test_forward_on_the_balanced_schedule(gpu):
    """The differentiation forward writes single-slice templates into z in the balanced
    schedule too (no peaks)."""
    import torch
    D, n = 1, 1500
    bank = mixed_bank(90)
    x = torch.from_numpy(packets(91, D, n, 1)).cuda()
    kw = dict(n_detectors=D, max_chunk=n, filters_per_lane=4, ckpt_stride=256)
    with gpu.SpiirBank.from_bank(bank, balance_wgs=2, **kw) as bal, \
            gpu.SpiirBank.from_bank(bank, balance_wgs=0, **kw) as sta:
        assert bal.info.balance_waves > 0
        z, _ = bal.forward(x)
        zr, _ = sta.forward(x)
        assert torch.equal(z, zr)


def test_balanced_packets_without_outputs_keep_the_stream(gpu):
    """A packet that asks for neither z nor peaks still moves the state and the history:
    the next packet's outputs equal those of a bank that produced every output."""
    import torch
    D, n = 2, 1024
    bank = mixed_bank(95)
    x = torch.from_numpy(packets(96, D, n, 3)).cuda()
    kw = dict(n_detectors=D, max_chunk=n, filters_per_lane=4, balance_wgs=2)
    with gpu.SpiirBank.from_bank(bank, **kw) as quiet, gpu.SpiirBank.from_bank(bank, **kw) as full:
        for c in range(3):
            xc = x[:, c * n:(c + 1) * n].contiguous()
            zf, pf, af = full.filter_chunk(xc)
            if c == 1:
                z, p, a = quiet.filter_chunk(xc, want_z=False, want_peaks=False)
                assert z is None and p is None
            else:
                z, p, a = quiet.filter_chunk(xc)
                assert torch.equal(z, zf) and torch.equal(p, pf) and torch.equal(a, af)


@pytest.mark.parametrize("seed, D, fpl, wgs, n, window", [
    (1, 1, 4, 2, 2048, 0), (2, 3, 8, 3, 512, 0), (3, 2, 2, 4, 1000, 0),
    (4, 1, 4, 1, 2048, 256), (5, 3, 4, 3, 1024, 128), (6, 2, 8, 2, 768, 0),
    (7, 2, 1, 4, 1024, 256)])
def test_balanced_equals_static_on_random_banks(gpu, seed, D, fpl, wgs, n, window):
    """Seeded random banks (empty, one-slice and many-slice templates, delays up to 2047; 1-8
    filters per lane):
    two packets through the balanced schedule give the one-wave-per-slice schedule's z and
    peaks bit for bit."""
    import torch
    rng = np.random.default_rng(1000 + seed)
    counts = rng.integers(0, 1200, size=int(rng.integers(20, 60)))
    counts[rng.random(counts.size) < 0.1] = 0
    bank = synth.draw_filters(rng, counts)
    x = torch.from_numpy(rng.standard_normal((D, 2 * n)).astype(np.float32)).cuda()
    kw = dict(n_detectors=D, max_chunk=n, filters_per_lane=fpl, peak_window=window)
    with gpu.SpiirBank.from_bank(bank, balance_wgs=wgs, **kw) as bal, \
            gpu.SpiirBank.from_bank(bank, balance_wgs=0, **kw) as sta:
        assert bal.info.balance_waves > 0
        for c in range(2):
            xc = x[:, c * n:(c + 1) * n].contiguous()
            z, p, a = bal.filter_chunk(xc)
            zr, pr, ar = sta.filter_chunk(xc)
            assert torch.equal(z, zr) and torch.equal(p, pr) and torch.equal(a, ar)
        assert bal.refresh_info().scan_wait_timeouts == 0

"""GPU parity of the split-bf16 time-blocked form against the FP64 oracle.

Tolerance: relative SNR error per (detector, template) at most 1e-3 for the
split-bf16 block form (the products run as hi*hi + hi*lo + lo*hi in bf16 with
FP32 accumulation, the block-to-block carry in FP64 for every tile of 16 filters
holding one with |a| > 0.999).
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import check_peaks

pytestmark = pytest.mark.gpu

TOL_BF16 = 1e-3


def run_block(gpu, bank, x, chunk, *, block_len=128, peak_window=0, want_z=True,
              long_pole=0.999):
    import torch
    D, N = x.shape
    zs, pk, am = [], [], []
    with gpu.SpiirBank.from_bank(bank, n_detectors=D, max_chunk=chunk, peak_window=peak_window,
                                 mode=gpu.MODE_BF16_BLOCK, block_len=block_len,
                                 long_pole_abs_a=long_pole) as sb:
        xd = torch.from_numpy(x).cuda()
        for lo in range(0, N, chunk):
            z, p, a = sb.filter_chunk(xd[:, lo:lo + chunk].contiguous(), want_z=want_z)
            if want_z:
                zs.append(z.cpu().numpy())
            pk.append(p.cpu().numpy()); am.append(a.cpu().numpy())
        torch.cuda.synchronize()
        info = sb.refresh_info()
    return (np.concatenate(zs, axis=-1) if want_z else None), pk, am, info


@pytest.mark.parametrize("block_len", [64, 128, 256])
def test_block_form_small_bank(gpu, block_len):
    rng = np.random.default_rng(1000 + block_len)
    bank = synth.draw_filters(rng, np.array([37, 5, 130, 16, 1]))
    x = rng.standard_normal((2, 8 * 1024)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, pk, am, info = run_block(gpu, bank, x, 2048, block_len=block_len)
    err = oracle.rel_err(z, z_ref)
    print(f"L={block_len}: max rel err {err.max():.3e}, long-pole filters {info.n_long_pole}")
    assert err.max() <= TOL_BF16
    for c in range(4):
        sl = slice(c * 2048, (c + 1) * 2048)
        check_peaks(pk[c], am[c], z[..., sl], z_ref[..., sl], 2048)


def test_block_form_streaming_equals_whole(gpu):
    rng = np.random.default_rng(1100)
    bank = synth.draw_filters(rng, rng.integers(1, 200, size=9))
    x = rng.standard_normal((1, 6 * 512)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z_whole, _, _, _ = run_block(gpu, bank, x, 6 * 512)
    z_chunks, _, _, _ = run_block(gpu, bank, x, 512)
    assert oracle.rel_err(z_whole, z_ref).max() <= TOL_BF16
    assert oracle.rel_err(z_chunks, z_ref).max() <= TOL_BF16


def test_long_pole_carry_in_fp64(gpu):
    # every filter with |a| close to 1: the FP64 carry path; also all-FP32 for contrast
    rng = np.random.default_rng(1200)
    bank = synth.draw_filters(rng, np.array([64, 64]), tau_range=(2.0, 4.0))
    x = rng.standard_normal((1, 32768)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, _, _, info = run_block(gpu, bank, x, 32768)
    assert info.n_long_pole == int(np.sum(np.abs(bank.a.astype(np.complex128)) > 0.999))
    assert info.n_long_pole > 0
    assert oracle.rel_err(z, z_ref).max() <= TOL_BF16


@pytest.mark.parametrize("threshold", [0.5, 0.999, 0.99985, 0.9999999])
def test_carry_precision_is_chosen_per_tile(gpu, threshold):
    """Memory times log-uniform in [5 ms, 4 s] put filters on both sides of every threshold
    in most tiles of 16: every tile carries in FP64 (0.5, 0.999), most tiles in FP32 and
    the others in FP64 (0.99985: 9 of the 316 filters above it), or every tile in FP32
    (0.9999999: above the largest |a|); each within the tolerance."""
    rng = np.random.default_rng(1250)
    bank = synth.draw_filters(rng, np.array([40, 9, 170, 33, 64]))
    x = rng.standard_normal((2, 8192)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, _, _, info = run_block(gpu, bank, x, 4096, long_pole=threshold)
    absa = np.abs(bank.a.astype(np.complex128))
    assert info.n_long_pole == int(np.sum(absa > threshold))
    err = oracle.rel_err(z, z_ref).max()
    print(f"threshold {threshold}: {info.n_long_pole} long-pole filters, max rel err {err:.3e}")
    assert err <= TOL_BF16


def test_block_form_empty_template_and_zero_delay(gpu):
    rng = np.random.default_rng(1300)
    bank = synth.draw_filters(rng, np.array([20, 0, 3]), max_delay=0)
    x = rng.standard_normal((1, 1024)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z, _, _, _ = run_block(gpu, bank, x, 1024, block_len=64)
    assert np.all(z[:, 1] == 0)
    nz = [0, 2]
    assert oracle.rel_err(z[:, nz], z_ref[:, nz]).max() <= TOL_BF16


def test_block_form_rejects_ragged_packets(gpu):
    import torch
    rng = np.random.default_rng(1400)
    bank = synth.draw_filters(rng, np.array([8]))
    with gpu.SpiirBank.from_bank(bank, max_chunk=1024, mode=gpu.MODE_BF16_BLOCK) as sb:
        with pytest.raises(gpu.SpiirError):
            sb.filter_chunk(torch.zeros((1, 1000), device="cuda"))
    with pytest.raises(gpu.SpiirError):
        gpu.SpiirBank.from_bank(bank, max_chunk=1000, mode=gpu.MODE_BF16_BLOCK)


def test_precision_workload_full_size_sampled(gpu):
    """The precision workload (1024-template bank, 3 detector streams of 32 s) in one
    packet per detector; sampled templates checked against the oracle."""
    w = synth.precision()
    x = w.input()
    z, pk, am, info = run_block(gpu, w.bank, x, w.n_samples)
    pick = sorted(set([0, w.bank.n_templates - 1]) |
                  set(np.random.default_rng(5).choice(w.bank.n_templates, 6, replace=False).tolist()))
    z_ref = oracle.filter(w.bank.subset(pick), x)
    err = oracle.rel_err(z[:, pick], z_ref)
    print(f"precision workload: max rel err {err.max():.3e}, median {np.median(err):.3e}, "
          f"long-pole filters {info.n_long_pole}")
    assert err.max() <= TOL_BF16
    n_win, n_amb, _ = check_peaks(pk[0][:, pick], am[0][:, pick], z[:, pick], z_ref, w.n_samples)
    print(f"argmax windows {n_win}, ambiguous {n_amb}")


@pytest.mark.parametrize("block_len", [64, 256])
def test_block_set_coeffs_regenerates_the_operands(gpu, block_len):
    """Replacing the coefficients of a block-form bank (delays kept) regenerates every
    operand on the GPU: the output equals, bit for bit, that of a bank created with the
    new coefficients, and the oracle's within the split-bf16 tolerance."""
    import torch
    rng = np.random.default_rng(1200 + block_len)
    counts = np.array([40, 3, 160, 17])
    bank = synth.draw_filters(rng, counts)
    other = synth.draw_filters(np.random.default_rng(1300 + block_len), counts)
    moved = synth.Bank(bank.offsets, other.a, other.b, bank.d)
    x = rng.standard_normal((2, 2048)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    kw = dict(n_detectors=2, max_chunk=2048, mode=gpu.MODE_BF16_BLOCK, block_len=block_len)
    with gpu.SpiirBank.from_bank(bank, **kw) as sb:
        sb.set_coeffs(torch.from_numpy(other.a).cuda(), torch.from_numpy(other.b).cuda())
        z1, _, _ = sb.filter_chunk(xd)
        z1 = z1.cpu().numpy()
    with gpu.SpiirBank.from_bank(moved, **kw) as sb:
        z2, _, _ = sb.filter_chunk(xd)
        z2 = z2.cpu().numpy()
    assert np.array_equal(z1, z2)
    assert oracle.rel_err(z1, oracle.filter(moved, x)).max() <= TOL_BF16


@pytest.mark.parametrize("block_len", [64, 128])
def test_block_form_is_deterministic_across_detectors_and_chunks(gpu, block_len):
    """Three detectors and several 64-block chunks per detector: two banks given the
    same packet return bit-identical z (the block form has no order-dependent step), and
    the result stays within the oracle's tolerance."""
    import torch
    rng = np.random.default_rng(31 + block_len)
    bank = synth.draw_filters(rng, rng.integers(100, 700, size=24))
    D, n = 3, 160 * block_len                       # 160 blocks: chunks of 64, 64, 32
    x = torch.from_numpy(rng.standard_normal((D, n)).astype(np.float32)).cuda()
    kw = dict(n_detectors=D, max_chunk=n, mode=gpu.MODE_BF16_BLOCK, block_len=block_len)
    zs = []
    for _ in range(2):
        with gpu.SpiirBank.from_bank(bank, **kw) as sb:
            z, _, _ = sb.filter_chunk(x, want_peaks=False)
            torch.cuda.synchronize()
            zs.append(z.clone())
    assert torch.equal(zs[0], zs[1])
    err = oracle.rel_err(zs[0].cpu().numpy(), oracle.filter(bank, x.cpu().numpy()))
    assert err.max() <= TOL_BF16


def test_matrix_core_work_reported_per_column(gpu):
    """One template of 16 filters with zero delays at L = 64: the input-to-state operand is
    one tile of 4 K steps (offsets 0..63), the output operand 4 row tiles x (2 state + 4
    input K steps); each 32x16 operand block makes 3 split products of 32 x 16 x 2 flop per
    column.  The FP32 scan reports none."""
    rng = np.random.default_rng(1500)
    bank = synth.draw_filters(rng, np.array([16]), max_delay=0)
    with gpu.SpiirBank.from_bank(bank, max_chunk=1024, mode=gpu.MODE_BF16_BLOCK,
                                 block_len=64) as sb:
        assert sb.info.block_mfma_flop_per_column == (4 + 4 * (2 + 4)) * 32 * 16 * 2 * 3
    with gpu.SpiirBank.from_bank(bank, max_chunk=1024) as sb:
        assert sb.info.block_mfma_flop_per_column == 0


@pytest.mark.parametrize("block_len", [64, 128])
def test_small_bank_split_output_streaming_three_detectors(gpu, block_len):
    """A bank of 6 templates fills only a few compute units with output tiles, so the output
    product's K steps are split over workgroups and the parts summed in order: three
    detectors streamed in three packets match the oracle, and a second identical bank
    gives the same output bit for bit."""
    rng = np.random.default_rng(1600 + block_len)
    bank = synth.draw_filters(rng, np.array([128, 40, 300, 7, 64, 200]))
    x = rng.standard_normal((3, 3 * 1024)).astype(np.float32)
    z_ref = oracle.filter(bank, x)
    z1, _, _, _ = run_block(gpu, bank, x, 1024, block_len=block_len)
    z2, _, _, _ = run_block(gpu, bank, x, 1024, block_len=block_len)
    assert np.array_equal(z1, z2)
    assert oracle.rel_err(z1, z_ref).max() <= TOL_BF16

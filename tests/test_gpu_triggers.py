"""Trigger selection (Section II.C.1) on the GPU: normalised SNR, loudest template per
sample above threshold, one candidate per template per window."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


# the last case is long enough for the 32-samples-per-workgroup kernel (ragged tail)
@pytest.mark.parametrize("D, T, n, window", [(1, 7, 1000, 256), (3, 40, 2048, 2048), (2, 3, 100, 7),
                                             (2, 5, 20011, 512)])
def test_triggers_bit_exact_on_seeded_series(gpu, D, T, n, window):
    import torch
    rng = np.random.default_rng(D * 100 + T)
    z = ((rng.standard_normal((D, T, n)) + 1j * rng.standard_normal((D, T, n))) * 1.7).astype(np.complex64)
    z[0, 1, 5] = z[0, 2, 5] = 11 + 11j           # tie across templates
    w = rng.uniform(0.4, 1.6, size=T).astype(np.float32)
    snr, idx = gpu.triggers(torch.from_numpy(z).cuda(), torch.from_numpy(w).cuda(), 4.0, window)
    snr_ref, idx_ref = oracle.triggers(z, w, 4.0, window)
    assert np.array_equal(idx.cpu().numpy(), idx_ref)
    assert np.array_equal(snr.cpu().numpy(), snr_ref)
    assert (idx_ref >= 0).sum() > 0


@pytest.mark.parametrize("D, T, n, window", [(1, 7, 1000, 256), (2, 5, 20011, 512)])
@pytest.mark.parametrize("threshold", [0.0, 1.0e4])
def test_triggers_threshold_extremes(gpu, D, T, n, window, threshold):
    # threshold 0: every window of every template keeps its loudest sample; a threshold
    # no sample reaches: no candidate anywhere (index -1, snr 0)
    import torch
    rng = np.random.default_rng(D * 1000 + T)
    z = (rng.standard_normal((D, T, n)) + 1j * rng.standard_normal((D, T, n))).astype(np.complex64)
    w = rng.uniform(0.4, 1.6, size=T).astype(np.float32)
    snr, idx = gpu.triggers(torch.from_numpy(z).cuda(), torch.from_numpy(w).cuda(), threshold, window)
    snr_ref, idx_ref = oracle.triggers(z, w, threshold, window)
    assert np.array_equal(idx.cpu().numpy(), idx_ref)
    assert np.array_equal(snr.cpu().numpy(), snr_ref)
    if threshold > 0:
        assert np.all(idx_ref == -1) and np.all(snr_ref == 0)
    else:
        assert (idx_ref >= 0).any()


def test_noise_power_matches_oracle(gpu):
    w = synth.tiny()
    rng = np.random.default_rng(5)
    bank = synth.draw_filters(rng, np.array([30, 1, 200, 64]))
    for bk in (w.bank, bank):
        with gpu.SpiirBank.from_bank(bk, max_chunk=256) as sb:
            p = sb.noise_power()
        assert np.allclose(p, oracle.noise_power(bk), rtol=1e-10, atol=0)


def test_triggers_end_to_end_on_noise(gpu):
    """Normalised SNR of the filtered noise has unit variance per quadrature (so
    E rho^2 = 2), and every trigger is consistent with the series it came from."""
    import torch
    w = synth.realistic(n_templates=64, seconds=8)
    with gpu.SpiirBank.from_bank(w.bank, max_chunk=2048) as sb:
        power = sb.noise_power()
        weight = torch.from_numpy((2.0 / power).astype(np.float32)).cuda()
        x = torch.from_numpy(w.input()).cuda()
        zs = []
        for i in range(8):
            z, _, _ = sb.filter_chunk(x[:, i * 2048:(i + 1) * 2048].contiguous(), want_peaks=False)
            zs.append(z.clone())
        z = torch.cat(zs, dim=-1)
        snr, idx = gpu.triggers(z, weight, 4.0, 2048)
    zc = z.cpu().numpy()
    rho2 = np.abs(zc[:, :, 4096:]) ** 2 * (2.0 / power)[None, :, None]   # after 2 s of warm-up
    assert abs(rho2.mean() / 2.0 - 1.0) < 0.1
    snr, idx = snr.cpu().numpy(), idx.cpu().numpy()
    d, t, k = np.nonzero(idx >= 0)
    assert len(d) > 0
    vals = np.abs(zc[d, t, idx[d, t, k]]) * np.sqrt(2.0 / power[t])   # index is in [0, n)
    assert np.all(idx[d, t, k] // 2048 == k)
    assert np.allclose(snr[d, t, k], vals, rtol=1e-5)
    assert np.all(snr[d, t, k] > 4.0)


def test_triggers_threshold_is_strict(gpu):
    # samples at exactly threshold^2 are not candidates, one just above is (Sec. II.C.1:
    # SNRs over the threshold); expected values written out by hand
    import torch
    from helpers import threshold_fixture
    z, w, window, exp_idx, exp_snr = threshold_fixture()
    snr, idx = gpu.triggers(torch.from_numpy(z).cuda(), torch.from_numpy(w).cuda(), 4.0, window)
    assert np.array_equal(idx.cpu().numpy(), exp_idx)
    assert np.array_equal(snr.cpu().numpy(), exp_snr)


@pytest.mark.parametrize("mode", [0, 1])
def test_trigger_weights_on_the_gpu(gpu, mode):
    """2 / E|z_t|^2 from the bank's device coefficients equals 2 / the oracle's closed-form
    noise power (float32 rounding of an FP64 value), also for a template without filters,
    and follows set_coeffs."""
    import torch
    rng = np.random.default_rng(95 + mode)
    counts = np.array([30, 0, 200, 64, 1])
    bank = synth.draw_filters(rng, counts)
    other = synth.draw_filters(np.random.default_rng(97 + mode), counts)
    with gpu.SpiirBank.from_bank(bank, max_chunk=256, mode=mode) as sb:
        w = sb.trigger_weights().cpu().numpy()
        sb.set_coeffs(torch.from_numpy(other.a).cuda(), torch.from_numpy(other.b).cuda())
        w2 = sb.trigger_weights().cpu().numpy()
    for got, bk in ((w, bank), (w2, synth.Bank(bank.offsets, other.a, other.b, bank.d))):
        p = oracle.noise_power(bk)
        assert got[1] == 0.0 and p[1] == 0.0
        ok = p > 0
        assert np.allclose(got[ok], (2.0 / p[ok]).astype(np.float32), rtol=2e-7, atol=0)

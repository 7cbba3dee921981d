"""Pins for the FP64 oracle: each checks it against something other than itself.

Sources of truth used here: the closed-form summed impulse response of the
SPIIR bank (Section II.B.1), a brute-force direct convolution, scipy's
``lfilter``, the steady-state frequency response, the white-noise output
variance, linearity / shift / chunking invariance, the block-carry identity, the
paper's cost-model arithmetic (Section II.B.2), and for the signal-consistency
statistic (Section II.C.1) the brute-force correlation of the impulse response, the
noise power at lag 0, exact special cases and its unit mean on white noise.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.signal

import oracle
import synth
from helpers import threshold_fixture

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_bank(seed, counts, max_delay=40, tau=(0.002, 0.05)):
    rng = np.random.default_rng(seed)
    return synth.draw_filters(rng, np.asarray(counts), tau_range=tau, max_delay=max_delay)


def closed_form_impulse(bank, n, at=0):
    """sum_k b_k a_k^(m-d_k) for m >= d_k, via numpy complex powers."""
    z = np.zeros((bank.n_templates, n), dtype=np.complex128)
    m = np.arange(n)
    for t in range(bank.n_templates):
        for k in range(bank.offsets[t], bank.offsets[t + 1]):
            a = complex(bank.a[k]); b = complex(bank.b[k]); d = int(bank.d[k])
            e = m - d - at
            ok = e >= 0
            z[t, ok] += b * np.power(a, e[ok].astype(np.float64))
    return z


def test_impulse_response_closed_form():
    bank = small_bank(1, [5, 1, 9], max_delay=60, tau=(0.001, 0.5))
    n = 700
    for at in (0, 13):
        x = synth.impulse(n, at)
        z = oracle.filter(bank, x)[0]
        ref = closed_form_impulse(bank, n, at)
        err = oracle.rel_err(z, ref)
        assert err.max() < 1e-12, err
        # and nothing before the first delayed impulse
        first = at + bank.d[bank.offsets[0]:bank.offsets[1]].min()
        assert np.all(z[0, :first] == 0)


def test_brute_force_direct_convolution():
    bank = small_bank(2, [4, 7], max_delay=50, tau=(0.001, 0.3))
    n = 400
    x = np.random.default_rng(3).standard_normal((2, n)).astype(np.float32)
    z = oracle.filter(bank, x)
    ref = np.zeros_like(z)
    xd = x.astype(np.float64)
    for det in range(2):
        for t in range(bank.n_templates):
            for k in range(bank.offsets[t], bank.offsets[t + 1]):
                a = complex(bank.a[k]); b = complex(bank.b[k]); d = int(bank.d[k])
                for i in range(n):
                    if i - d < 0:
                        continue
                    mm = np.arange(0, i - d + 1)
                    ref[det, t, i] += b * np.sum(np.power(a, mm.astype(np.float64)) * xd[det, i - d - mm])
    assert oracle.rel_err(z, ref).max() < 1e-12


def test_scipy_lfilter():
    bank = small_bank(4, [3, 6, 2], max_delay=300, tau=(0.005, 4.0))
    n = 3000
    x = np.random.default_rng(5).standard_normal(n).astype(np.float32)
    z = oracle.filter(bank, x)[0]
    ref = np.zeros_like(z)
    for t in range(bank.n_templates):
        for k in range(bank.offsets[t], bank.offsets[t + 1]):
            a = complex(bank.a[k]); b = complex(bank.b[k]); d = int(bank.d[k])
            xd = np.concatenate([np.zeros(d), x.astype(np.float64)])[:n].astype(np.complex128)
            ref[t] += scipy.signal.lfilter([b], [1.0, -a], xd)
    assert oracle.rel_err(z, ref).max() < 1e-12


def test_steady_state_frequency_response():
    # H_k(w) = b e^{-i w d} / (1 - a e^{-i w}); for x = cos(w0 n) the steady state is
    # (H(w0) e^{i w0 n} + H(-w0) e^{-i w0 n}) / 2.
    bank = small_bank(6, [3], max_delay=20, tau=(0.002, 0.01))
    n = 6000
    w0 = 2 * math.pi * 0.0371
    i = np.arange(n)
    x = np.cos(w0 * i)
    z = oracle.filter(bank, x)[0, 0]
    ref = np.zeros(n, dtype=np.complex128)
    for k in range(3):
        a = complex(bank.a[k]); b = complex(bank.b[k]); d = int(bank.d[k])
        h = lambda w: b * np.exp(-1j * w * d) / (1 - a * np.exp(-1j * w))
        ref += 0.5 * (h(w0) * np.exp(1j * w0 * i) + h(-w0) * np.exp(-1j * w0 * i))
    tail = slice(4000, n)   # |a|^4000 < 1e-40 for tau <= 0.01 s
    assert oracle.rel_err(z[tail], ref[tail]) < 1e-10


def test_white_noise_variance():
    # E|y|^2 = |b|^2 sigma^2 / (1 - |a|^2) for one filter; for two filters
    # E|z|^2 = sum_kl b_k conj(b_l) conj(a_l)^(d_k - d_l) / (1 - a_k conj(a_l)) (d_k >= d_l).
    bank = small_bank(7, [2], max_delay=10, tau=(0.002, 0.004))
    n_samp = 400_000
    x = np.random.default_rng(8).standard_normal(n_samp)
    z = oracle.filter(bank, x)[0, 0][1000:]
    a = bank.a.astype(np.complex128); b = bank.b.astype(np.complex128); d = bank.d.astype(int)

    def cross(k, l):
        if d[k] >= d[l]:
            return b[k] * np.conj(b[l]) * np.conj(a[l]) ** (d[k] - d[l]) / (1 - a[k] * np.conj(a[l]))
        return np.conj(cross(l, k))
    expected = sum(cross(k, l) for k in range(2) for l in range(2)).real
    measured = np.mean(np.abs(z) ** 2)
    # effective number of independent samples ~ n (1 - |a|); allow 6 sigma of a chi-square mean
    n_eff = len(z) * (1 - np.abs(a).max())
    assert abs(measured / expected - 1) < 6 * math.sqrt(2.0 / n_eff)
    # single filter
    bank1 = synth.Bank(np.array([0, 1], np.int32), bank.a[:1], bank.b[:1], bank.d[:1])
    y = oracle.filter(bank1, x)[0, 0][1000:]
    exp1 = abs(b[0]) ** 2 / (1 - abs(a[0]) ** 2)
    assert abs(np.mean(np.abs(y) ** 2) / exp1 - 1) < 6 * math.sqrt(2.0 / n_eff)


def test_linearity_and_superposition():
    bank = small_bank(9, [5, 4], max_delay=100, tau=(0.005, 1.0))
    n = 2000
    rng = np.random.default_rng(10)
    x1 = rng.standard_normal(n); x2 = rng.standard_normal(n)
    al, be = 0.37, -1.9
    lhs = oracle.filter(bank, al * x1 + be * x2)
    rhs = al * oracle.filter(bank, x1) + be * oracle.filter(bank, x2)
    assert oracle.rel_err(lhs, rhs).max() < 1e-12
    # bank(A u B) = bank(A) + bank(B): splitting a template's filters in two adds up
    half = synth.Bank(np.array([0, 2, 5, 7, 9], np.int32), bank.a, bank.b, bank.d)
    zs = oracle.filter(half, x1)[0]
    zf = oracle.filter(bank, x1)[0]
    assert oracle.rel_err(zs[0] + zs[1], zf[0]).max() < 1e-12
    assert oracle.rel_err(zs[2] + zs[3], zf[1]).max() < 1e-12


def test_shift_invariance():
    bank = small_bank(11, [6], max_delay=30, tau=(0.005, 0.2))
    n, s = 1500, 37
    x = np.random.default_rng(12).standard_normal(n)
    xs = np.concatenate([np.zeros(s), x[:n - s]])
    z = oracle.filter(bank, x)[0, 0]
    zs = oracle.filter(bank, xs)[0, 0]
    assert np.array_equal(zs[:s], np.zeros(s))
    assert oracle.rel_err(zs[s:], z[:n - s]) < 1e-13


@pytest.mark.parametrize("chunk", [1, 7, 512, 2048, 5000])
def test_chunking_is_bit_exact(chunk):
    bank = small_bank(13, [9, 3], max_delay=2047, tau=(0.005, 4.0))
    n = 5000
    x = np.random.default_rng(14).standard_normal((2, n)).astype(np.float32)
    whole = oracle.filter(bank, x)
    assert np.array_equal(oracle.filter_stream(bank, x, chunk), whole)


def test_block_carry_identity():
    # y[BL+L-1] = a^L y[BL-1] + sum_{i<L} b a^(L-1-i) x[BL+i-d]
    bank = small_bank(15, [1], max_delay=90, tau=(0.5, 4.0))
    a = complex(bank.a[0]); b = complex(bank.b[0]); d = int(bank.d[0])
    L, n_blk = 128, 6
    x = np.random.default_rng(16).standard_normal(L * n_blk)
    state = np.zeros((1, 1), np.complex128)
    hist = np.zeros((1, bank.max_delay + 1))
    ends = []
    for B in range(n_blk):
        oracle.filter(bank, x[B * L:(B + 1) * L], hist=hist, state=state)
        ends.append(state[0, 0])
        hist = np.concatenate([hist[0], x[B * L:(B + 1) * L]])[-hist.shape[1]:][None]
    xp = np.concatenate([np.zeros(d), x])
    prev = 0j
    for B in range(n_blk):
        i = np.arange(L)
        s = np.sum(b * np.power(a, (L - 1 - i).astype(float)) * xp[B * L + i])
        pred = a ** L * prev + s
        assert abs(ends[B] - pred) <= 1e-12 * max(abs(pred), 1e-30)
        prev = ends[B]


def test_peaks_brute_force_and_ties():
    rng = np.random.default_rng(17)
    z = (rng.standard_normal((3, 1000)) + 1j * rng.standard_normal((3, 1000)))
    z[1, 10] = z[1, 50] = 100.0          # exact tie in window 0 -> lowest index
    z[2, 990] = 7 + 7j                   # ragged last window
    peak, arg, margin = oracle.peaks(z, 256)
    assert peak.shape == (3, 4)
    for r in range(3):
        for w in range(4):
            seg = z[r, w * 256:(w + 1) * 256]
            p = [v.real * v.real + v.imag * v.imag for v in seg]
            best = max(p)
            i1 = p.index(best)
            assert arg[r, w] == i1
            assert peak[r, w] == math.sqrt(best)
            second = sorted(p)[-2]
            assert margin[r, w] == pytest.approx((math.sqrt(best) - math.sqrt(second)) / math.sqrt(best),
                                                 abs=1e-15)
    assert arg[1, 0] == 10 and margin[1, 0] == 0.0


def test_peaks_f32_matches_scalar_loop():
    rng = np.random.default_rng(18)
    z = (rng.standard_normal((2, 300)) + 1j * rng.standard_normal((2, 300))).astype(np.complex64)
    z[0, 5] = z[0, 6]
    peak, arg = oracle.peaks_f32(z, 100)
    for r in range(2):
        for w in range(3):
            best, bi = np.float32(-1), -1
            for i in range(100):
                v = z[r, w * 100 + i]
                re, im = np.float32(v.real), np.float32(v.imag)
                p = np.float32(np.float32(re * re) + np.float32(im * im))
                if p > best:
                    best, bi = p, i
            assert arg[r, w] == bi and peak[r, w] == np.sqrt(best)


def _loss_and_gz(z, w):
    """L = sum |z|^2 + Re sum conj(w) z  ->  dL/dRe z + i dL/dIm z = 2 z + w."""
    return float(np.sum(np.abs(z) ** 2) + np.sum(np.conj(w) * z).real), 2 * z + w


def test_grad_matches_central_differences():
    bank = small_bank(19, [3, 2], max_delay=25, tau=(0.002, 0.05))
    n = 300
    rng = np.random.default_rng(20)
    x = rng.standard_normal((2, n))
    w = rng.standard_normal((2, 2, n)) + 1j * rng.standard_normal((2, 2, n))
    z = oracle.filter(bank, x)
    _, gz = _loss_and_gz(z, w)
    ga, gb = oracle.grad(bank, x, gz)
    # FD on an FP64 copy of the bank (complex128 coefficients)
    base = synth.Bank(bank.offsets, bank.a.astype(np.complex128), bank.b.astype(np.complex128), bank.d)
    h = 1e-6

    def loss(bk):
        return _loss_and_gz(oracle.filter(bk, x), w)[0]

    for k in range(bank.n_filters):
        for which, g in (("a", ga), ("b", gb)):
            num = []
            for step in (h, 1j * h):
                bp = synth.Bank(base.offsets, base.a.copy(), base.b.copy(), base.d)
                bm = synth.Bank(base.offsets, base.a.copy(), base.b.copy(), base.d)
                getattr(bp, which)[k] += step
                getattr(bm, which)[k] -= step
                num.append((loss(bp) - loss(bm)) / (2 * h))
            fd = num[0] + 1j * num[1]
            assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (which, k, fd, g[k])


def test_grad_matches_torch_autograd():
    import torch
    bank = small_bank(21, [4, 3], max_delay=20, tau=(0.002, 0.08))
    n = 200
    rng = np.random.default_rng(22)
    x = rng.standard_normal(n)
    w = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    a = torch.tensor(bank.a.astype(np.complex128), requires_grad=True)
    b = torch.tensor(bank.b.astype(np.complex128), requires_grad=True)
    xt = torch.tensor(x)
    # direct convolution z_t[i] = sum_k b_k sum_m a_k^m x[i-d_k-m]
    zs = []
    for t in range(2):
        zt = torch.zeros(n, dtype=torch.complex128)
        for k in range(bank.offsets[t], bank.offsets[t + 1]):
            d = int(bank.d[k])
            m = torch.arange(n, dtype=torch.float64)
            kern = b[k] * a[k] ** m                       # impulse response, undelayed
            xp = torch.cat([torch.zeros(d, dtype=torch.float64), xt[:n - d]]).to(torch.complex128)
            conv = torch.stack([torch.sum(kern[:i + 1].flip(0) * xp[:i + 1]) for i in range(n)])
            zt = zt + conv
        zs.append(zt)
    z = torch.stack(zs)
    wt = torch.tensor(w)
    loss = torch.sum(z.abs() ** 2) + torch.sum(torch.conj(wt) * z).real
    loss.backward()
    zo = oracle.filter(bank, x)
    _, gz = _loss_and_gz(zo, w[None])
    ga, gb = oracle.grad(bank, x, gz)
    assert np.allclose(ga, a.grad.numpy(), rtol=1e-9, atol=1e-12)
    assert np.allclose(gb, b.grad.numpy(), rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("mode", [0, 1])
def test_overlap_grad_matches_torch_and_fd(mode):
    import torch
    bank = small_bank(23, [4, 5], max_delay=30, tau=(0.002, 0.1))
    n = 256
    rng = np.random.default_rng(24)
    target = (rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n)))
    ov, ga, gb = oracle.overlap_grad(bank, target, mode=mode)
    a = torch.tensor(bank.a.astype(np.complex128), requires_grad=True)
    b = torch.tensor(bank.b.astype(np.complex128), requires_grad=True)
    g = torch.tensor(target)
    m = torch.arange(n, dtype=torch.float64)
    losses = []
    for t in range(2):
        u = torch.zeros(n, dtype=torch.complex128)
        for k in range(bank.offsets[t], bank.offsets[t + 1]):
            d = int(bank.d[k])
            e = (m - d).clamp(min=0)
            u = u + torch.where(m >= d, b[k] * a[k] ** e, torch.zeros((), dtype=torch.complex128))
        c = torch.sum(torch.conj(g[t]) * u)
        num = c.abs() if mode == 0 else c.real
        o = num / (torch.linalg.vector_norm(u) * torch.linalg.vector_norm(g[t]))
        assert float(o) == pytest.approx(ov[t], rel=1e-12)
        losses.append(1 - o)
    loss = sum(losses) / 2
    loss.backward()
    assert np.allclose(ga, a.grad.numpy(), rtol=1e-9, atol=1e-13)
    assert np.allclose(gb, b.grad.numpy(), rtol=1e-9, atol=1e-13)
    # the forward-mode gradient of the same loss, chained through the impulse response
    ov2, _, _ = oracle.overlap_grad(bank, target, mode=mode)
    assert np.array_equal(ov, ov2)


def test_overlap_special_cases():
    # target = e^{i theta} * (the bank's own response): O = 1 (mode 0), cos(theta) (mode 1),
    # and the mode-0 gradient vanishes at this maximum.
    bank = small_bank(25, [6], max_delay=40, tau=(0.002, 0.05))
    n = 512
    u = closed_form_impulse(bank, n)
    theta = 0.7
    ov0, ga0, gb0 = oracle.overlap_grad(bank, np.exp(1j * theta) * u, mode=0)
    ov1, _, _ = oracle.overlap_grad(bank, np.exp(1j * theta) * u, mode=1)
    assert ov0[0] == pytest.approx(1.0, abs=1e-12)
    assert ov1[0] == pytest.approx(math.cos(theta), abs=1e-12)
    assert np.max(np.abs(ga0)) < 1e-9 and np.max(np.abs(gb0)) < 1e-9


def test_overlap_grad_equals_grad_through_impulse():
    # grad() with an impulse input and dL/dz from the overlap loss must agree with
    # the closed-form overlap gradient.
    bank = small_bank(26, [5, 3], max_delay=30, tau=(0.002, 0.1))
    n = 300
    rng = np.random.default_rng(27)
    g = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    u = oracle.filter(bank, synth.impulse(n))[0]
    gz = np.zeros_like(u)
    for t in range(2):
        c = np.sum(np.conj(g[t]) * u[t]); uu = np.sum(np.abs(u[t]) ** 2); ng = np.linalg.norm(g[t])
        alpha = c / (abs(c) * math.sqrt(uu) * ng); beta = abs(c) / (uu * math.sqrt(uu) * ng)
        gz[t] = -(alpha * g[t] - beta * u[t]) / 2
    ga, gb = oracle.grad(bank, synth.impulse(n), gz[None])
    _, ga2, gb2 = oracle.overlap_grad(bank, g, mode=0)
    assert np.allclose(ga, ga2, rtol=1e-9, atol=1e-14)
    assert np.allclose(gb, gb2, rtol=1e-9, atol=1e-14)


def test_cost_model_matches_paper():
    # Section II.B.2: 12 flops per filter per sample; N_m ~ 350, N_T = 412000, 2048 Hz,
    # 3 detectors -> about 10.6 TFLOPS, i.e. about 2200 CPU cores of 4.8 GFLOPS.
    with open(os.path.join(GOLDEN, "cost_model.json")) as f:
        g = json.load(f)
    flops = g["flops_per_filter_sample"] * g["filters_per_template"] * g["templates"] \
        * g["sample_rate_hz"] * g["detectors"]
    assert flops / 1e12 == pytest.approx(g["tflops"], abs=0.05)
    assert flops / g["core_gflops"] / 1e9 == pytest.approx(g["cpu_cores"], rel=0.01)


def test_invalid_arguments_rejected():
    bank = small_bank(28, [2], max_delay=10)
    bad = synth.Bank(bank.offsets, bank.a, bank.b, np.array([-1, 0], np.int32))
    with pytest.raises(ValueError):
        oracle.filter(bad, np.zeros(10))
    with pytest.raises(ValueError):
        oracle.filter(bank, np.zeros(10), hist=np.zeros((1, 3)))   # history shorter than a delay


def test_empty_inputs():
    bank = small_bank(29, [3, 0, 2], max_delay=10)
    z = oracle.filter(bank, np.zeros((1, 0)))
    assert z.shape == (1, 3, 0)
    z = oracle.filter(bank, np.ones(5))
    assert np.all(z[0, 1] == 0)   # a template with no filters outputs zero


def test_noise_power_single_filter_textbook():
    # one filter: E|y|^2 = |b|^2 / (1 - |a|^2) for unit white input
    bank = small_bank(40, [1], max_delay=100, tau=(0.01, 4.0))
    a = complex(bank.a[0]); b = complex(bank.b[0])
    assert oracle.noise_power(bank)[0] == pytest.approx(abs(b) ** 2 / (1 - abs(a) ** 2), rel=1e-12)


def test_noise_power_equals_impulse_energy():
    # Parseval for white input: E|z_t|^2 = sum_m |u_t[m]|^2 (impulse response energy)
    bank = small_bank(41, [7, 3, 12], max_delay=200, tau=(0.002, 0.05))
    n = 6000      # |a|^n < 1e-30 for tau <= 0.05 s
    u = oracle.filter(bank, synth.impulse(n))[0]
    energy = np.sum(np.abs(u) ** 2, axis=-1)
    assert np.allclose(oracle.noise_power(bank), energy, rtol=1e-10)


def test_noise_power_monte_carlo():
    bank = small_bank(42, [6], max_delay=40, tau=(0.002, 0.004))
    x = np.random.default_rng(43).standard_normal(300_000)
    z = oracle.filter(bank, x)[0, 0][500:]
    n_eff = len(z) * (1 - np.abs(bank.a.astype(complex)).max())
    assert abs(np.mean(np.abs(z) ** 2) / oracle.noise_power(bank)[0] - 1) < 6 * math.sqrt(2.0 / n_eff)


def _triggers_brute(z, w, thr, window):
    D, T, n = z.shape
    W = (n + window - 1) // window
    snr = np.zeros((D, T, W), np.float32)
    idx = np.full((D, T, W), -1, np.int32)
    thr2 = np.float32(thr) * np.float32(thr)
    for det in range(D):
        for i in range(n):
            best, bt = np.float32(-1), -1
            for t in range(T):
                re, im = np.float32(z[det, t, i].real), np.float32(z[det, t, i].imag)
                r2 = np.float32(np.float32(np.float32(re * re) + np.float32(im * im)) * np.float32(w[t]))
                if r2 > best:
                    best, bt = r2, t
            if best > thr2:
                wd = i // window
                cur = snr[det, bt, wd] if idx[det, bt, wd] >= 0 else np.float32(-1)
                if best > cur:
                    snr[det, bt, wd], idx[det, bt, wd] = best, i
    got = idx >= 0
    snr[got] = np.sqrt(snr[got])
    return snr, idx


def test_triggers_brute_force_with_ties_and_threshold():
    rng = np.random.default_rng(44)
    D, T, n, window = 2, 5, 300, 64
    z = ((rng.standard_normal((D, T, n)) + 1j * rng.standard_normal((D, T, n))) * 1.6).astype(np.complex64)
    z[0, 2, 10] = z[0, 3, 10] = 9 + 9j          # tie across templates at one sample -> lower t
    z[1, 1, 70] = z[1, 1, 75] = 8 + 8j          # tie within a template's window -> lower sample
    w = rng.uniform(0.5, 1.5, size=T).astype(np.float32)
    snr, idx = oracle.triggers(z, w, 4.0, window)
    snr_b, idx_b = _triggers_brute(z, w, 4.0, window)
    assert np.array_equal(idx, idx_b) and np.array_equal(snr, snr_b)
    assert idx[0, 2, 0] == 10 and idx[0, 3, 0] != 10
    assert idx[1, 1, 1] == 70
    # every trigger is above threshold and at most one per (template, window)
    assert np.all(snr[idx >= 0] > 4.0) and np.all(snr[idx < 0] == 0)


def test_triggers_threshold_is_strict():
    z, w, window, exp_idx, exp_snr = threshold_fixture()
    assert np.float32(np.float32(4.0) * np.float32(4.0)) == np.float32(16.0)
    snr, idx = oracle.triggers(z, w, 4.0, window)
    assert np.array_equal(idx, exp_idx)
    assert np.array_equal(snr, exp_snr)


# ---- signal-consistency statistic (Section II.C.1) ----

def test_autocorr_matches_brute_force_correlation():
    # R_t[j] = sum_m u_t[m+j] conj(u_t[m]) from the impulse response itself, both signs of j
    bank = small_bank(51, [9, 4, 13], max_delay=300, tau=(0.002, 0.03))
    nj, n = 120, 7000            # |a|^n < 1e-40 for tau <= 0.03 s
    u = oracle.filter(bank, synth.impulse(n))[0]
    R = oracle.autocorr(bank, nj)
    for t in range(bank.n_templates):
        for j in range(-nj, nj + 1):
            if j >= 0:
                bf = np.sum(u[t, j:] * np.conj(u[t, :n - j]))
                ref = R[t, j]
            else:
                bf = np.sum(u[t, :n + j] * np.conj(u[t, -j:]))
                ref = np.conj(R[t, -j])
            assert abs(bf - ref) <= 1e-10 * abs(R[t, 0])


def test_autocorr_lag0_is_noise_power():
    bank = small_bank(52, [5, 11], max_delay=2047, tau=(0.005, 4.0))
    R = oracle.autocorr(bank, 3)
    assert np.allclose(R[:, 0].real, oracle.noise_power(bank), rtol=1e-12)
    assert np.all(np.abs(R[:, 0].imag) <= 1e-12 * R[:, 0].real)


def test_xi2_special_cases():
    # a series that is exactly the scaled autocorrelation around the candidate gives 0;
    # one extra complex offset e at one lag gives |e|^2 * (2 / R0) / sum(2 - 2|A|^2)
    bank = small_bank(53, [6, 8], max_delay=100, tau=(0.002, 0.02))
    nj, n, c = 50, 400, 200
    R = oracle.autocorr(bank, nj)
    z = np.zeros((1, 2, n), dtype=np.complex128)
    for t in range(2):
        A = np.concatenate([np.conj(R[t, nj:0:-1]), R[t, :nj + 1]]) / R[t, 0].real
        z[0, t, c - nj:c + nj + 1] = (3.0 - 1.5j) * A
    e = 0.7 + 0.2j
    z[0, 1, c + 7] += e
    idx = np.array([[[c, -1], [c, 5]]], dtype=np.int32)     # second column: none / too close
    x2 = oracle.xi2(z, idx, R, nj)
    A1 = np.concatenate([np.conj(R[1, nj:0:-1]), R[1, :nj + 1]]) / R[1, 0].real
    expect = abs(e) ** 2 * (2.0 / R[1, 0].real) / np.sum(2 - 2 * np.abs(A1) ** 2)
    assert abs(x2[0, 0, 0]) < 1e-24
    assert abs(x2[0, 1, 0] - expect) < 1e-12 * expect
    assert np.isnan(x2[0, 0, 1]) and np.isnan(x2[0, 1, 1])


def test_xi2_has_mean_one_on_white_noise():
    # reduced chi-square: for unit white input every term has expectation 2 - 2|A[j]|^2
    bank = small_bank(54, [8, 8, 8], max_delay=150, tau=(0.002, 0.01))
    nj, n = 60, 240_000
    x = np.random.default_rng(55).standard_normal(n)
    z = oracle.filter(bank, x)
    R = oracle.autocorr(bank, nj)
    pos = np.arange(2000, n - nj - 1, 2 * nj + 1)
    idx = np.broadcast_to(pos, (1, bank.n_templates, len(pos))).astype(np.int32).copy()
    x2 = oracle.xi2(z, idx, R, nj)
    m = float(np.mean(x2))
    assert abs(m - 1.0) < 0.02, m     # mean 1.001, std of the mean 0.003 at this seed


def _acf(R, t, nj):
    return np.concatenate([np.conj(R[t, nj:0:-1]), R[t, :nj + 1]]) / R[t, 0].real


def test_xi2_network_reads_every_detector_at_its_arrival_time():
    # Each detector holds the exact scaled autocorrelation centred where the candidate's
    # direction puts it, s_J = c + tau[p, J] - tau[p, I]: every xi_J^2 is 0 there, so
    # xi^2_C = 0.  The direction with the offsets reversed reads the wrong samples
    # (xi^2_C > 0.1).  An offset e at one lag of one detector gives that detector
    # |e|^2 (2 / R0) / sum(2 - 2|A|^2) and the mean a third of it.
    bank = small_bank(56, [7, 9], max_delay=60, tau=(0.002, 0.02))
    nj, n, c, I = 40, 600, 300, 1
    R = oracle.autocorr(bank, nj)
    tau = np.array([[5, -3, 12], [-5, 3, -12]], dtype=np.int32)
    z = np.zeros((3, 2, n), dtype=np.complex128)
    amp = [1.0 + 2.0j, -0.5 + 0.3j, 2.5 - 1.0j]
    for t in range(2):
        for J in range(3):
            s = c + tau[0, J] - tau[0, I]
            z[J, t, s - nj:s + nj + 1] = amp[J] * _acf(R, t, nj)
    e = 0.4 - 0.9j
    s2 = c + tau[0, 2] - tau[0, I]
    z[2, 1, s2 - 11] += e
    idx = np.full((3, 2, 1), -1, dtype=np.int32)
    idx[I, :, 0] = c
    pix = np.zeros((3, 2, 1), dtype=np.int32)
    per, mean = oracle.xi2_network(z, idx, pix, tau, R, nj)
    assert np.all(np.abs(per[I, 0, 0]) < 1e-24) and abs(mean[I, 0, 0]) < 1e-24
    A1 = _acf(R, 1, nj)
    expect = abs(e) ** 2 * (2.0 / R[1, 0].real) / np.sum(2 - 2 * np.abs(A1) ** 2)
    assert abs(per[I, 1, 0, 2] - expect) < 1e-12 * expect
    assert abs(per[I, 1, 0, 0]) < 1e-24 and abs(per[I, 1, 0, 1]) < 1e-24
    assert abs(mean[I, 1, 0] - expect / 3.0) < 1e-12 * expect
    assert np.all(np.isnan(mean[[0, 2]])) and np.all(np.isnan(per[[0, 2]]))   # no candidate
    pix[:] = 1
    _, wrong = oracle.xi2_network(z, idx, pix, tau, R, nj)
    assert np.all(wrong[I, :, 0] > 0.1)


def test_xi2_network_single_detector_is_xi2():
    bank = small_bank(57, [10, 4, 30], max_delay=200, tau=(0.002, 0.05))
    nj, n = 50, 3000
    x = np.random.default_rng(58).standard_normal((1, n))
    z = oracle.filter(bank, x)
    R = oracle.autocorr(bank, nj)
    idx = np.random.default_rng(59).integers(-1, n, size=(1, 3, 6)).astype(np.int32)
    idx[0, 0, :2] = [10, n - 5]                    # too close to the ends: NaN
    tau = np.array([[17], [-4]], dtype=np.int32)   # one detector: every offset cancels
    pix = (np.arange(18).reshape(1, 3, 6) % 2).astype(np.int32)
    per, mean = oracle.xi2_network(z, idx, pix, tau, R, nj)
    ref = oracle.xi2(z, idx, R, nj)
    assert np.array_equal(np.isnan(mean), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert ok.sum() >= 8
    assert np.array_equal(mean[ok], ref[ok]) and np.array_equal(per[..., 0][ok], ref[ok])


def test_xi2_network_has_mean_one_on_white_noise():
    # three detectors of independent unit white noise, candidates at spaced samples with
    # random directions: the detector average keeps the reduced chi-square's mean 1
    bank = small_bank(60, [8, 8], max_delay=150, tau=(0.002, 0.01))
    nj, n, D = 60, 120_000, 3
    x = np.random.default_rng(61).standard_normal((D, n))
    z = oracle.filter(bank, x)
    R = oracle.autocorr(bank, nj)
    rng = np.random.default_rng(62)
    tau = rng.integers(-44, 45, size=(16, D)).astype(np.int32)
    pos = np.arange(2000, n - 200, 2 * nj + 101)
    idx = np.broadcast_to(pos, (D, bank.n_templates, len(pos))).astype(np.int32).copy()
    pix = rng.integers(0, 16, size=idx.shape).astype(np.int32)
    per, mean = oracle.xi2_network(z, idx, pix, tau, R, nj)
    assert not np.isnan(mean).any()
    m = float(np.mean(mean))
    assert abs(m - 1.0) < 0.03, m
    assert np.allclose(mean, per.mean(axis=-1), rtol=1e-12)


def test_xi2_network_undefined_cases():
    bank = small_bank(63, [5], max_delay=20, tau=(0.002, 0.01))
    nj, n = 10, 200
    R = oracle.autocorr(bank, nj)
    z = np.ones((2, 1, n), dtype=np.complex128)
    tau = np.array([[0, 30]], dtype=np.int32)
    idx = np.array([[[100, 165, -1, 100]], [[50, 20, 100, 100]]], dtype=np.int32)
    pix = np.array([[[0, 0, 0, -1]], [[0, 0, 0, 0]]], dtype=np.int32)
    per, mean = oracle.xi2_network(z, idx, pix, tau, R, nj)
    # det 0: c=100 fine (s_1 = 130); c=165 puts detector 1 at 195 (+10 leaves the series);
    # no candidate; no direction.  det 1: c=50 puts detector 0 at 20 (fine), c=20 at -10
    ok = ~np.isnan(mean)
    assert ok.tolist() == [[[True, False, False, False]], [[True, False, True, True]]]
    assert np.array_equal(np.isnan(per).all(axis=-1), ~ok)


# ---- coherent search (Section II.C.1) ----

def _rand_z(rng, D, T, n, scale=1.0):
    return (rng.standard_normal((D, T, n)) + 1j * rng.standard_normal((D, T, n))) * scale


def test_coherent_plus_null_is_total_power():
    # Eq. null_def: rho_N^2 = sum_I |z_I|^2 - rho_C^2 (U orthogonal); here rho_N^2 comes from
    # the null-space columns, so this checks the two projections against each other
    rng = np.random.default_rng(71)
    D, T, n = 3, 2, 400
    z = _rand_z(rng, D, T, n)
    tab = synth.sky_tables(72, D, 40)
    sh = synth.time_shifts(D, 2, step=20)
    idx = np.array([[[150, 220]] * T] * D, dtype=np.int32)
    assert np.all(sh[:, 0] == 0) and np.all(sh[1, 1:] < 0)      # past data only
    rc, rn = oracle.coherent_map(z, idx, tab.U, tab.tau, sh)
    for I in range(D):
        for t in range(T):
            for w in range(2):
                c = idx[I, t, w]
                for k in range(2):
                    for p in range(40):
                        rel = [(J - I) % D for J in range(D)]
                        s = c + tab.tau[p] - tab.tau[p, I] + sh[k][rel] - sh[k, 0]
                        tot = sum(abs(z[J, t, s[J]]) ** 2 for J in range(D))
                        assert abs(rc[I, t, w, k, p] + rn[I, t, w, k, p] - tot) <= 1e-6 * tot


def test_coherent_signal_in_the_plane_is_found():
    # v = U[p][:, :2] s at direction p: rho_C^2 = |s|^2 there, no null power, and every
    # other direction projects less
    rng = np.random.default_rng(73)
    D, n, c, p0 = 3, 300, 150, 17
    tab = synth.sky_tables(74, D, 64)
    U = tab.U.astype(np.float64)
    s = np.array([2.0 - 1.0j, 0.5 + 3.0j])
    v = U[p0][:, :2] @ s
    z = np.zeros((D, 1, n), dtype=np.complex128)
    idx = np.full((D, 1, 1), -1, dtype=np.int32)
    idx[0, 0, 0] = c
    for J in range(D):
        z[J, 0, c + tab.tau[p0, J] - tab.tau[p0, 0]] = v[J]
    best, pix, null = oracle.coherent(z, idx, tab.U, tab.tau, np.zeros((1, D), np.int32))
    assert pix[0, 0, 0, 0] == p0
    assert abs(best[0, 0, 0, 0] - np.sum(np.abs(s) ** 2)) <= 1e-6 * np.sum(np.abs(s) ** 2)
    assert abs(null[0, 0, 0, 0]) <= 1e-6
    assert np.isnan(best[1:]).all() and (pix[1:] == -1).all()


def test_coherent_two_detectors_has_no_null_space():
    rng = np.random.default_rng(75)
    z = _rand_z(rng, 2, 1, 200)
    tab = synth.sky_tables(76, 2, 10)
    idx = np.array([[[100]], [[80]]], dtype=np.int32)
    rc, rn = oracle.coherent_map(z, idx, tab.U, tab.tau, np.zeros((1, 2), np.int32))
    assert np.all(rn[~np.isnan(rn)] == 0.0)
    for I, c in ((0, 100), (1, 80)):
        for p in range(10):
            s = c + tab.tau[p] - tab.tau[p, I]
            tot = abs(z[0, 0, s[0]]) ** 2 + abs(z[1, 0, s[1]]) ** 2
            assert abs(rc[I, 0, 0, 0, p] - tot) <= 1e-6 * tot


def test_coherent_noise_statistics():
    # Gaussian z of unit variance per quadrature: rho_C^2 is chi-square with 4 degrees of
    # freedom (mean 4), rho_N^2 with 2 N_d - 4 (mean 2 for N_d = 3), at a fixed direction
    rng = np.random.default_rng(77)
    D, n = 3, 60_000
    z = _rand_z(rng, D, 1, n)
    tab = synth.sky_tables(78, D, 3)
    pos = np.arange(100, n - 100, 7)
    idx = np.full((D, 1, len(pos)), -1, dtype=np.int32)
    idx[0, 0, :] = pos
    rc, rn = oracle.coherent_map(z, idx, tab.U, tab.tau, np.zeros((1, D), np.int32))
    mc, mn = np.mean(rc[0, 0, :, 0, :]), np.mean(rn[0, 0, :, 0, :])
    assert abs(mc - 4.0) < 0.1 and abs(mn - 2.0) < 0.07, (mc, mn)

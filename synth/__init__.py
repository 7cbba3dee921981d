"""Seeded synthetic inputs for the SPIIR filter-bank hot path.

This module only draws random numbers and lays them out in arrays.  It holds
none of the filtering arithmetic: both the FP64 oracle and the HIP path read
the arrays it produces, and neither computes its own inputs.

Workload recipe (shapes follow the paper's O3 setting, Section II.B.2:
about 350 filters per template, 2048 Hz sampling, whitened strain):

* filter feedback ``a_k = exp(-dt/tau_k + i*omega_k*dt)`` with
  ``dt = 1/2048 s``, ``tau_k`` log-uniform in [0.005, 4] s and ``omega_k``
  uniform in [2*pi*20, 2*pi*900] rad/s (a first-order complex pole, the
  form ``a = e^{gamma + i omega}`` of Section II.B.1);
* feedforward ``b_k`` complex normal, real and imaginary parts each
  N(0, 1/2), scaled by 1/sqrt(128);
* integer delays ``d_k`` uniform in {0, ..., 2047} samples;
* input: float32 white Gaussian noise with unit variance standing in for
  whitened strain (Eq. whiten), or a unit impulse.

Draw order, per bank generator ``numpy.random.default_rng(seed)`` (PCG64):
filter counts per template (if random), then the vectors ``tau[F]``,
``omega[F]``, ``b_re[F]``, ``b_im[F]``, ``d[F]``.  Noise is ``standard_normal``
float64 draws rounded to float32: either continued from the bank generator
right after the bank (detector 0 first), or, where a workload names noise
seeds, from ``default_rng(noise_seed[i])`` for detector ``i``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

FS = 2048.0            # sample rate, Hz (Section II.A)
DT = 1.0 / FS          # sample interval, s
MAX_DELAY = 2047       # largest integer delay drawn by the recipe
GM_SUN_S = 4.925491e-6  # G*M_sun/c^3 in seconds (textbook constant)


@dataclasses.dataclass
class Bank:
    """A SPIIR bank in CSR form: template t owns filters offsets[t]..offsets[t+1]."""
    offsets: np.ndarray   # int32 [T+1]
    a: np.ndarray         # complex64 [F]
    b: np.ndarray         # complex64 [F]
    d: np.ndarray         # int32 [F]

    @property
    def n_templates(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_filters(self) -> int:
        return int(self.offsets[-1])

    @property
    def max_delay(self) -> int:
        return int(self.d.max()) if self.d.size else 0

    def subset(self, templates: Sequence[int]) -> "Bank":
        """The bank restricted to the given templates, in the given order."""
        offs = [0]
        a, b, d = [], [], []
        for t in templates:
            lo, hi = int(self.offsets[t]), int(self.offsets[t + 1])
            a.append(self.a[lo:hi]); b.append(self.b[lo:hi]); d.append(self.d[lo:hi])
            offs.append(offs[-1] + hi - lo)
        return Bank(np.asarray(offs, np.int32), np.concatenate(a).astype(np.complex64),
                    np.concatenate(b).astype(np.complex64), np.concatenate(d).astype(np.int32))


def counts_uniform(rng: np.random.Generator, n_templates: int, lo: int, hi: int) -> np.ndarray:
    """Filter counts uniform in {lo..hi} (inclusive)."""
    return rng.integers(lo, hi + 1, size=n_templates).astype(np.int64)


def counts_lognormal(rng: np.random.Generator, n_templates: int, median: float = 300.0,
                     sigma: float = 0.5, lo: int = 50, hi: int = 1500) -> np.ndarray:
    """Filter counts lognormal around ``median`` (sigma in ln-space), rounded and clipped."""
    raw = rng.lognormal(mean=math.log(median), sigma=sigma, size=n_templates)
    return np.clip(np.rint(raw), lo, hi).astype(np.int64)


def draw_filters(rng: np.random.Generator, counts: np.ndarray,
                 tau_range=(0.005, 4.0), f_range=(20.0, 900.0),
                 b_scale: float = 1.0 / math.sqrt(128.0), max_delay: int = MAX_DELAY) -> Bank:
    """Draw the per-filter parameters for a bank with the given filter counts."""
    counts = np.asarray(counts, dtype=np.int64)
    n_filters = int(counts.sum())
    offsets = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    tau = np.exp(rng.uniform(math.log(tau_range[0]), math.log(tau_range[1]), size=n_filters))
    omega = rng.uniform(2.0 * math.pi * f_range[0], 2.0 * math.pi * f_range[1], size=n_filters)
    b_re = rng.normal(0.0, math.sqrt(0.5), size=n_filters) * b_scale
    b_im = rng.normal(0.0, math.sqrt(0.5), size=n_filters) * b_scale
    d = rng.integers(0, max_delay + 1, size=n_filters)
    a = np.exp(-DT / tau + 1j * omega * DT).astype(np.complex64)
    b = (b_re + 1j * b_im).astype(np.complex64)
    return Bank(offsets.astype(np.int32), a, b, d.astype(np.int32))


def white_noise(seed: int, n: int) -> np.ndarray:
    """Unit-variance float32 white Gaussian noise from ``default_rng(seed)``."""
    return np.random.default_rng(seed).standard_normal(n).astype(np.float32)


def _noise_from_state(state: dict, n_det: int, n: int) -> np.ndarray:
    rng = np.random.default_rng()
    rng.bit_generator.state = state
    return rng.standard_normal((n_det, n)).astype(np.float32)


def impulse(n: int, at: int = 0) -> np.ndarray:
    x = np.zeros(n, dtype=np.float32)
    if n:
        x[at] = 1.0
    return x


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    bank: Bank
    n_det: int
    n_samples: int          # per detector
    chunk: int              # streaming chunk length (samples)
    description: str
    noise_seeds: Optional[List[int]] = None   # one generator per detector, or
    noise_state: Optional[dict] = None        # continue the bank generator
    impulse_input: bool = False

    def input(self, det: Optional[int] = None) -> np.ndarray:
        """float32 input [n_det][n_samples] (or one detector's row)."""
        if self.impulse_input:
            x = np.stack([impulse(self.n_samples) for _ in range(self.n_det)])
        elif self.noise_seeds is not None:
            x = np.stack([white_noise(s, self.n_samples) for s in self.noise_seeds])
        else:
            x = _noise_from_state(self.noise_state, self.n_det, self.n_samples)
        return x if det is None else x[det]

    @property
    def updates(self) -> int:
        """Filter-sample updates in one pass over the whole stream."""
        return self.bank.n_filters * self.n_det * self.n_samples


def tiny(seed: int = 0) -> Workload:
    """4 templates x 128 filters, 1 detector, 8 s (16384 samples)."""
    rng = np.random.default_rng(seed)
    bank = draw_filters(rng, np.full(4, 128))
    return Workload("tiny", bank, 1, 16384, 16384,
                    "D=1, T=4, F_t=128, N=16384 (8 s), whole stream",
                    noise_state=rng.bit_generator.state)


def realistic(seed: int = 0, n_templates: int = 1024, seconds: int = 64) -> Workload:
    """1024 templates with U{200..800} filters, 1 detector, 64 s in 1-s chunks."""
    rng = np.random.default_rng(seed)
    bank = draw_filters(rng, counts_uniform(rng, n_templates, 200, 800))
    return Workload("realistic", bank, 1, int(FS) * seconds, int(FS),
                    f"D=1, T={n_templates}, F_t~U{{200..800}}, N={int(FS) * seconds}, 1-s chunks",
                    noise_state=rng.bit_generator.state)


def precision(bank_seed: int = 0, noise_seeds=(1, 2, 3), seconds: int = 32,
              n_templates: int = 1024) -> Workload:
    """The realistic bank over 3 independent detector streams of 32 s."""
    rng = np.random.default_rng(bank_seed)
    bank = draw_filters(rng, counts_uniform(rng, n_templates, 200, 800))
    n = int(FS) * seconds
    return Workload("precision", bank, len(noise_seeds), n, n,
                    f"D={len(noise_seeds)}, T={n_templates}, F_t~U{{200..800}}, N={n} each",
                    noise_seeds=list(noise_seeds))


def batching(seed: int = 0, n_templates: int = 16384, seconds: float = 60.0,
             chunk: int = 512, n_det: int = 3) -> Workload:
    """16384 templates with lognormal filter counts, 3 detectors, 0.25-s chunks."""
    rng = np.random.default_rng(seed)
    bank = draw_filters(rng, counts_lognormal(rng, n_templates))
    n = int(round(FS * seconds))
    return Workload("batching", bank, n_det, n, chunk,
                    f"D={n_det}, T={n_templates}, F_t~clip(lognormal(ln 300, 0.5), 50, 1500), "
                    f"N={n}, chunks of {chunk}",
                    noise_state=rng.bit_generator.state)


def differentiation(seed: int = 0, n_templates: int = 256, per_template: int = 512,
                    n_samples: int = 8192) -> Workload:
    """256 x 512 filters driven by a unit impulse; targets from ``chirp_targets``."""
    rng = np.random.default_rng(seed)
    bank = draw_filters(rng, np.full(n_templates, per_template))
    return Workload("differentiation", bank, 1, n_samples, n_samples,
                    f"T={n_templates}, F_t={per_template}, N={n_samples}, impulse input",
                    impulse_input=True)


# ----------------------------------------------------------------------------
# Fit targets: time-reversed complex Newtonian chirps (differentiation workload)
# ----------------------------------------------------------------------------

def chirp_masses(seed: int, n_templates: int, lo: float = 1.0, hi: float = 5.0) -> np.ndarray:
    """Chirp masses (solar masses) uniform in [lo, hi], from ``default_rng(seed + 1000)``."""
    return np.random.default_rng(seed + 1000).uniform(lo, hi, size=n_templates)


def chirp_target(mchirp: float, n_samples: int = 8192, f_end: float = 1024.0) -> np.ndarray:
    """Unit-norm complex64 fit target for one chirp mass.

    Leading-order (Newtonian) inspiral with tau = t_c - t:
    f(tau) = (1/pi) (5/(256 tau))^{3/8} (G Mc/c^3)^{-5/8},
    phi(tau) = -2 (tau / (5 G Mc/c^3))^{5/8}, amplitude ~ tau^{-1/4}.
    The window is the ``n_samples`` samples ending where f reaches ``f_end``.
    The complex template h(phi0=0) + i h(phi0=pi/2) = A e^{-i phi}
    (Section II.B.1) is time-reversed (target[m] = h[N-1-m]) and normalised.
    """
    m = mchirp * GM_SUN_S
    tau_end = (5.0 / 256.0) * (math.pi * f_end) ** (-8.0 / 3.0) * m ** (-5.0 / 3.0)
    j = np.arange(n_samples, dtype=np.float64)
    tau = tau_end + (n_samples - 1 - j) * DT
    phi = -2.0 * (tau / (5.0 * m)) ** (5.0 / 8.0)
    amp = tau ** (-0.25)
    h = amp * np.exp(-1j * phi)
    tgt = h[::-1].copy()
    tgt /= np.linalg.norm(tgt)
    return tgt.astype(np.complex64)


def chirp_targets(seed: int, n_templates: int, n_samples: int = 8192) -> np.ndarray:
    """complex64 [T][n_samples] targets, one chirp mass per template."""
    return np.stack([chirp_target(mc, n_samples) for mc in chirp_masses(seed, n_templates)])


WORKLOADS = {
    "tiny": tiny,
    "realistic": realistic,
    "precision": precision,
    "batching": batching,
    "differentiation": differentiation,
}


# ---- coherent search inputs (Section II.C.1) ----

@dataclasses.dataclass
class SkyTables:
    """Per sky direction p: an orthogonal N_d x N_d matrix U[p] (stands in for the SVD
    factor of the noise-weighted detector response) and the arrival-time offset of every
    detector in samples, tau[p][J].  Detector geometry and sensitivities are not in
    the paper, so the tables are random: U from the QR factorisation of a Gaussian
    matrix (sign-fixed), tau uniform in [-max_offset, max_offset] (44 samples ~ the
    21 ms light travel time across the Earth at 2048 Hz)."""
    U: np.ndarray      # float32 [P][N_d][N_d]
    tau: np.ndarray    # int32 [P][N_d]

    @property
    def n_pix(self) -> int:
        return int(self.U.shape[0])


def sky_tables(seed: int, n_det: int, n_pix: int, max_offset: int = 44) -> SkyTables:
    """Draw order from ``default_rng(seed)``: n_pix Gaussian N_d x N_d matrices, then the
    offsets [n_pix][N_d]."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n_pix, n_det, n_det))
    U = np.empty_like(g)
    for p in range(n_pix):
        q, r = np.linalg.qr(g[p])
        U[p] = q * np.sign(np.diag(r))[None, :]
    tau = rng.integers(-max_offset, max_offset + 1, size=(n_pix, n_det))
    return SkyTables(U.astype(np.float32), tau.astype(np.int32))


def time_shifts(n_det: int, n_shifts: int, step: int = 205) -> np.ndarray:
    """Background time shifts: in shift k (k = 0..n_shifts-1) the detector r positions
    after the candidate's own (cyclically) is read k * step * r samples earlier (step 205
    samples ~ 0.1 s at 2048 Hz), so shift 0 is the unshifted foreground and every shift
    reads only past data.  int32 [n_shifts][N_d], column r."""
    k = np.arange(n_shifts)[:, None]
    r = np.arange(n_det)[None, :]
    return (-k * step * r).astype(np.int32)

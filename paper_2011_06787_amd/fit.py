"""Fitting SPIIR coefficients to target responses with the library's adjoint.

A template is approximated by the summed impulse response of its filters (Section
II.B.1); the fit raises the overlap of Eq. overlap between each template's summed
response u_t and its target g_t.  The paper's own design algorithm is in references
that are not available, so the fit is built here in three steps:

1. ``design`` (host, per template, from the target's phase): filters start where the
   target is, spaced by the target's local coherence length, each with the target's
   local frequency and a decay over that length (delays are then kept fixed);
2. ``project_b``: b_k = <phi_k, g> / ||phi_k||^2, the projection of the target on each
   filter's unit response phi_k[m] = a_k^(m - d_k) (m >= d_k).  Its numerator is the
   library's adjoint: for an impulse input and grad_z = g, spiir_backward returns
   grad_b_k = sum_{m >= d_k} conj(a_k)^(m - d_k) g[m];
3. ``fit``: Adam on the complex a_k, b_k with forward and gradient in libspiir
   (spiir_forward / spiir_backward through the autograd function) and a step schedule
   for the learning rates; a_k is pulled back inside |a| <= a_max after every step.

Torch only holds the parameters and applies the optimiser update.
"""
from __future__ import annotations

import time
from typing import List, Sequence, Tuple

import numpy as np

from . import spiir


def overlap(z, g):
    """|<g, z>| / (||z|| ||g||) per template; z, g complex [T][n] (torch)."""
    import torch
    c = torch.sum(torch.conj(g) * z, dim=-1)
    return c.abs() / (torch.linalg.vector_norm(z, dim=-1) * torch.linalg.vector_norm(g, dim=-1))


def design(targets: np.ndarray, n_filters: int, coherence: float = 1.0,
           min_len: float = 3.0, max_len: float = 4096.0) -> Tuple[np.ndarray, np.ndarray,
                                                                  np.ndarray]:
    """Delays and poles of ``n_filters`` filters per template from each target's phase.

    For target g (complex [n]) with local frequency w[m] = arg(g[m+1] conj(g[m])) (rad per
    sample) and chirp rate k[m] = |w[m+1] - w[m]| (wrapped), a filter that starts at m
    and keeps the frequency w stays in phase with g for about L[m] = coherence / sqrt(k[m])
    samples (clipped to [min_len, max_len]).  Start points are spaced evenly in the
    cumulative density 1/L (dense where the frequency changes fast); filter k gets
    d_k = its start, and a_k = exp(-1/L_k + i w_c) with w_c the frequency at d_k + L_k / 2.
    Returns (offsets int32 [T+1], a complex64 [T*n_filters], d int32 [T*n_filters]).
    """
    targets = np.asarray(targets)
    T, n = targets.shape
    a_all, d_all = [], []
    for t in range(T):
        g = targets[t].astype(np.complex128)
        w = np.angle(g[1:] * np.conj(g[:-1]))
        w = np.concatenate([w, w[-1:]])
        dw = np.angle(np.exp(1j * np.diff(w)))
        k = np.abs(np.concatenate([dw, dw[-1:]])) + 1e-12
        L = np.clip(coherence / np.sqrt(k), min_len, max_len)
        cum = np.concatenate([[0.0], np.cumsum(1.0 / L)])
        q = np.arange(n_filters) / n_filters * cum[-1]
        d = np.clip(np.searchsorted(cum, q, side="right") - 1, 0, n - 1)
        Lk = L[d]
        c = np.clip((d + 0.5 * Lk).astype(np.int64), 0, n - 1)
        a_all.append(np.exp(-1.0 / Lk + 1j * w[c]))
        d_all.append(d)
    offsets = (np.arange(T + 1) * n_filters).astype(np.int32)
    return (offsets, np.concatenate(a_all).astype(np.complex64),
            np.concatenate(d_all).astype(np.int32))


def project_b(bank: spiir.SpiirBank, a, delay, target):
    """b_k = <phi_k, g> / ||phi_k||^2 for every filter (see the module notes).

    ``a`` cuda complex64 [F]; ``delay`` int [F] (host or cuda); ``target`` cuda complex64
    [T][n].  The numerator comes from one spiir_forward (for the checkpoints) and one
    spiir_backward with an impulse input and grad_z = target; ||phi_k||^2 is the closed
    form (1 - |a|^(2(n - d))) / (1 - |a|^2).
    """
    import torch
    n = int(target.shape[-1])
    x = torch.zeros((1, n), dtype=torch.float32, device=target.device)
    x[0, 0] = 1.0
    bank.set_coeffs(a, torch.ones_like(a))
    _, ckpt = bank.forward(x)
    _, num = bank.backward(x, target.reshape(1, *target.shape).contiguous(), ckpt)
    d = torch.as_tensor(np.asarray(delay), device=target.device, dtype=torch.float64)
    r2 = a.abs().double() ** 2
    norm = (1.0 - r2 ** (n - d)) / (1.0 - r2)
    return (num.to(torch.complex128) / norm).to(torch.complex64)


def fit(bank: spiir.SpiirBank, a0, b0, target, steps: int = 50, lr: float = 1e-3,
        a_max: float = 0.99995, lr_a: float = None, milestones: Sequence[int] = (),
        gamma: float = 0.3) -> dict:
    """Adam on (a, b) to maximise the mean overlap with ``target`` (cuda complex64 [T][n]).

    ``bank`` must be an FP32-scan bank with one detector and max_chunk >= n, built on the
    same filter layout (its delays are kept).  ``lr`` is the rate of b, ``lr_a`` that of a
    (default ``lr``); both are multiplied by ``gamma`` at every step in ``milestones``.
    Returns the fitted a, b and the overlap history (mean over templates, one entry per
    step, before the step, then the final value).
    """
    import torch
    n = int(target.shape[-1])
    x = torch.zeros((1, n), dtype=torch.float32, device=target.device)
    x[0, 0] = 1.0                                         # impulse: z is the response u
    a = a0.detach().clone().requires_grad_(True)
    b = b0.detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([{"params": [a], "lr": lr if lr_a is None else lr_a},
                            {"params": [b], "lr": lr}])
    sched = torch.optim.lr_scheduler.MultiStepLR(opt, milestones=list(milestones), gamma=gamma)
    history: List[float] = []
    for _ in range(steps):
        opt.zero_grad()
        z = spiir.spiir_filter(a, b, x, bank)[0]
        ov = overlap(z, target)
        loss = torch.mean(1.0 - ov)
        history.append(float(ov.detach().mean()))
        loss.backward()
        opt.step()
        sched.step()
        with torch.no_grad():
            mag = a.abs()
            scale = torch.clamp(a_max / torch.clamp(mag, min=1e-30), max=1.0)
            a.mul_(scale)
    with torch.no_grad():
        z = spiir.spiir_filter(a, b, x, bank)[0]
        final = overlap(z, target)
    history.append(float(final.mean()))
    return {"a": a.detach(), "b": b.detach(), "overlap_history": history,
            "final_overlap": final.detach()}


def fit_targets(targets: np.ndarray, n_filters: int = 512, steps: int = 200,
                lr_b: float = 1e-3, lr_a: float = 1e-4, milestones: Sequence[int] = (100,),
                coherence: float = 1.0, ckpt_stride: int = 2048, filters_per_lane: int = 4) -> dict:
    """Design, project and fit ``n_filters`` filters to every target (complex [T][n]).

    Returns the bank (offsets, a, b, delays as host arrays), the design's overlap (after
    the projection), the fit's history, and the wall time of each stage (seconds, GPU
    work synchronised).
    """
    import torch
    targets = np.ascontiguousarray(targets, dtype=np.complex64)
    T, n = targets.shape
    t0 = time.perf_counter()
    offsets, a, d = design(targets, n_filters, coherence)
    t1 = time.perf_counter()
    g = torch.from_numpy(targets).cuda()
    a_d = torch.from_numpy(a).cuda()
    with spiir.SpiirBank(offsets, a, np.ones_like(a), d, max_chunk=n, ckpt_stride=ckpt_stride,
                         filters_per_lane=filters_per_lane) as bank:
        b_d = project_b(bank, a_d, d, g)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = fit(bank, a_d, b_d, g, steps=steps, lr=lr_b, lr_a=lr_a, milestones=milestones)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
    return {"offsets": offsets, "delay": d, "a": res["a"].cpu().numpy(),
            "b": res["b"].cpu().numpy(), "a_design": a, "b_design": b_d.cpu().numpy(),
            "design_overlap": res["overlap_history"][0],
            "overlap_history": res["overlap_history"],
            "final_overlap": res["final_overlap"].cpu().numpy(),
            "seconds": {"design": t1 - t0, "projection": t2 - t1, "adam": t3 - t2},
            "steps": steps}

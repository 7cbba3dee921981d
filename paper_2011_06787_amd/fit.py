"""Fitting SPIIR coefficients to target responses with the library's adjoint.

The overlap of Eq. overlap (Section II.B.1) between each template's summed
impulse response u_t and its target g_t is raised by gradient steps on the
complex a_k, b_k (delays fixed).  Forward and gradient both run in libspiir
(spiir_forward / spiir_backward through the autograd function); torch only
holds the parameters and applies the optimiser update.  After every step a_k is
pulled back inside |a| <= a_max so that every filter stays stable.
"""
from __future__ import annotations

from typing import List

from . import spiir


def overlap(z, g):
    """|<g, z>| / (||z|| ||g||) per template; z, g complex [T][n] (torch)."""
    import torch
    c = torch.sum(torch.conj(g) * z, dim=-1)
    return c.abs() / (torch.linalg.vector_norm(z, dim=-1) * torch.linalg.vector_norm(g, dim=-1))


def fit(bank: spiir.SpiirBank, a0, b0, target, steps: int = 50, lr: float = 1e-3,
        a_max: float = 0.99995) -> dict:
    """Adam on (a, b) to maximise the mean overlap with ``target`` (cuda complex64 [T][n]).

    ``bank`` must be an FP32-scan bank with one detector and max_chunk >= n, built on the
    same filter layout (its delays are kept).  Returns the fitted a, b and the overlap
    history (mean over templates, one entry per step, before the step).
    """
    import torch
    n = int(target.shape[-1])
    x = torch.zeros((1, n), dtype=torch.float32, device=target.device)
    x[0, 0] = 1.0                                         # impulse: z is the response u
    a = a0.detach().clone().requires_grad_(True)
    b = b0.detach().clone().requires_grad_(True)
    opt = torch.optim.Adam([a, b], lr=lr)
    history: List[float] = []
    for _ in range(steps):
        opt.zero_grad()
        z = spiir.spiir_filter(a, b, x, bank)[0]
        ov = overlap(z, target)
        loss = torch.mean(1.0 - ov)
        history.append(float(ov.mean()))
        loss.backward()
        opt.step()
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

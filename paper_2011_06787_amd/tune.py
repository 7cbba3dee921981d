"""Autotuner for the schedule of a SPIIR bank.

Times candidate configurations (FP32 scan: filters per lane x schedule, where
the schedule is one wave per filter group walking the packet, the balanced static
schedule with a given number of resident workgroups per compute unit, or the
persistent time-tiled work queue; split-bf16 block form: block length) on the caller's
packet length and detector count, and returns the fastest.  Candidates run on
the real bank, or, for the block form whose operand set grows with the number
of templates, on a seeded sample of templates (the time per filter-sample
update is what is compared; every trial records how many templates it ran).  A
sampled winner is timed again on the whole bank, when its operands fit in device
memory, before it is returned; otherwise the fastest whole-bank trial is.  Every
timing runs the library's own kernels; this module only chooses options.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import spiir

DEFAULT_SCAN = ([dict(filters_per_lane=f, time_tile=t) for f in (1, 2, 4, 8) for t in (0, 512)] +
                [dict(filters_per_lane=f, time_tile=0, balance_wgs=c)
                 for f, c in ((2, 4), (4, 2), (4, 3), (4, 4), (8, 2), (8, 3))])
DEFAULT_BLOCK = [dict(block_len=L) for L in (64, 128, 256)]


@dataclasses.dataclass
class Trial:
    mode: int
    opts: Dict[str, int]
    templates: int
    updates_per_s: float
    ms_per_packet: float
    device_bytes: int = 0


@dataclasses.dataclass
class _Bank:
    offsets: np.ndarray
    a: np.ndarray
    b: np.ndarray
    d: np.ndarray

    @property
    def n_templates(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_filters(self) -> int:
        return int(self.offsets[-1])


def _subset(bank, templates) -> _Bank:
    offs, idx = [0], []
    for t in templates:
        lo, hi = int(bank.offsets[t]), int(bank.offsets[t + 1])
        idx.append(np.arange(lo, hi))
        offs.append(offs[-1] + hi - lo)
    idx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
    return _Bank(np.asarray(offs, np.int32), np.asarray(bank.a)[idx], np.asarray(bank.b)[idx],
                 np.asarray(bank.d)[idx])


def _time_config(bank, x_packets, mode: int, opts: Dict[str, int], reps: int) -> Trial:
    import torch
    D, n = x_packets[0].shape
    kw = dict(n_detectors=D, max_chunk=n, mode=mode, **opts)
    with spiir.SpiirBank.from_bank(bank, **kw) as sb:
        T = sb.n_templates
        z = torch.empty((D, T, n), dtype=torch.complex64, device=x_packets[0].device)
        W = sb.n_windows(n)
        pk = torch.empty((D, T, W), dtype=torch.float32, device=z.device)
        am = torch.empty((D, T, W), dtype=torch.int32, device=z.device)
        for i in range(2):                       # warm-up
            sb.filter_chunk(x_packets[i % len(x_packets)], z, pk, am)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for i in range(reps):
            sb.filter_chunk(x_packets[i % len(x_packets)], z, pk, am)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / reps
        dev_bytes = int(sb.info.device_bytes)
    upd = int(bank.offsets[-1]) * D * n
    return Trial(mode, dict(opts), bank.n_templates, upd / (ms * 1e-3), ms, dev_bytes)


def autotune(bank, x_packets: Sequence, *, scan_candidates: Optional[List[dict]] = None,
             block_candidates: Optional[List[dict]] = None, block_sample_templates: int = 1024,
             reps: int = 10, seed: int = 0):
    """Return (best_trial, all_trials).

    ``x_packets``: a few cuda float32 [D][n] packets of the stream to tune for.
    Block-form candidates need n to be a multiple of their block length; they are
    timed on ``block_sample_templates`` seeded templates (all when fewer; 1024 templates
    of a few hundred filters fill every compute unit).  The returned trial always ran
    on the whole bank.
    """
    scan_candidates = DEFAULT_SCAN if scan_candidates is None else scan_candidates
    block_candidates = DEFAULT_BLOCK if block_candidates is None else block_candidates
    n = int(x_packets[0].shape[1])
    trials: List[Trial] = []
    for opts in scan_candidates:
        trials.append(_time_config(bank, x_packets, spiir.MODE_FP32_SCAN, opts, reps))
    if block_candidates:
        T = bank.n_templates
        if T > block_sample_templates:
            pick = np.sort(np.random.default_rng(seed).choice(T, block_sample_templates,
                                                              replace=False))
            sub = _subset(bank, pick.tolist())
        else:
            sub = bank
        for opts in block_candidates:
            if n % opts.get("block_len", 128) != 0:
                continue
            trials.append(_time_config(sub, x_packets, spiir.MODE_BF16_BLOCK, opts, reps))
    best = max(trials, key=lambda t: t.updates_per_s)
    if best.templates < bank.n_templates:
        # a sampled winner: time it on the whole bank if its operands fit, else fall back
        import torch
        free, _ = torch.cuda.mem_get_info()
        need = best.device_bytes * bank.n_templates / max(best.templates, 1)
        if need < 0.8 * free:
            trials.append(_time_config(bank, x_packets, best.mode, best.opts, reps))
        whole = [t for t in trials if t.templates == bank.n_templates]
        best = max(whole, key=lambda t: t.updates_per_s)
    return best, trials

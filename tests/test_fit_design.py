"""Host part of coefficient fitting: the filter design from a target's phase (no GPU).

The design places filters where the target is and with its local frequency; with b from
the exact projection of the target on each filter's response (an FP64 basis written out
here) the summed response already overlaps the chirp targets of the differentiation
workload above 0.99 (the paper reports overlaps over 97-99% for its designs, Sec. II.B.1
and Sec. III)."""
import numpy as np
import pytest

import oracle
import synth
from paper_2011_06787_amd import fit


def _projection(a, d, g):
    m = np.arange(g.shape[-1])
    k = m[None, :] - d[:, None]
    B = np.where(k >= 0, a.astype(np.complex128)[:, None] ** np.maximum(k, 0), 0)
    return (B.conj() @ g.astype(np.complex128)) / np.sum(np.abs(B) ** 2, axis=1)


def test_design_shapes_and_stability():
    tg = synth.chirp_targets(0, 4, 8192)
    off, a, d = fit.design(tg, 512)
    assert off.tolist() == [0, 512, 1024, 1536, 2048]
    assert a.dtype == np.complex64 and d.dtype == np.int32 and a.shape == d.shape == (2048,)
    assert np.all(np.abs(a) < 1.0) and np.all(np.abs(a) > 0.5)
    assert d.min() == 0 and d.max() < 8192
    for t in range(4):
        assert np.all(np.diff(d[t * 512:(t + 1) * 512]) >= 0)    # start points in order
    # positive frequencies, as the time-reversed chirp has (Sec. II.B.1 template)
    assert np.all(np.angle(a) > 0)


@pytest.mark.parametrize("mc", [1.0, 3.0, 5.0])
def test_design_with_projection_overlaps_the_chirp(mc):
    g = synth.chirp_target(mc, 8192)[None, :]
    off, a, d = fit.design(g, 512)
    b = _projection(a, d, g[0]).astype(np.complex64)
    ov, _, _ = oracle.overlap_grad(synth.Bank(off, a, b, d), g)
    assert ov[0] > 0.99, ov

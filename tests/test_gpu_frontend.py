"""Front end: raw received blocks with a cyclic prefix (Section II-A: the
prefix is the last C samples of the sequence period and is removed before
correlation; Section III-B: removed together with the conversion), and a
chunked host-to-device stream that overlaps copies with estimation.

The prefix is skipped by addressing only, so results equal the estimate of
the prefix-free frames bit for bit; those are checked against the FP64
oracle. Codes from raw blocks equal the oracle's quantiser bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import bf16_round, dev, host, perr

pytestmark = pytest.mark.gpu

SHAPES = [(31, 2, 4, 3, 2, 4), (127, 4, 16, 16, 3, 16), (1023, 16, 32, 64, 4, 32),
          (255, 4, 32, 40, 2, 7)]


def _plan(N, T, L, R):
    from paper_2206_05506_amd import Plan
    return Plan(N, T, L, R)


def _raw(y, cp, seed):
    """Raw blocks: a prefix of cp samples (random here, a real receiver's
    prefix repeats the period's tail) before each row."""
    B, R, N = y.shape
    pre = synth.gaussian((B, R, cp), seed).astype(np.complex64) * 100.0
    return np.concatenate([pre, y], axis=-1)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "N%d_T%d_L%d_R%d_B%d_C%d" % s)
@pytest.mark.parametrize("prec", ["bf16", "f32s", "f32"])
def test_estimate_cp_equals_prefix_free_estimate(shape, prec):
    N, T, L, R, B, cp = shape
    y = synth.gaussian((B, R, N), N + cp).astype(np.complex64)
    yr = _raw(y, cp, 3)
    with _plan(N, T, L, R) as p:
        Hc = p.estimate_cp(dev(yr), cp, prec)
        H = p.estimate(dev(y), prec)
        assert torch.equal(Hc, H)
        s = p.sequence()
        Hh = host(Hc)
    x = bf16_round(y) if prec == "bf16" else y.astype(np.complex128)
    assert perr(Hh, oracle.correlate(x, s, T * L)) <= 1e-5


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("shape", SHAPES[:3], ids=lambda s: "N%d_T%d_L%d_R%d_B%d_C%d" % s)
def test_pack_cp_bit_exact(shape, fmt):
    N, T, L, R, B, cp = shape
    y = synth.gaussian((B, R, N), 2 * N).astype(np.complex64) * np.float32(3.0)
    yr = _raw(y, cp, 4)
    with _plan(N, T, L, R) as p:
        q, sc = p.pack_cp(dev(yr), cp, fmt)
        q, sc = host(q), host(sc)
    ref_q, ref_sc = oracle.quantize(y, fmt)
    assert np.array_equal(sc, ref_sc)
    assert np.array_equal(q.view(ref_q.dtype), ref_q)


def test_stream_from_host_equals_device_estimate():
    N, T, L, R, F, cp, chunk = 1023, 16, 32, 64, 40, 32, 16   # 3 chunks, the last ragged
    y = synth.gaussian((F, R, N), 9).astype(np.complex64)
    yr = _raw(y, cp, 5)
    with _plan(N, T, L, R) as p:
        yh = torch.from_numpy(yr).pin_memory()
        H = p.stream_from_host(yh, cp, chunk, "bf16")
        Hd = p.estimate(dev(y), "bf16")
        torch.cuda.synchronize()
        assert torch.equal(H, Hd)

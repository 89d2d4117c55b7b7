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
@pytest.mark.parametrize("prec", ["bf16", "f32s", "f32", "exact", "exact32"])
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


@pytest.mark.parametrize("prec", ["bf16", "f32s", "f64", "exact"])
@pytest.mark.parametrize("chunk", [16, 1, 64])   # ragged last chunk; one frame; one chunk
def test_stream_from_host_equals_device_estimate(prec, chunk):
    N, T, L, R, F, cp = 1023, 16, 32, 64, 40, 32
    cdt = np.complex128 if prec == "f64" else np.complex64
    y = synth.gaussian((F, R, N), 9).astype(cdt)
    yr = _raw(y, cp, 5).astype(cdt)
    with _plan(N, T, L, R) as p:
        yh = torch.from_numpy(yr).pin_memory()
        H = p.stream_from_host(yh, cp, chunk, prec)
        Hd = p.estimate_cp(dev(yr, yh.dtype), cp, prec)
        torch.cuda.synchronize()
        assert torch.equal(H, Hd)
        s = p.sequence()
        Hh = host(H[::13])
    x = bf16_round(y[::13]) if prec == "bf16" else y[::13].astype(np.complex128)
    assert perr(Hh, oracle.correlate(x, s, T * L)) <= 1e-5


def test_stream_from_host_back_to_back_reuses_staging():
    """Two calls sharing one staging buffer and one copy stream, the second
    with other frames and the copy stream equal to the compute stream: the
    second call's copies must wait for the first call's estimates."""
    N, T, L, R, cp, chunk = 255, 4, 32, 40, 8, 3
    ya = synth.gaussian((7, R, N + cp), 11).astype(np.complex64)
    yb = synth.gaussian((5, R, N + cp), 12).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        staging = torch.empty((2 * chunk * R * (N + cp) * 8,), dtype=torch.uint8, device="cuda")
        ha = torch.from_numpy(ya).pin_memory()
        hb = torch.from_numpy(yb).pin_memory()
        Ha = p.stream_from_host(ha, cp, chunk, "f32s", staging=staging)
        Hb = p.stream_from_host(hb, cp, chunk, "f32s", staging=staging,
                                copy_stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert torch.equal(Ha, p.estimate_cp(dev(ya), cp, "f32s"))
        assert torch.equal(Hb, p.estimate_cp(dev(yb), cp, "f32s"))
        with pytest.raises(ValueError):
            p.stream_from_host(ha, cp, chunk, "f32s", staging=staging[:-1])
        with pytest.raises(ValueError):
            p.stream_from_host(ha, cp, 0, "f32s")
        # a chunk larger than the batch is one chunk of the whole batch
        Hc = p.stream_from_host(ha, cp, 1 << 30, "f32s")
        torch.cuda.synchronize()
        assert torch.equal(Hc, Ha)
        empty = torch.empty((0, R, N + cp), dtype=torch.complex64).pin_memory()
        assert p.stream_from_host(empty, cp, chunk, "bf16").shape == (0, R, T * L)

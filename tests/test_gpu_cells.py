"""Eq. 8 lag spacing and per-cell m-sequences (Section II-B) on the GPU.

Plans made with spacing "eq8" put transmitter t's L lags at floor(N/T)*t + l
(the circular shift of Eq. 8), leaving guard lags between the blocks; plans
made with another primitive feedback polynomial use another cell's
m-sequence. Every entry point follows the plan's lags; each is compared with
the oracle at the same lags and sequence, to the same bars as the adjacent
layout: bit-exact sequences and lag lists, 1e-5 normwise for FP32-accurate
and bf16-operand contractions (the oracle rounding the same operands),
2e-7 for FP64 sums rounded once to FP32, 1e-12 for FP64.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import bf16_round, dev, host, perr

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL_F64ACC = 2e-7
TOL_EXACT32 = 4e-7  # exact sums, then an FP32 epilogue of a few roundings
TOLS = {"f64acc": TOL_F64ACC, "exact": TOL_F64ACC, "exact32": TOL_EXACT32}
TOL64 = 1e-12

# (N, T, L, R, B) with T*L <= N: guards of every width (none for D = L), L
# not a multiple of 32 (padded column segments), single-tap channels, one
# transmitter, ragged antenna blocks, several column groups, the FP32
# baseline frame shape.
SHAPES = [
    (7, 2, 3, 5, 2),
    (7, 7, 1, 3, 1),
    (31, 3, 5, 7, 3),
    (63, 5, 12, 9, 2),
    (127, 3, 1, 4, 2),
    (127, 4, 16, 16, 1),
    (255, 1, 100, 8, 2),
    (255, 7, 36, 40, 2),
    (511, 8, 32, 33, 2),
    (1023, 16, 32, 64, 3),
    (2047, 16, 64, 32, 1),
    (4095, 32, 64, 32, 1),
]
IDS = ["N%d_T%d_L%d_R%d_B%d" % s for s in SHAPES]


def other_mask(d):
    """A primitive feedback mask of degree d other than the plan default:
    the largest below 2^d that the oracle accepts."""
    for m in range((1 << d) - 1, 0, -1):
        if oracle.mseq_mask(d, m) is not None:
            return m
    raise AssertionError(d)


def _plan(N, T, L, R, spacing="eq8", feedback=0):
    from paper_2206_05506_amd import Plan
    return Plan(N, T, L, R, feedback=feedback, spacing=spacing)


def _y(N, R, B, seed):
    return synth.gaussian((B, R, N), seed).astype(np.complex64)


@pytest.mark.parametrize("d", list(range(2, 17)))
def test_cell_sequence_and_feedback_bit_exact(d):
    N = (1 << d) - 1
    m = other_mask(d)
    with _plan(N, 1, 1, 1, "adjacent", feedback=m) as p:
        assert p.feedback() == m
        assert np.array_equal(p.sequence(), oracle.mseq_mask(d, m))
    with _plan(N, 1, 1, 1, "adjacent") as p:
        assert np.array_equal(p.sequence(), oracle.mseq(d))


@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_lags_bit_exact(shape):
    N, T, L, R, _ = shape
    for spacing in ("adjacent", "eq8"):
        with _plan(N, T, L, R, spacing) as p:
            want = oracle.lags(N, T, L, "contiguous" if spacing == "adjacent" else "eq8")
            assert np.array_equal(p.lags(), want)


def test_eq8_rejects_overlapping_blocks():
    from paper_2206_05506_amd._lib import PnceError
    with pytest.raises(PnceError):
        _plan(127, 8, 16, 4)
    with pytest.raises(PnceError):
        _plan(63, 2, 4, 4, "adjacent", feedback=0x9)   # not primitive


@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
@pytest.mark.parametrize("prec", ["f32", "f32s", "bf16", "f64acc", "exact", "exact32"])
def test_estimate_parity(shape, prec):
    N, T, L, R, B = shape
    d = oracle.degree_of(N)
    m = other_mask(d)
    y = _y(N, R, B, N + T + L)
    with _plan(N, T, L, R, feedback=m) as p:
        s, lag = p.sequence(), p.lags()
        H = host(p.estimate(dev(y), prec))
    assert np.array_equal(s, oracle.mseq_mask(d, m))
    assert np.array_equal(lag, oracle.lags(N, T, L, "eq8"))
    x = bf16_round(y) if prec == "bf16" else y.astype(np.complex128)
    ref = oracle.correlate(x, s, T * L, lag)
    err = perr(H, ref)
    print(f"eq8 estimate {prec} N={N} T={T} L={L}: relerr {err:.3e}")
    assert err <= TOLS.get(prec, TOL32)


@pytest.mark.parametrize("shape", [SHAPES[1], SHAPES[2], SHAPES[7]], ids=[IDS[1], IDS[2], IDS[7]])
def test_estimate_f64_parity(shape):
    N, T, L, R, B = shape
    y = synth.gaussian((B, R, N), 5)
    with _plan(N, T, L, R) as p:
        H = host(p.estimate(dev(y, torch.complex128), "f64"))
        ref = oracle.correlate(y, p.sequence(), T * L, oracle.lags(N, T, L, "eq8"))
    assert perr(H, ref) <= TOL64


@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
@pytest.mark.parametrize("prec", ["f32", "f32s", "bf16", "f64acc", "exact", "exact32"])
def test_adjoint_parity(shape, prec):
    """One contraction over the lag blocks (zero in the guard lags), with
    alpha / beta."""
    N, T, L, R, B = shape
    K = T * L
    G = synth.gaussian((B, R, K), K + R).astype(np.complex64)
    C = synth.gaussian((B, R, N), N).astype(np.complex64)
    lag = oracle.lags(N, T, L, "eq8")
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        A = host(p.adjoint(dev(G), prec))
        A2 = host(p.adjoint(dev(G), prec, alpha=-1.0, beta=1.0, C=dev(C)))
    g = bf16_round(G) if prec == "bf16" else G.astype(np.complex128)
    ref = oracle.adjoint(g, s, lag)
    tol = TOLS.get(prec, TOL32)
    err = perr(A, ref)
    print(f"eq8 adjoint {prec} N={N} T={T} L={L}: relerr {err:.3e}")
    assert err <= tol
    assert perr(A2, C.astype(np.complex128) - N * ref) <= tol


def test_adjoint_f64_and_dot_identity():
    N, T, L, R, B = 63, 3, 7, 4, 2
    K = T * L
    G = synth.gaussian((B, R, K), 1)
    Y = synth.gaussian((B, R, N), 2)
    lag = oracle.lags(N, T, L, "eq8")
    with _plan(N, T, L, R) as p:
        A = host(p.adjoint(dev(G, torch.complex128), "f64"))
        H = host(p.estimate(dev(Y, torch.complex128), "f64"))
        s = p.sequence()
    assert perr(A, oracle.adjoint(G, s, lag)) <= TOL64
    assert abs(np.vdot(G, H) - np.vdot(A, Y)) <= 1e-12 * abs(np.vdot(G, H))


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_estimate_packed_parity(shape, fmt):
    N, T, L, R, B = shape
    y = _y(N, R, B, 11)
    with _plan(N, T, L, R) as p:
        q, sc = p.pack(dev(y), fmt)
        H = host(p.estimate_packed(q, sc, fmt))
        s = p.sequence()
        qh, sch = host(q), host(sc)
    x = oracle.dequantize(qh.view(np.uint8 if fmt == "e4m3" else np.uint16), sch, fmt, N)
    ref = oracle.correlate(x, s, T * L, oracle.lags(N, T, L, "eq8"))
    assert perr(H, ref) <= TOL32


@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
@pytest.mark.parametrize("prec", ["f32s", "bf16"])
def test_estimate_ls_parity(shape, prec):
    """The closed form holds for any K distinct lags, so the same rows."""
    N, T, L, R, B = shape
    y = _y(N, R, B, 3 * N)
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        yd = dev(y)
        X = host(p.estimate_ls(yd, prec))
        H = p.estimate(yd, prec)
        p.debias(H)
        Hh = host(H)
    x = bf16_round(y) if prec == "bf16" else y.astype(np.complex128)
    ref = oracle.ls_closed_form(oracle.correlate(x, s, T * L, oracle.lags(N, T, L, "eq8")), N)
    assert perr(X, ref) <= TOL32
    assert perr(Hh, ref) <= TOL32


@pytest.mark.parametrize("shape", [(127, 4, 16, 8, 2), (1023, 16, 32, 16, 2), (255, 3, 50, 8, 1)],
                         ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
def test_noiseless_eq8_channels_are_recovered(shape):
    """Frames built by the oracle's receive model with Eq. 8's shifts:
    least-squares rows give back every CIR to FP32 rounding, the correlator
    alone leaves the -sum(h)/N bias of Eq. 1."""
    N, T, L, R, B = shape
    s = oracle.mseq(oracle.degree_of(N))
    lag = oracle.lags(N, T, L, "eq8")
    h = synth.gaussian((B, R, T, L), 7)
    y, _ = oracle.received(s, h, np.zeros((B, R, N)), np.full(B, 300.0),
                           shifts=lag.reshape(T, L)[:, 0])
    with _plan(N, T, L, R) as p:
        X = host(p.estimate_ls(dev(y.astype(np.complex64)), "f32s"))
        H = host(p.estimate(dev(y.astype(np.complex64)), "f32s"))
    hs = h.reshape(B, R, T * L)
    assert perr(X, hs) <= 1e-5
    expect = hs + (hs - hs.sum(axis=-1, keepdims=True)) / N
    assert perr(H, expect) <= 1e-5


@pytest.mark.parametrize("shape", [(127, 4, 16, 16, 1), (1023, 16, 32, 64, 2), (255, 7, 36, 8, 2)],
                         ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
def test_refine_tracks_fp64_iterates(shape):
    """Refinement on an Eq. 8 plan: each iterate within 1e-5 of the FP64
    oracle iterate at the same lags (last residual on FP64 matrix cores)."""
    N, T, L, R, B = shape
    s = oracle.mseq(oracle.degree_of(N))
    lag = oracle.lags(N, T, L, "eq8")
    h = synth.gaussian((B, R, T, L), 9)
    w = synth.gaussian((B, R, N), 10)
    y, _ = oracle.received(s, h, w, np.full(B, 20.0), shifts=lag.reshape(T, L)[:, 0])
    y = y.astype(np.complex64)
    its = oracle.refine(y, s, T * L, 5, lag)
    with _plan(N, T, L, R) as p:
        yd = dev(y)
        for k in range(6):
            X = p.estimate(yd, "f32s")
            p.refine(yd, X, k)
            err = perr(host(X), its[k])
            print(f"eq8 refine k={k}: relerr vs FP64 iterate {err:.3e}")
            assert err <= TOL32


@pytest.mark.parametrize("prec", ["f32s", "bf16"])
def test_estimate_cp_parity(prec):
    N, T, L, R, B, cp = 255, 5, 24, 12, 3, 24
    raw = synth.gaussian((B, R, cp + N), 12).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        H = host(p.estimate_cp(dev(raw), cp, prec))
        s = p.sequence()
    y = raw[:, :, cp:]
    x = bf16_round(y) if prec == "bf16" else y.astype(np.complex128)
    assert perr(H, oracle.correlate(x, s, T * L, oracle.lags(N, T, L, "eq8"))) <= TOL32


def test_other_cell_interference_matches_oracle():
    """A receiver of cell A correlating a frame of cell B (the decimated
    sequence, a preferred pair): the GPU output equals the oracle's
    correlation of that frame with A's sequence (the cross-correlation
    floor), while B's own plan recovers B's channels."""
    d = 9
    N = (1 << d) - 1
    T, L, R, B = 4, 32, 8, 2
    sa = oracle.mseq(d)
    sb = sa[(3 * np.arange(N)) % N].copy()
    mb = [m for m in oracle.primitive_masks(d)
          if any(np.array_equal(np.roll(oracle.mseq_mask(d, m), k), sb) for k in range(N))][0]
    sb = oracle.mseq_mask(d, mb)                      # B's own plan sequence
    lag = oracle.lags(N, T, L, "eq8")
    h = synth.gaussian((B, R, T, L), 13)
    y, _ = oracle.received(sb, h, np.zeros((B, R, N)), np.full(B, 300.0),
                           shifts=lag.reshape(T, L)[:, 0])
    y = y.astype(np.complex64)
    with _plan(N, T, L, R) as pa, _plan(N, T, L, R, feedback=mb) as pb:
        Ha = host(pa.estimate(dev(y), "f32s"))
        Hb = host(pb.estimate_ls(dev(y), "f32s"))
    assert perr(Ha, oracle.correlate(y, sa, T * L, lag)) <= TOL32
    assert perr(Hb, h.reshape(B, R, T * L)) <= 1e-5


def test_autograd_follows_eq8_lags():
    from paper_2206_05506_amd.autograd import correlate, residual_loss
    N, T, L, R, B = 255, 4, 20, 8, 2
    lag = oracle.lags(N, T, L, "eq8")
    Y = synth.gaussian((B, R, N), 3).astype(np.complex64)
    G = synth.gaussian((B, R, T * L), 4).astype(np.complex64)
    x = synth.gaussian((B, R, T * L), 6).astype(np.complex64) * 0.1
    with _plan(N, T, L, R) as p:
        Yd = dev(Y).requires_grad_(True)
        (gY,) = torch.autograd.grad(correlate(Yd, p, "f32s"), Yd, grad_outputs=dev(G))
        xd = dev(x).requires_grad_(True)
        loss = residual_loss(dev(Y), xd, p, "f32s")
        (g,) = torch.autograd.grad(loss, xd)
        s = p.sequence()
    assert perr(host(gY), oracle.adjoint(G, s, lag)) <= TOL32
    ref_loss, ref_g = oracle.loss_grad(Y, s, x, lag)
    assert abs(float(loss.detach()) - ref_loss) <= 1e-5 * ref_loss
    assert perr(host(g), ref_g) <= TOL32


def test_fp32_baseline_shape_eq8_full_batch_sampled():
    """The FP32-baseline workload (N=1023, T=16, L=32, R=64, B=256) on an
    Eq. 8 plan in the benchmark's launch configuration; sampled frames
    checked against the oracle."""
    cfg = synth.FP32
    N, T, L, R, B = cfg.N, cfg.T, cfg.L, cfg.R, cfg.B
    y = synth.gaussian((B, R, N), 21).astype(np.complex64)
    lag = oracle.lags(N, T, L, "eq8")
    with _plan(N, T, L, R) as p:
        yd = dev(y)
        Hb = host(p.estimate(yd, "bf16"))
        Xs = host(p.estimate_ls(yd, "f32s"))
        s = p.sequence()
    pick = [0, 101, 255]
    assert perr(Hb[pick], oracle.correlate(bf16_round(y[pick]), s, T * L, lag)) <= TOL32
    ref = oracle.ls_closed_form(oracle.correlate(y[pick], s, T * L, lag), N)
    assert perr(Xs[pick], ref) <= TOL32

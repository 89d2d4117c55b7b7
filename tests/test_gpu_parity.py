"""GPU parity of libpnce.so against the FP64 oracle, through the C ABI.

Tolerances (written here, derived in the design notes):
  * FP32-accurate contractions (f32, f32s): normwise relative error per frame
    <= 1e-5 against the FP64 oracle on the same input.
  * bf16 in-register rounding: the oracle correlates the same bf16-rounded
    input, so only FP32 accumulation differs: the same 1e-5 bound.
  * f64: 1e-12.
  * integer/byte work (sequence, quantised codes, scales): bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import bf16_round, dev, frames, host, perr, tol_sum

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-12

# (N, T, L, R, B): several tiles, ragged antenna blocks and column groups,
# tiny degenerate sizes, the lag-alias case (T*L > N) and the plain workload.
SHAPES = [
    (3, 1, 2, 1, 1),        # d = 2: one-chunk reduction, K < 32
    (7, 2, 3, 5, 2),        # d = 3
    (31, 2, 4, 2, 1),       # gradient-check instance
    (31, 3, 5, 7, 3),       # ragged R and K
    (63, 5, 16, 9, 2),      # T*L = 80 > N = 63: lag alias
    (127, 4, 16, 16, 1),    # plain workload
    (255, 4, 32, 40, 2),    # K = 128, two antenna blocks (ragged)
    (511, 8, 32, 33, 2),    # K = 256, NC = 2 tiles, 33 antennas
    (1023, 16, 32, 64, 3),  # FP32-baseline frame shape
    (2047, 16, 64, 32, 1),  # K = 1024: two column groups
    (4095, 32, 64, 32, 1),  # precision-study frame shape (R reduced)
]


def _plan(N, T, L, R):
    from paper_2206_05506_amd import Plan
    return Plan(N, T, L, R)


def _rand_frames(N, R, B, seed):
    return synth.gaussian((B, R, N), seed).astype(np.complex64)


@pytest.mark.parametrize("d", list(range(2, 17)))
def test_sequence_bit_exact(d):
    N = (1 << d) - 1
    with _plan(N, 1, 1, 1) as p:
        assert np.array_equal(p.sequence(), oracle.mseq(d))


TOL_F64ACC = 2e-7   # FP64 sums, one rounding of each output to FP32
# four int8 digits: exact sums (fixed point at 2^-30 of the row's largest
# element), then an FP32 epilogue of a few roundings of 2^-24
TOL_EXACT32 = 4e-7
TOLS = {"f64acc": TOL_F64ACC, "exact": TOL_F64ACC, "exact32": TOL_EXACT32}


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
@pytest.mark.parametrize("prec", ["f32", "f32s", "bf16", "f64acc", "exact", "exact32"])
def test_estimate_parity(shape, prec):
    N, T, L, R, B = shape
    K = T * L
    y = _rand_frames(N, R, B, seed=N + K + R)
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        H = host(p.estimate(dev(y), prec))
        torch.cuda.synchronize()
    x = bf16_round(y) if prec == "bf16" else y.astype(np.complex128)
    ref = oracle.correlate(x, s, K)
    err = perr(H, ref)
    print(f"estimate {prec} N={N} K={K} R={R} B={B}: relerr {err:.3e}")
    assert err <= TOLS.get(prec, TOL32)


@pytest.mark.parametrize("shape", [SHAPES[2], SHAPES[4], SHAPES[6]],
                         ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
def test_estimate_f64_parity(shape):
    N, T, L, R, B = shape
    y = synth.gaussian((B, R, N), 5)
    with _plan(N, T, L, R) as p:
        H = host(p.estimate(dev(y, torch.complex128), "f64"))
        ref = oracle.correlate(y, p.sequence(), T * L)
    assert perr(H, ref) <= TOL64


def test_estimate_plain_workload_structured():
    """Plain workload (N=127, T=4, L=16, R=16, SNR 10 dB) on the seeded
    multiplexed frame, and the noiseless bias closed form on the GPU."""
    cfg = synth.PLAIN
    y, h, s = frames(cfg)
    with _plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
        H = host(p.estimate(dev(y), "f32s"))
        y0, _ = oracle.received(s, h, np.zeros_like(y), np.array([300.0]))
        H0 = host(p.estimate(dev(y0.astype(np.complex64)), "f32"))
    assert perr(H, oracle.correlate(y, s, cfg.K)) <= TOL32
    hs = h.reshape(1, cfg.R, cfg.K)
    expect = hs + (hs - hs.sum(axis=-1, keepdims=True)) / cfg.N
    assert perr(H0, expect) <= TOL32


def test_estimate_scales_and_beta():
    N, T, L, R, B = 255, 4, 16, 8, 3
    y = _rand_frames(N, R, B, 7)
    H0 = synth.gaussian((B, R, T * L), 8).astype(np.complex64)
    sc = np.array([0.5, 2.0, 3.0], dtype=np.float32)
    with _plan(N, T, L, R) as p:
        Hd = dev(H0)
        p.estimate(dev(y), "f32s", out=Hd, scales=torch.from_numpy(sc).cuda(), beta=0.25)
        H = host(Hd)
        ref = sc[:, None, None] * oracle.correlate(y, p.sequence(), T * L) + 0.25 * H0
    assert perr(H, ref) <= TOL32


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
@pytest.mark.parametrize("prec", ["f32", "f32s", "f64acc", "exact", "exact32"])
def test_adjoint_parity(shape, prec):
    N, T, L, R, B = shape
    K = T * L
    G = synth.gaussian((B, R, K), K + R).astype(np.complex64)
    C = synth.gaussian((B, R, N), N).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        A = host(p.adjoint(dev(G), prec))
        A2 = host(p.adjoint(dev(G), prec, alpha=-1.0, beta=1.0, C=dev(C)))
    ref = oracle.adjoint(G, s)
    tol = TOLS.get(prec, TOL32)
    assert perr(A, ref) <= tol
    ref2 = C.astype(np.complex128) - N * ref
    assert perr(A2, ref2) <= tol


def test_adjoint_f64_and_dot_identity():
    N, T, L, R, B = 63, 3, 8, 4, 2
    G = synth.gaussian((B, R, T * L), 1)
    Y = synth.gaussian((B, R, N), 2)
    with _plan(N, T, L, R) as p:
        A = host(p.adjoint(dev(G, torch.complex128), "f64"))
        H = host(p.estimate(dev(Y, torch.complex128), "f64"))
        assert perr(A, oracle.adjoint(G, p.sequence())) <= TOL64
    assert abs(np.vdot(G, H) - np.vdot(A, Y)) < 1e-10 * abs(np.vdot(G, H))


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("shape", [(31, 2, 4, 3, 2), (255, 4, 32, 40, 2), (1023, 16, 32, 64, 2)],
                         ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
def test_pack_bit_exact(shape, fmt):
    N, T, L, R, B = shape
    y = _rand_frames(N, R, B, 3) * np.array([1e-3, 40.0])[:B, None, None].astype(np.float32)
    y[0, 0, 0] = 0.0
    with _plan(N, T, L, R) as p:
        q, sc = p.pack(dev(y), fmt)
        q = host(q)
        sc = host(sc)
    ref_q, ref_sc = oracle.quantize(y, fmt)
    assert np.array_equal(sc, ref_sc)
    assert np.array_equal(q.view(ref_q.dtype), ref_q)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
def test_pack_degenerate_frames(fmt):
    """An all-zero frame and a frame holding +-inf both get scale 1; the
    infinity encodes as the format's inf (e4m3: saturates to +-448); a frame
    whose maximum sits exactly on a power of two keeps that power."""
    N, T, L, R = 63, 2, 8, 5
    y = _rand_frames(N, R, 4, 21)
    y[0] = 0.0
    y[1, 2, 9] = np.inf
    y[1, 4, 0] = -np.inf + 1j
    y[2] *= np.float32(0.49) / max(np.abs(y[2].real).max(), np.abs(y[2].imag).max())
    y[2, 1, 3] = 0.5
    y[3, 0, 0] = 1e-30
    with _plan(N, T, L, R) as p:
        q, sc = p.pack(dev(y), fmt)
        q, sc = host(q), host(sc)
    ref_q, ref_sc = oracle.quantize(y, fmt)
    assert sc[0] == 1.0 and sc[1] == 1.0
    assert sc[2] == (0.5 if fmt != "e4m3" else 2.0 ** -9)
    assert np.array_equal(sc, ref_sc)
    assert np.array_equal(q.view(ref_q.dtype), ref_q)


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
def test_estimate_packed_parity(shape, fmt):
    N, T, L, R, B = shape
    y = _rand_frames(N, R, B, 11)
    with _plan(N, T, L, R) as p:
        q, sc = p.pack(dev(y), fmt)
        H = host(p.estimate_packed(q, sc, fmt))
        s = p.sequence()
        qh, sch = host(q), host(sc)
    x = oracle.dequantize(qh.view(np.uint8 if fmt == "e4m3" else np.uint16), sch, fmt, N)
    ref = oracle.correlate(x, s, T * L)
    assert perr(H, ref) <= TOL32


@pytest.mark.parametrize("shape", [(127, 4, 16, 16, 1), (1023, 16, 32, 64, 2), (255, 4, 16, 8, 2)],
                         ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
def test_refine_tracks_fp64_iterates(shape):
    """Each refinement iterate within 1e-5 of the FP64 oracle iterate with the
    same step count (started from the FP64 correlation of the same y)."""
    N, T, L, R, B = shape
    cfg = synth.Config("t", oracle.degree_of(N), T, L, R, B, 8.0, 0.0, 20.0, 9)
    y, h, s = frames(cfg)
    its = oracle.refine(y, s, cfg.K, 5)
    with _plan(N, T, L, R) as p:
        yd = dev(y)
        for k in range(6):
            X = p.estimate(yd, "f32s")
            p.refine(yd, X, k)
            err = perr(host(X), its[k])
            print(f"refine k={k}: relerr vs FP64 iterate {err:.3e}")
            assert err <= TOL32


def test_fp32_baseline_full_batch_sampled():
    """Full FP32-baseline workload (N=1023, T=16, L=32, R=64, B=256) in the
    benchmark's launch configuration; sampled frames checked by the oracle."""
    cfg = synth.FP32
    y, _, s = frames(cfg)
    with _plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
        yd = dev(y)
        Hs = host(p.estimate(yd, "f32s"))
        Hb = host(p.estimate(yd, "bf16"))
        Hf = host(p.estimate(yd, "f32"))
    pick = [0, 1, 97, 128, 255]
    ref = oracle.correlate(y[pick], s, cfg.K)
    assert perr(Hs[pick], ref) <= TOL32
    assert perr(Hf[pick], ref) <= TOL32
    refb = oracle.correlate(bf16_round(y[pick]), s, cfg.K)
    assert perr(Hb[pick], refb) <= TOL32


def test_tile_width_does_not_change_results():
    """One frame alone launches narrow column tiles (spread over more compute
    units); the same frame inside a 256-frame batch uses full-width tiles.
    The k-step order per output is the same, so the CIRs agree bit for bit."""
    cfg = synth.FP32
    y, _, s = frames(cfg)
    with _plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
        yd = dev(y)
        for prec in ("bf16", "f32s", "f32"):
            Hb = p.estimate(yd, prec)
            for f in (0, 131, 255):
                H1 = p.estimate(yd[f:f + 1].contiguous(), prec)
                assert torch.equal(H1[0], Hb[f]), (prec, f)


def test_nonfinite_inputs_propagate():
    N, T, L, R = 63, 2, 8, 2
    y = _rand_frames(N, R, 1, 4)
    y[0, 0, 5] = np.nan
    y[0, 1, 7] = np.inf
    with _plan(N, T, L, R) as p:
        for prec in ("f32", "f32s", "bf16"):
            H = host(p.estimate(dev(y), prec))
            assert np.all(np.isnan(H[0, 0].real))
            assert np.all(~np.isfinite(H[0, 1].real))
            assert np.all(np.isfinite(H[0, 1].imag))


@pytest.mark.parametrize("d", [13, 14, 15, 16])
def test_longest_sequences(d):
    """The largest sequence lengths (bit streams up to 16 KiB of LDS): every
    precision of the correlator, the adjoint, packed codes and LS rows."""
    N = (1 << d) - 1
    T, L, R, B = 3, 40, 5, 2
    K = T * L
    y = _rand_frames(N, R, B, d)
    G = synth.gaussian((B, R, K), d + 1).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        yd = dev(y)
        H = {prec: host(p.estimate(yd, prec)) for prec in ("f32", "f32s", "bf16", "f64acc")}
        X = host(p.estimate_ls(yd, "f32s"))
        A = host(p.adjoint(dev(G), "f32s"))
        q, sc = p.pack(yd, "e4m3")
        He = host(p.estimate_packed(q, sc, "e4m3"))
        qh, sch = host(q), host(sc)
    ref = oracle.correlate(y, s, K)
    tol = tol_sum(TOL32, N)
    for prec in ("f32", "f32s"):
        assert perr(H[prec], ref) <= tol, prec
    assert perr(H["f64acc"], ref) <= TOL_F64ACC
    assert perr(H["bf16"], oracle.correlate(bf16_round(y), s, K)) <= tol
    assert perr(X, oracle.ls_closed_form(ref, N)) <= tol
    assert perr(A, oracle.adjoint(G, s)) <= TOL32
    xe = oracle.dequantize(qh.view(np.uint8), sch, "e4m3", N)
    assert perr(He, oracle.correlate(xe, s, K)) <= tol


def test_longest_sequence_with_lag_alias():
    """d = 16 with T*L > N: the lags wrap mod N; the adjoint reduces over more
    lags than the sequence is long."""
    N, T, L, R, B = 65535, 1, 65600, 1, 1
    y = _rand_frames(N, R, B, 77)
    G = synth.gaussian((B, R, T * L), 78).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        assert p.lag_alias
        s = p.sequence()
        H = host(p.estimate(dev(y), "f32s"))
        A = host(p.adjoint(dev(G), "f32s"))
    assert np.array_equal(H[..., N:], H[..., :T * L - N])
    assert perr(H[..., :4096], oracle.correlate(y, s, 4096)) <= tol_sum(TOL32, N)
    assert perr(A, oracle.adjoint(G, s)) <= tol_sum(TOL32, T * L)


def test_most_antennas():
    """R = 65535 (the largest plan): 2048 antenna blocks, the last ragged."""
    N, T, L, R, B = 7, 1, 3, 65535, 1
    y = _rand_frames(N, R, B, 79)
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        H = {prec: host(p.estimate(dev(y), prec)) for prec in ("f32s", "bf16")}
    assert perr(H["f32s"], oracle.correlate(y, s, T * L)) <= TOL32
    assert perr(H["bf16"], oracle.correlate(bf16_round(y), s, T * L)) <= TOL32


def test_graph_replays_match_eager():
    """Correlator, LS rows, quantiser + packed e4m3 estimate, adjoint,
    refinement and the separate de-bias captured in one HIP graph. Every replay, with eager work and
    synchronisations between replays, equals the eager results bit for bit
    (the quantiser clears its counters with a kernel, not a memset)."""
    N, T, L, R, B = 1023, 16, 32, 64, 4
    y = dev(_rand_frames(N, R, B, 90))
    with _plan(N, T, L, R) as p:
        H_e = p.estimate(y, "bf16")
        X_e = p.estimate_ls(y, "f32s")
        q_e, sc_e = p.pack(y, "e4m3")
        Hq_e = p.estimate_packed(q_e, sc_e, "e4m3")
        A_e = p.adjoint(H_e, "f32s")
        W = torch.empty_like(y)
        Xr_e = p.refine(y, p.estimate(y, "f32s"), 3, work=W)
        D_e = p.debias(p.estimate(y, "bf16"))
        torch.cuda.synchronize()
        H, X, Hq = torch.empty_like(H_e), torch.empty_like(X_e), torch.empty_like(Hq_e)
        q, sc, A = torch.empty_like(q_e), torch.empty_like(sc_e), torch.empty_like(A_e)
        Xr, D = torch.empty_like(Xr_e), torch.empty_like(D_e)

        def work():
            p.estimate(y, "bf16", out=H)
            p.estimate_ls(y, "f32s", out=X)
            p.pack(y, "e4m3", out=q, scales=sc)
            p.estimate_packed(q, sc, "e4m3", out=Hq)
            p.adjoint(H, "f32s", out=A)
            p.estimate(y, "f32s", out=Xr)
            p.refine(y, Xr, 3, work=W)
            p.estimate(y, "bf16", out=D)
            p.debias(D)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            work()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            work()
        for _ in range(3):
            for t in (H, X, Hq, A, sc, Xr, D, W):
                t.zero_()
            q.fill_(0x7F)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(H, H_e) and torch.equal(X, X_e) and torch.equal(A, A_e)
            assert torch.equal(q, q_e) and torch.equal(sc, sc_e) and torch.equal(Hq, Hq_e)
            assert torch.equal(Xr, Xr_e) and torch.equal(D, D_e)
        del g


def _random_cases(n, seed):
    """Seeded random shapes: degree 2..12, any T and L with T*L <= 4N, R up to
    100, 1..3 frames, adjacent or Eq. 8 lags (when T*L <= N), the built-in or
    another primitive polynomial (d <= 10); oracle work kept under 4e7."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        d = int(rng.integers(2, 13))
        N = (1 << d) - 1
        T = int(rng.integers(1, 9))
        L = int(rng.integers(1, max(2, (4 * N) // T) + 1))
        R = int(rng.integers(1, 101))
        B = int(rng.integers(1, 4))
        if T * L > 4 * N or B * R * N * T * L > 4e7:
            continue
        spacing = "eq8" if T * L <= N and rng.random() < 0.5 else "adjacent"
        fb = 0
        if d <= 10 and rng.random() < 0.5:
            masks = oracle.primitive_masks(d)
            fb = int(masks[int(rng.integers(len(masks)))])
        out.append((N, T, L, R, B, spacing, fb))
    return out


@pytest.mark.parametrize("case", _random_cases(40, 2026),
                         ids=lambda c: "N%d_T%d_L%d_R%d_B%d_%s_fb%x" % c)
def test_random_shapes(case):
    N, T, L, R, B, spacing, fb = case
    K = T * L
    y = _rand_frames(N, R, B, N + K + R)
    G = synth.gaussian((B, R, K), K + 7).astype(np.complex64)
    from paper_2206_05506_amd import Plan
    with Plan(N, T, L, R, feedback=fb, spacing=spacing) as p:
        s, lag = p.sequence(), p.lags()
        yd = dev(y)
        Hb = host(p.estimate(yd, "bf16"))
        Hs = host(p.estimate(yd, "f32s"))
        A = host(p.adjoint(dev(G), "f32s"))
        X = host(p.estimate_ls(yd, "f32s")) if K <= N else None
    if fb:
        assert np.array_equal(s, oracle.mseq_mask(oracle.degree_of(N), fb))
    assert np.array_equal(lag, oracle.lags(N, T, L, "eq8" if spacing == "eq8" else "contiguous"))
    ref = oracle.correlate(y, s, K, lag)
    assert perr(Hs, ref) <= TOL32
    assert perr(Hb, oracle.correlate(bf16_round(y), s, K, lag)) <= TOL32
    assert perr(A, oracle.adjoint(G, s, lag)) <= TOL32
    if X is not None:
        assert perr(X, oracle.ls_closed_form(ref, N)) <= TOL32


def test_one_plan_on_two_streams_concurrently():
    """A plan is immutable: estimates and adjoints enqueued on two streams at
    once, interleaved, give the same bits as the same calls one at a time."""
    N, T, L, R, B = 1023, 16, 32, 64, 8
    ya = dev(_rand_frames(N, R, B, 91))
    yb = dev(_rand_frames(N, R, B, 92))
    with _plan(N, T, L, R) as p:
        ref_a, ref_b = p.estimate(ya, "bf16"), p.estimate(yb, "f32s")
        ref_aa = p.adjoint(ref_a, "f32s")
        torch.cuda.synchronize()
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        sa.wait_stream(torch.cuda.current_stream())
        sb.wait_stream(torch.cuda.current_stream())
        outs = []
        for _ in range(4):
            with torch.cuda.stream(sa):
                Ha = p.estimate(ya, "bf16")
                Aa = p.adjoint(Ha, "f32s")
            with torch.cuda.stream(sb):
                Hb = p.estimate(yb, "f32s")
            outs.append((Ha, Aa, Hb))
        torch.cuda.synchronize()
        for Ha, Aa, Hb in outs:
            assert torch.equal(Ha, ref_a) and torch.equal(Hb, ref_b) and torch.equal(Aa, ref_aa)


def test_lazy_conjugate_views_are_refused():
    """torch's conj() only flips a flag; the library reads memory, so such a
    view must be resolved first (refused, not silently mis-read)."""
    N, T, L, R = 127, 4, 16, 4
    y = dev(_rand_frames(N, R, 1, 93))
    with _plan(N, T, L, R) as p:
        with pytest.raises(ValueError):
            p.estimate(y.conj(), "f32s")
        H = host(p.estimate(y.conj().resolve_conj(), "f32s"))
        ref = oracle.correlate(np.conj(host(y)), p.sequence(), T * L)
    assert perr(H, ref) <= TOL32


def test_empty_batch_is_a_no_op():
    """batch == 0 through the C ABI: every batch entry point returns PNCE_OK
    with NULL tensor pointers and enqueues nothing, while its other scalar
    arguments are still checked; the Python wrappers return empty outputs."""
    from paper_2206_05506_amd import _lib
    lib = _lib.lib
    N, T, L, R = 127, 4, 16, 4
    with _plan(N, T, L, R) as p:
        h = p.handle
        assert lib.pnce_estimate(h, None, None, None, 0, 1, 1.0 / N, None, 0.0) == 0
        assert lib.pnce_estimate_ls(h, None, None, None, 0, 1, None) == 0
        assert lib.pnce_debias(h, None, None, 0) == 0
        assert lib.pnce_pack(h, None, None, None, None, 0, 1) == 0
        assert lib.pnce_estimate_packed(h, None, None, None, None, 0, 1, 0.0) == 0
        assert lib.pnce_adjoint(h, None, None, None, None, 0, 1, 1.0 / N, 0.0) == 0
        assert lib.pnce_refine(h, None, None, None, None, 0, 3) == 0
        assert lib.pnce_estimate_cp(h, None, None, 8, None, 0, 1, None) == 0
        assert lib.pnce_pack_cp(h, None, None, 8, None, None, 0, 1) == 0
        # the scalar arguments are checked before the early return
        assert lib.pnce_estimate(h, None, None, None, 0, 99, 1.0, None, 0.0) == -1
        assert lib.pnce_pack(h, None, None, None, None, 0, 99) == -1
        assert lib.pnce_refine(h, None, None, None, None, 0, -1) == -1
        assert lib.pnce_estimate_cp(h, None, None, -1, None, 0, 1, None) == -1
        assert lib.pnce_estimate(h, None, None, None, -1, 1, 1.0, None, 0.0) == -1
        y = torch.empty((0, R, N), dtype=torch.complex64, device="cuda")
        assert p.estimate(y, "bf16").shape == (0, R, T * L)
        q, sc = p.pack(y, "e4m3")
        assert q.shape == (0, R, 2, N + 1) and sc.shape == (0,)
        assert p.estimate_packed(q, sc, "e4m3").shape == (0, R, T * L)
        X = p.estimate_ls(y, "f32s")
        assert p.refine(y, X, 2).shape == (0, R, T * L)
        assert p.adjoint(X).shape == (0, R, N)
        torch.cuda.synchronize()


def test_refine_checks_the_callers_workspace():
    """A workspace of the wrong shape is refused before any launch (a short
    one would otherwise be written past its end)."""
    N, T, L, R = 127, 4, 16, 4
    y = dev(_rand_frames(N, R, 2, 94))
    with _plan(N, T, L, R) as p:
        X = p.estimate(y, "f32s")
        with pytest.raises(ValueError):
            p.refine(y, X, 1, work=torch.empty((1, R, N), dtype=torch.complex64, device="cuda"))
        with pytest.raises(ValueError):
            p.refine(y, X, 1, work=torch.empty((2, R, N), dtype=torch.complex128, device="cuda"))
        p.refine(y, X, 1, work=torch.empty((2, R, N), dtype=torch.complex64, device="cuda"))
        torch.cuda.synchronize()


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("N,R,cp", [(127, 5, 0), (1023, 33, 0), (63, 3, 7), (3, 1, 0)])
def test_pack_one_launch_path_bit_exact(fmt, N, R, cp):
    """Batches of 256 frames or more are quantised by one launch with a
    workgroup per frame. Its codes and scales equal the oracle's bit for
    bit, including degenerate frames (all zero, +-inf, NaN, a maximum on a
    power of two, subnormal-size values) and raw rows with a cyclic prefix,
    and equal those of the slice path (255 frames) and of the two-pass path."""
    from paper_2206_05506_amd.api import _CODE_DTYPE
    B = 256
    rng = np.random.default_rng(N + R + cp)
    y = (rng.standard_normal((B, R, N)) + 1j * rng.standard_normal((B, R, N))).astype(np.complex64)
    y *= (10.0 ** rng.uniform(-6, 6, size=(B, 1, 1))).astype(np.float32)
    y[0] = 0.0
    y[1, 0, N - 1] = np.inf
    y[2, R - 1, 0] = np.nan + 1j
    y[3] *= np.float32(0.49) / max(np.abs(y[3].real).max(), np.abs(y[3].imag).max())
    y[3, 0, 0] = 0.5
    y[4] = np.float32(1e-39)
    raw = np.concatenate([y[:, :, N - cp:], y], axis=2) if cp else y
    with _plan(N, 1, 1, R) as p:
        yd = dev(raw)
        work = torch.full((1024 * B + 1,), 5, dtype=torch.int32, device="cuda")
        q, sc = p.pack_cp(yd, cp, fmt, work=work)
        assert int(host(work)[1024 * B]) == 0   # written by every launch plan
        part = yd[:B - 1].contiguous()
        q4, sc4 = (p.pack_cp(part, cp, fmt) if cp else p.pack(part, fmt))
        q2, sc2 = p.pack_cp_two_pass(yd, cp, fmt)
        q, sc, q4, sc4, q2, sc2 = (host(q), host(sc), host(q4), host(sc4), host(q2),
                                   host(sc2))
    ref_q, ref_sc = oracle.quantize(y, fmt)
    assert q.dtype == np.dtype(str(_CODE_DTYPE[fmt]).replace("torch.", ""))
    assert np.array_equal(sc, ref_sc)
    assert np.array_equal(q.view(ref_q.dtype), ref_q)
    assert np.array_equal(sc4, sc[:B - 1]) and np.array_equal(q4, q[:B - 1])
    assert np.array_equal(sc2, sc) and np.array_equal(q2, q)


def _special_frames(y):
    """Degenerate frames in place (as many as the batch holds): a maximum on
    a power of two, all zero, +-inf and NaN, subnormal-size values."""
    B, R, N = y.shape
    if B > 1:
        y[1] *= np.float32(0.49) / max(np.abs(y[1].real).max(), np.abs(y[1].imag).max())
        y[1, R - 1, N - 1] = 0.5
    if B > 2:
        y[2] = 0.0
    if B > 3:
        y[3, 0, N - 1] = np.inf
        y[3, R - 1, 0] = np.nan + 1j
    if B > 4:
        y[4] = np.float32(1e-39)
    return y


@pytest.mark.parametrize("fmt", ["bf16", "f16", "e4m3"])
@pytest.mark.parametrize("N,R,B,cp", [(4095, 40, 3, 0), (2047, 37, 5, 17), (7, 3, 2, 0),
                                      (65535, 3, 2, 5), (1023, 300, 4, 0), (255, 2, 5, 3)])
def test_pack_single_read_path_bit_exact(fmt, N, R, B, cp):
    """The quantiser with a workspace (pnce_pack_ws) on batches the
    one-launch path does not take: each frame is cut into slices of 8192
    samples held in registers while the frame maximum is gathered (full,
    ragged and single slices). Codes and scales equal the oracle's bit for
    bit, degenerate frames included, and equal the two-pass path's; the
    workspace's wait flag stays zero."""
    from paper_2206_05506_amd import _lib
    rng = np.random.default_rng(N + R + B + cp)
    y = (rng.standard_normal((B, R, N)) + 1j * rng.standard_normal((B, R, N))).astype(np.complex64)
    y *= (10.0 ** rng.uniform(-4, 4, size=(B, 1, 1))).astype(np.float32)
    y = _special_frames(y)
    raw = np.concatenate([y[:, :, N - cp:], y], axis=2) if cp else y
    print(f"pack_ws fmt={fmt} N={N} R={R} B={B} cp={cp}", flush=True)
    with _plan(N, 1, 1, R) as p:
        yd = dev(raw)
        work = torch.full(((_lib.pack_work_bytes(B) + 3) // 4,), -1, dtype=torch.int32,
                          device="cuda")
        q, sc = p.pack_cp(yd, cp, fmt, work=work)
        q2, sc2 = p.pack_cp_two_pass(yd, cp, fmt)
        q, sc, q2, sc2 = host(q), host(sc), host(q2), host(sc2)
        flag = int(host(work)[1024 * B])
    ref_q, ref_sc = oracle.quantize(y, fmt)
    assert flag == 0
    assert np.array_equal(sc, ref_sc)
    assert np.array_equal(q.view(ref_q.dtype), ref_q)
    assert np.array_equal(sc2, sc) and np.array_equal(q2, q)


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_pack_single_read_path_precision_frames(fmt):
    """Eight frames of the precision workload's shape (256 x 4095, 8.4 MB:
    128 slices each): the single-read codes equal the two-pass codes bit for
    bit, and the oracle's on the first frame."""
    N, R, B = 4095, 256, 8
    g = torch.Generator(device="cuda")
    g.manual_seed(41)
    with _plan(N, 32, 64, R) as p:
        y = torch.complex(torch.randn((B, R, N), generator=g, device="cuda"),
                          torch.randn((B, R, N), generator=g, device="cuda")).contiguous()
        y[3] *= 1e-5
        q, sc = p.pack(y, fmt)
        q2, sc2 = p.pack_two_pass(y, fmt)
        assert torch.equal(sc, sc2) and torch.equal(q, q2)
        y0, q0, s0 = host(y[:1]), host(q[:1]), host(sc[:1])
    ref_q, ref_sc = oracle.quantize(y0, fmt)
    assert np.array_equal(s0, ref_sc)
    assert np.array_equal(q0.view(ref_q.dtype), ref_q)


def test_pack_frames_too_large_for_slices_fall_back():
    """A frame of 2048 x 4095 samples (67 MB, 512 slices: more than half of
    what the chip holds at once) cannot be gathered in registers; the call
    with a workspace then takes the two-pass path and still writes the
    oracle's codes and scale."""
    from paper_2206_05506_amd import _lib
    N, R, B = 4095, 2048, 1
    g = torch.Generator(device="cuda")
    g.manual_seed(43)
    with _plan(N, 1, 1, R) as p:
        y = torch.complex(torch.randn((B, R, N), generator=g, device="cuda"),
                          torch.randn((B, R, N), generator=g, device="cuda")).contiguous()
        y *= 3.0e-3
        work = torch.full(((_lib.pack_work_bytes(B) + 3) // 4,), 7, dtype=torch.int32,
                          device="cuda")
        q, sc = p.pack(y, "bf16", work=work)
        yh, qh, sh = host(y), host(q), host(sc)
        flag = int(host(work)[1024 * B])
    assert flag == 0   # written by every launch plan
    ref_q, ref_sc = oracle.quantize(yh, "bf16")
    assert np.array_equal(sh, ref_sc)
    assert np.array_equal(qh.view(ref_q.dtype), ref_q)


def test_pack_workspace_path_under_graph_capture():
    """pnce_pack_ws (slices gathered through the workspace, cleared by a fill
    kernel, no memset) captured in a HIP graph and replayed three times on new
    frames, with eager work between the replays: every replay's codes and
    scales equal the eager call's."""
    N, T, L, R, B = 4095, 32, 64, 40, 3
    g = torch.Generator(device="cuda")
    g.manual_seed(47)

    def frames(k):
        return (torch.complex(torch.randn((B, R, N), generator=g, device="cuda"),
                              torch.randn((B, R, N), generator=g, device="cuda"))
                * (10.0 ** (k - 1))).contiguous()

    with _plan(N, T, L, R) as p:
        y = frames(0)
        q, sc = p.pack(y, "bf16")
        work = torch.empty((1024 * B + 1,), dtype=torch.int32, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            p.pack(y, "bf16", out=q, scales=sc, work=work)
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            p.pack(y, "bf16", out=q, scales=sc, work=work)
        for k in range(3):
            y.copy_(frames(k))
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            q2, sc2 = p.pack_two_pass(y, "bf16")
            torch.cuda.synchronize()
            assert torch.equal(q, q2) and torch.equal(sc, sc2), k
            assert int(host(work)[1024 * B]) == 0
        del graph


def test_pack_workspace_path_random_shapes():
    """120 seeded (N, R, batch, cyclic prefix, format) cases through the
    quantiser with a workspace, spread over its three launch plans (slices
    for most, one workgroup per frame and two passes for some): codes and
    scales bit-exact against the two-pass path, the wait flag 0, and one
    frame per case bit-exact against the oracle."""
    import random
    from paper_2206_05506_amd import _lib
    rnd = random.Random(2206)
    g = torch.Generator(device="cuda")
    g.manual_seed(2206)
    for case in range(120):
        d = rnd.choice([2, 3, 5, 7, 8, 9, 10, 11, 12, 13])
        N = (1 << d) - 1
        R = rnd.choice([1, 2, 3, 31, 32, 33, 64, 100, 255])
        B = rnd.choice([1, 2, 3, 5, 17])
        if rnd.random() < 0.05:
            B, R, N = 256, 4, 127             # the one-workgroup-per-frame plan
        cp = rnd.choice([0, 0, 1, 7, 32])
        fmt = rnd.choice(["bf16", "f16", "e4m3"])
        scale = 10.0 ** rnd.uniform(-8, 8)
        raw = (torch.complex(torch.randn((B, R, cp + N), generator=g, device="cuda"),
                             torch.randn((B, R, cp + N), generator=g, device="cuda"))
               * scale).contiguous()
        with _plan(N, 1, 1, R) as p:
            work = torch.full(((_lib.pack_work_bytes(B) + 3) // 4,), -1, dtype=torch.int32,
                              device="cuda")
            q, sc = p.pack_cp(raw, cp, fmt, work=work)
            q2, sc2 = p.pack_cp_two_pass(raw, cp, fmt)
            torch.cuda.synchronize()
            where = (case, N, R, B, cp, fmt)
            assert torch.equal(sc, sc2) and torch.equal(q, q2), where
            assert int(host(work)[1024 * B]) == 0, where
            f = rnd.randrange(B)
            y = host(raw[f:f + 1, :, cp:].contiguous())
            qh, sh = host(q[f:f + 1]), host(sc[f:f + 1])
        ref_q, ref_sc = oracle.quantize(y, fmt)
        assert np.array_equal(sh, ref_sc), where
        assert np.array_equal(qh.view(ref_q.dtype), ref_q), where


def test_pack_workspace_is_checked():
    """pnce_pack_ws refuses a missing, misaligned or short workspace before
    anything is enqueued."""
    from paper_2206_05506_amd import _lib
    lib = _lib.lib
    N, R, B = 127, 3, 4
    with _plan(N, 1, 1, R) as p:
        y = dev(_rand_frames(N, R, B, 77))
        q = torch.zeros((B, R, 2, N + 1), dtype=torch.int16, device="cuda")
        sc = torch.zeros((B,), dtype=torch.float32, device="cuda")
        w = torch.zeros((1024 * B + 2,), dtype=torch.int32, device="cuda")
        need = _lib.pack_work_bytes(B)
        args = (p.handle, None, y.data_ptr(), 0, q.data_ptr(), sc.data_ptr(), B, 1)
        assert lib.pnce_pack_ws(*args, None, need) == -1
        assert lib.pnce_pack_ws(*args, w.data_ptr(), need - 1) == -1
        assert lib.pnce_pack_ws(*args, w.data_ptr() + 2, need) == -1
        torch.cuda.synchronize()
        assert not q.any() and not sc.any()
        with pytest.raises(ValueError):
            p.pack(y, "bf16", work=torch.zeros((1024 * B,), dtype=torch.int32, device="cuda"))
        assert lib.pnce_pack_ws(*args, w.data_ptr(), need) == 0
        torch.cuda.synchronize()
        assert sc.all()


def test_misaligned_pointers_are_refused():
    """Every tensor pointer must be aligned to its element; a misaligned one
    returns PNCE_E_INVALID and nothing is written."""
    from paper_2206_05506_amd import _lib
    lib = _lib.lib
    N, T, L, R, B = 127, 4, 16, 4, 2
    K = T * L
    with _plan(N, T, L, R) as p:
        h = p.handle
        y = dev(_rand_frames(N, R, B, 95))
        H = torch.zeros((B, R, K), dtype=torch.complex64, device="cuda")
        q, sc = p.pack(y, "bf16")
        q8, sc8 = p.pack(y, "e4m3")
        A = torch.zeros_like(y)
        W = torch.empty_like(y)
        yp, Hp, qp, sp = y.data_ptr(), H.data_ptr(), q.data_ptr(), sc.data_ptr()
        torch.cuda.synchronize()
        assert lib.pnce_estimate(h, None, yp + 4, Hp, B, 1, 1.0 / N, None, 0.0) == -1
        assert lib.pnce_estimate(h, None, yp, Hp + 4, B, 1, 1.0 / N, None, 0.0) == -1
        assert lib.pnce_estimate(h, None, yp, Hp, B, 1, 1.0 / N, sp + 2, 0.0) == -1
        assert b"aligned" in lib.pnce_last_error()
        assert lib.pnce_estimate_packed(h, None, qp + 4, sp, Hp, B, 1, 0.0) == -1
        assert lib.pnce_estimate_packed(h, None, q8.data_ptr() + 2, sc8.data_ptr(), Hp, B, 3,
                                        0.0) == -1
        assert lib.pnce_pack(h, None, yp, qp + 2, sp, B, 1) == -1
        assert lib.pnce_adjoint(h, None, Hp + 4, A.data_ptr(), None, B, 1, 1.0 / N, 0.0) == -1
        assert lib.pnce_refine(h, None, yp, Hp, W.data_ptr() + 4, B, 1) == -1
        assert lib.pnce_debias(h, None, Hp + 4, B) == -1
        assert lib.pnce_estimate_ls(h, None, yp + 4, Hp, B, 1, None) == -1
        assert lib.pnce_estimate_cp(h, None, yp + 4, 0, Hp, B, 1, None) == -1
        assert lib.pnce_pack_cp(h, None, yp, 0, qp, sp + 1, B, 1) == -1
        # e4m3 codes need only 4-byte alignment: a 4-byte offset is accepted
        # (the buffer has 4 spare bytes, so the shifted codes stay inside it)
        q8s = torch.empty((B * R * 2 * (N + 1) + 4,), dtype=torch.uint8, device="cuda")
        assert lib.pnce_pack(h, None, yp, q8s.data_ptr() + 4, sc8.data_ptr(), B, 3) == 0
        torch.cuda.synchronize()
        assert not H.abs().any() and not A.abs().any()


def test_entry_point_statuses_follow_the_documented_checks():
    """Seeded calls of the batch entry points with valid and invalid scalar
    arguments and NULL buffers: every status follows the documented order
    (plan, scalar arguments, empty batch, pointers, batch sign); accepted
    calls run on correctly sized buffers and return PNCE_OK."""
    import random
    from paper_2206_05506_amd import _lib
    lib = _lib.lib
    N, T, L, R, BMAX, CP = 31, 2, 4, 3, 3, 5
    K = T * L
    rnd = random.Random(5)
    with _plan(N, T, L, R) as p:
        h = p.handle
        y = dev(_rand_frames(N, R, BMAX, 96))
        raw = dev(_rand_frames(N + CP, R, BMAX, 97))
        H = torch.empty((BMAX, R, K), dtype=torch.complex64, device="cuda")
        A = torch.empty_like(y)
        C = torch.zeros_like(y)
        W = torch.empty_like(y)
        q = torch.empty((BMAX, R, 2, N + 1), dtype=torch.int16, device="cuda")
        sc = torch.empty((BMAX,), dtype=torch.float32, device="cuda")
        ptr = {"y": y.data_ptr(), "raw": raw.data_ptr(), "H": H.data_ptr(), "A": A.data_ptr(),
               "C": C.data_ptr(), "W": W.data_ptr(), "q": q.data_ptr(), "sc": sc.data_ptr()}

        def maybe(name):  # a buffer, or now and then NULL
            return None if rnd.random() < 0.15 else ptr[name]

        n_ok = n_err = 0
        for _ in range(300):
            batch = rnd.choice([0, 1, 2, 3, -1])
            op = rnd.choice(["estimate", "pack", "estimate_cp", "refine", "adjoint"])
            if op == "estimate":
                prec = rnd.choice([0, 1, 2, 4, 5, 6, 9, -1])
                a, b = maybe("y"), maybe("H")
                want = (-1 if prec not in (0, 1, 2, 4, 5, 6) else 0 if batch == 0 else
                        -1 if a is None or b is None or batch < 0 else 0)
                st = lib.pnce_estimate(h, None, a, b, batch, prec, 1.0 / N, None, 0.0)
            elif op == "pack":
                fmt = rnd.choice([1, 2, 0, 4])
                a, b, c = maybe("y"), maybe("q"), maybe("sc")
                want = (-1 if fmt not in (1, 2) else 0 if batch == 0 else
                        -1 if None in (a, b, c) or batch < 0 else 0)
                st = lib.pnce_pack(h, None, a, b, c, batch, fmt)
            elif op == "estimate_cp":
                prec = rnd.choice([1, 2, 7])
                cp = rnd.choice([CP, -1, 1 << 26])
                a, b = maybe("raw"), maybe("H")
                want = (-1 if prec == 7 or cp < 0 else -2 if cp == 1 << 26 else
                        0 if batch == 0 else -1 if a is None or b is None or batch < 0 else 0)
                st = lib.pnce_estimate_cp(h, None, a, cp, b, batch, prec, None)
            elif op == "refine":
                steps = rnd.choice([0, 1, 2, -1])
                a, b, c = maybe("y"), maybe("H"), maybe("W")
                want = (-1 if steps < 0 else 0 if batch == 0 else
                        -1 if a is None or b is None or (c is None and steps > 0) or batch < 0
                        else 0)
                st = lib.pnce_refine(h, None, a, b, c, batch, steps)
            else:
                prec = rnd.choice([1, 2, 5, 6, 8])
                beta = rnd.choice([0.0, 1.0])
                a, b, c = maybe("H"), maybe("A"), maybe("C")
                want = (-1 if prec == 8 else 0 if batch == 0 else
                        -1 if a is None or b is None or (beta != 0.0 and c is None) or batch < 0
                        else 0)
                st = lib.pnce_adjoint(h, None, a, b, c, batch, prec, 1.0 / N, beta)
            assert st == want, (op, batch, st, want)
            n_ok += st == 0
            n_err += st < 0
        torch.cuda.synchronize()
    assert n_ok > 50 and n_err > 50

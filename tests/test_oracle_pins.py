"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here re-types an oracle formula: each check reaches the same result
by another road (Eq. 1's autocorrelation, closed forms that follow from it,
numpy's FFT, scipy's circulant and lstsq, dense brute force, finite
differences, torch's own float conversions).
"""
import numpy as np
import pytest
import scipy.linalg
import torch

import oracle
import synth


def dense_P(s, K):
    """Explicit N x K matrix whose column k is the sequence delayed by k."""
    return np.stack([np.roll(np.asarray(s, np.float64), k) for k in range(K)], axis=1)


def rand_c(shape, seed):
    return synth.gaussian(shape, seed)


# ---------------------------------------------------------------- a1: sequence
@pytest.mark.parametrize("d", list(range(2, 17)))
def test_mseq_balance_and_two_level_autocorrelation(d):
    """Eq. 1: circular autocorrelation N at lag 0 and -1 at every other lag
    (equivalently R[n] = 1 and -1/M after the 1/M normalisation)."""
    s = oracle.mseq(d).astype(np.float64)
    N = (1 << d) - 1
    assert s.shape == (N,)
    assert set(np.unique(s)) <= {-1.0, 1.0}
    assert np.sum(s == -1) == (N + 1) // 2            # (N+1)/2 ones
    ac = np.real(np.fft.ifft(np.abs(np.fft.fft(s)) ** 2))
    assert abs(ac[0] - N) < 1e-6
    assert np.max(np.abs(ac[1:] + 1.0)) < 1e-6
    R = ac / N
    assert abs(R[0] - 1.0) < 1e-9 and np.allclose(R[1:], -1.0 / N, atol=1e-9)


@pytest.mark.parametrize("d", [5, 7])
def test_mseq_autocorrelation_direct(d):
    """Eq. 1 again, by the direct sum over np.roll (no FFT)."""
    s = oracle.mseq(d).astype(np.int64)
    N = s.size
    for n in range(N):
        c = int(np.sum(s * np.roll(s, -n)))
        assert c == (N if n == 0 else -1)


def test_mseq_rejects_bad_degree():
    with pytest.raises(ValueError):
        oracle.mseq(1)
    with pytest.raises(ValueError):
        oracle.mseq(17)


# -------------------------------------------------------- a4: the correlator
@pytest.mark.parametrize("d,K", [(5, 8), (5, 31), (5, 40), (7, 64)])
def test_correlate_equals_dense_brute_force(d, K):
    s = oracle.mseq(d)
    N = s.size
    Y = rand_c((2, 3, N), seed=d * 100 + K)
    H = oracle.correlate(Y, s, K)
    ref = Y @ dense_P(s, K) / N
    assert np.max(np.abs(H - ref)) < 1e-13


@pytest.mark.parametrize("d,K", [(7, 64), (10, 512), (10, 1024), (12, 2048)])
def test_correlate_equals_fft_cross_correlation(d, K):
    """Textbook circular cross-correlation through the DFT."""
    s = oracle.mseq(d)
    N = s.size
    Y = rand_c((1, 2, N), seed=d + K)
    H = oracle.correlate(Y, s, K)
    c = np.fft.ifft(np.fft.fft(Y, axis=-1) * np.conj(np.fft.fft(s.astype(np.float64))), axis=-1)
    ref = c[..., np.arange(K) % N] / N
    assert np.max(np.abs(H - ref)) < 1e-12


def test_sequential_case_is_full_circulant():
    """T = 1, L = N: H = S^T y / N with S the circulant of Eq. 2 (first row
    s0, s_{M-1}, ..., s1), built by scipy."""
    s = oracle.mseq(6)
    N = s.size
    S = scipy.linalg.circulant(s.astype(np.float64))
    assert np.array_equal(S[0], np.concatenate([[s[0]], s[:0:-1]]))
    y = rand_c((1, 1, N), seed=7)
    H = oracle.correlate(y, s, N)
    ref = (S.T @ y[0, 0]) / N
    assert np.max(np.abs(H[0, 0] - ref)) < 1e-13


@pytest.mark.parametrize("d,T,L", [(7, 4, 16), (10, 16, 32), (5, 2, 4), (6, 1, 63)])
def test_noiseless_bias_closed_form(d, T, L):
    """From Eq. 1, P^T P = (N+1) I - J, so a noiseless frame gives
    h_hat = h + (h - sum(h)) / N (the -sum(h)/N bias, sum over the K lags)."""
    s = oracle.mseq(d)
    N = s.size
    h = rand_c((2, 3, T, L), seed=d * T * L)
    y, _ = oracle.received(s, h, np.zeros((2, 3, N)), np.full(2, 300.0))
    H = oracle.correlate(y, s, T * L)
    hs = h.reshape(2, 3, T * L)
    expect = hs + (hs - hs.sum(axis=-1, keepdims=True)) / N
    assert np.max(np.abs(H - expect)) < 1e-12


def test_noiseless_least_squares_recovers_channel():
    s = oracle.mseq(7)
    N = s.size
    h = rand_c((1, 4, 4, 16), seed=3)
    y, _ = oracle.received(s, h, np.zeros((1, 4, N)), np.array([400.0]))
    H = oracle.correlate(y, s, 64)
    x = oracle.ls_closed_form(H, N)
    assert np.max(np.abs(x - h.reshape(1, 4, 64))) < 1e-12


def test_demultiplex_view():
    """Eq. 10: transmitter t's CIR estimate is H[..., t*L:(t+1)*L]."""
    s = oracle.mseq(8)
    N = s.size
    T, L = 4, 16
    h = np.zeros((1, 1, T, L), dtype=np.complex128)
    h[0, 0, 2, 5] = 1.0
    y, _ = oracle.received(s, h, np.zeros((1, 1, N)), np.array([300.0]))
    H = oracle.correlate(y, s, T * L).reshape(1, 1, T, L)
    assert np.argmax(np.abs(H[0, 0]).ravel()) == 2 * L + 5
    assert abs(H[0, 0, 2, 5] - 1.0) < 1e-12        # the tap itself
    others = np.delete(H[0, 0].ravel(), 2 * L + 5)
    assert np.max(np.abs(others + 1.0 / N)) < 1e-12  # -1/M floor of Eq. 1


def test_linearity_and_shift_equivariance():
    s = oracle.mseq(7)
    N = s.size
    K = 40
    a = rand_c((1, 2, N), 1)
    b = rand_c((1, 2, N), 2)
    Ha, Hb = oracle.correlate(a, s, K), oracle.correlate(b, s, K)
    H = oracle.correlate(2.5 * a - 1j * b, s, K)
    assert np.max(np.abs(H - (2.5 * Ha - 1j * Hb))) < 1e-12
    Hs = oracle.correlate(np.roll(a, 1, axis=-1), s, K)
    assert np.max(np.abs(Hs[..., 1:] - Ha[..., :-1])) < 1e-12


def test_lag_alias_when_T_L_exceeds_N():
    """Lags are taken mod N: with T*L > N column k + N repeats column k."""
    s = oracle.mseq(5)
    N = s.size
    Y = rand_c((1, 2, N), 9)
    H = oracle.correlate(Y, s, N + 9)
    assert np.max(np.abs(H[..., N:] - H[..., :9])) < 1e-14


@pytest.mark.parametrize("d", [5, 7])
def test_refinement_with_an_aliased_lag_grows_along_one_direction(d):
    """K = N + 1 lags (every lag once, lag 0 twice, as in the differentiation
    workload's 16*64 > 1023): P P^T = (N+1) I - J + s s^T, whose nonzero
    eigenvalues are N+1 (multiplicity N-2) and N+1 +- sqrt(N^2 - 1) on the
    span of {1, s}. A step of 1/N therefore multiplies the residual along the
    top eigenvector by (N+1+sqrt(N^2-1))/N - 1 > 1: the iteration is slightly
    unstable there, and the oracle's refinement must show that exact rate."""
    s = oracle.mseq(d)
    N = s.size
    K = N + 1
    P = dense_P(s, K)
    w, V = np.linalg.eigh(P @ P.T)
    top = N + 1 + np.sqrt(N * N - 1.0)
    assert abs(w[-1] - top) < 1e-9 * top
    assert abs(w[0] - (N + 1 - np.sqrt(N * N - 1.0))) < 1e-9 * N
    assert np.allclose(w[1:-1], N + 1)
    y = (V[:, -1] * (0.8 - 0.6j)).reshape(1, 1, N)
    its = oracle.refine(y, s, K, 4)
    r = [np.linalg.norm(y[0, 0] - P @ x[0, 0]) for x in its]
    rate = top / N - 1
    assert rate > 1
    for j in range(4):
        assert abs(r[j + 1] / r[j] - rate) < 1e-12


# ------------------------------------------------------------ a7: adjoint
@pytest.mark.parametrize("d,K", [(5, 8), (5, 40), (7, 64)])
def test_adjoint_brute_force_and_dot_identity(d, K):
    s = oracle.mseq(d)
    N = s.size
    G = rand_c((2, 3, K), 11)
    Y = rand_c((2, 3, N), 12)
    A = oracle.adjoint(G, s)
    assert np.max(np.abs(A - G @ dense_P(s, K).T / N)) < 1e-13
    lhs = np.vdot(G, oracle.correlate(Y, s, K))      # <H(Y), G>
    rhs = np.vdot(oracle.adjoint(G, s), Y)           # <Y, A(G)>
    assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(lhs))


def test_received_model_equals_dense_product():
    """Eq. 9: the noiseless frame is P h_stack (dense), noise then scaled to
    the requested SNR."""
    s = oracle.mseq(6)
    N = s.size
    h = rand_c((2, 3, 3, 5), 4)
    w = rand_c((2, 3, N), 5)
    y, yc = oracle.received(s, h, w, np.array([10.0, 0.0]))
    ref = h.reshape(2, 3, 15) @ dense_P(s, 15).T
    assert np.max(np.abs(yc - ref)) < 1e-12
    noise_p = np.mean(np.abs(y - yc) ** 2, axis=(1, 2))
    sig_p = np.mean(np.abs(yc) ** 2, axis=(1, 2))
    wp = np.mean(np.abs(w) ** 2, axis=(1, 2))
    snr = 10 * np.log10(sig_p / (noise_p / wp))
    assert np.allclose(snr, [10.0, 0.0], atol=1e-9)


# ------------------------------------------------------- a6: refinement
def test_refinement_converges_to_lstsq():
    s = oracle.mseq(5)
    N = s.size
    K = 8
    y = rand_c((1, 2, N), 21)
    its = oracle.refine(y, s, K, 60)
    P = dense_P(s, K)
    ls = np.stack([np.linalg.lstsq(P, y[0, r], rcond=None)[0] for r in range(2)])
    assert np.max(np.abs(its[-1][0] - ls)) < 1e-12
    assert np.max(np.abs(oracle.ls_closed_form(its[0], N)[0] - ls)) < 1e-12


def test_refinement_contraction_rates():
    """Error to the LS point shrinks by (K-1)/N along the all-ones lag vector
    and by -1/N on its complement, per step."""
    s = oracle.mseq(7)
    N = s.size
    K = 64
    y = rand_c((1, 1, N), 22)
    its = oracle.refine(y, s, K, 3)
    ls = oracle.ls_closed_form(its[0], N)[0, 0]
    e = [x[0, 0] - ls for x in its]
    one = np.ones(K) / np.sqrt(K)
    for j in range(3):
        a0, a1 = np.vdot(one, e[j]), np.vdot(one, e[j + 1])
        c0, c1 = e[j] - a0 * one, e[j + 1] - a1 * one
        assert abs(a1 - (K - 1) / N * a0) < 1e-12 * max(1, abs(a0))
        assert np.max(np.abs(c1 + c0 / N)) < 1e-12


def test_loss_gradient_finite_differences():
    s = oracle.mseq(5)
    N = s.size
    K = 8
    y = rand_c((1, 2, N), 31)
    x = rand_c((1, 2, K), 32)
    loss, g = oracle.loss_grad(y, s, x)
    eps = 1e-6
    for idx in [(0, 0, 0), (0, 1, 5), (0, 0, 7)]:
        for unit, part in ((1.0, "re"), (1j, "im")):
            xp = x.copy(); xp[idx] += eps * unit
            xm = x.copy(); xm[idx] -= eps * unit
            fd = (oracle.loss_grad(y, s, xp)[0] - oracle.loss_grad(y, s, xm)[0]) / (2 * eps)
            got = g[idx].real if part == "re" else g[idx].imag
            assert abs(fd - got) < 1e-5 * max(1.0, abs(got))


# --------------------------------------------------- a3: reduced precision
def test_bf16_and_f16_codes_match_torch_rounding():
    v = rand_c((3, 4, 127), 41).astype(np.complex64) * 7.3
    for fmt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        codes, sc = oracle.quantize(v, fmt)
        planes = np.stack([v.real, v.imag], axis=2).astype(np.float32)
        t = torch.from_numpy(planes) * torch.from_numpy(1.0 / sc)[:, None, None, None]
        ref = t.to(tdt).view(torch.int16).numpy().view(np.uint16)
        assert np.array_equal(codes[..., :127], ref)
        assert np.all(codes[..., 127] == 0)


def test_e4m3_codes_and_decode_match_torch():
    allc = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(allc).view(torch.float8_e4m3fn).float().numpy().astype(np.float64)
    mine = oracle.decode(allc, "e4m3")
    fin = np.isfinite(ref)
    assert np.array_equal(np.isnan(mine), np.isnan(ref))
    assert np.array_equal(mine[fin], ref[fin])
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(-448, 448, 5000), rng.normal(0, 1, 5000),
                        rng.normal(0, 1e-2, 2000), _e4m3_midpoints()]).astype(np.float32)
    got = oracle._e4m3_bits(x)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(got, want)


def _e4m3_midpoints():
    v = oracle.decode(np.arange(127, dtype=np.uint8), "e4m3")
    mids = (v[:-1] + v[1:]) / 2
    return np.concatenate([mids, -mids])


def test_e4m3_saturates():
    x = np.array([448.0, 449.0, 480.0, 1e30, np.inf, -500.0, -np.inf], dtype=np.float32)
    c = oracle._e4m3_bits(x)
    assert list(c) == [0x7E, 0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0xFE]


@pytest.mark.parametrize("fmt", oracle.FORMATS)
def test_scale_is_smallest_power_of_two(fmt):
    y = rand_c((4, 3, 31), 51).astype(np.complex64) * np.array([1e-3, 1, 37, 5e4])[:, None, None]
    y[2, 0, 0] = 448.0 * 4 if fmt == "e4m3" else 4.0   # exact boundary
    sc = oracle.frame_scale(y, fmt)
    tgt = 448.0 if fmt == "e4m3" else 1.0
    mx = np.maximum(np.abs(y.real), np.abs(y.imag)).reshape(4, -1).max(axis=1)
    for b in range(4):
        m, e = np.frexp(sc[b])
        assert m == 0.5                       # power of two
        assert mx[b] <= tgt * sc[b] and mx[b] > tgt * sc[b] / 2
    assert oracle.frame_scale(np.zeros((1, 2, 3), np.complex64), fmt)[0] == 1.0


@pytest.mark.parametrize("fmt,tol", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11), ("e4m3", 2.0 ** -4)])
def test_subnormal_frames_get_the_smallest_normal_scale(fmt, tol):
    """A frame whose samples are all subnormal float32 values gets scale
    2^-126 (not a subnormal power of two, whose reciprocal would overflow),
    and its codes decode back to the samples within the format's rounding."""
    y = (rand_c((1, 2, 15), 53) * 1e-39).astype(np.complex64)
    assert np.abs(y.real).max() < 2.0 ** -126
    sc = oracle.frame_scale(y, fmt)
    assert sc[0] == np.float32(2.0 ** -126)
    q, sc2 = oracle.quantize(y, fmt)
    x = oracle.dequantize(q, sc2, fmt, 15)
    assert np.all(np.isfinite(x))
    err = np.abs(x - y.astype(np.complex128)).max()
    assert err <= tol * np.abs(y).max() * 2 + 2.0 ** -149


@pytest.mark.parametrize("fmt,tol", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11), ("e4m3", 2.0 ** -4)])
def test_dequantize_error_bound(fmt, tol):
    y = rand_c((2, 5, 63), 61).astype(np.complex64)
    codes, sc = oracle.quantize(y, fmt)
    z = oracle.dequantize(codes, sc, fmt, 63)
    big = np.abs(y) > 0.05 * np.abs(y).max()
    for part in (np.real, np.imag):
        a, b = part(z), part(y).astype(np.float64)
        m = big & (np.abs(b) > 0.05 * np.abs(y).max())
        assert np.max(np.abs(a[m] - b[m]) / np.abs(b[m])) <= tol


# ------------------------------------------------------------- metrics
def test_metrics_by_hand():
    h = np.array([[[1.0, 1j, -2.0]]])
    hh = np.array([[[1.5, 0.0, -2.0]]])
    assert abs(oracle.mae(hh, h) - (0.5 + 1.0 + 0.0) / 3) < 1e-15     # Eq. 12
    assert abs(oracle.nmse_db(hh, h) - 10 * np.log10(1.25 / 6.0)) < 1e-12
    assert abs(oracle.relerr(hh, h) - np.sqrt(1.25 / 6.0)) < 1e-15


def test_synth_is_deterministic_and_normalised():
    cfg = synth.PLAIN
    a = synth.batch_draws(cfg)
    b = synth.batch_draws(cfg)
    assert np.array_equal(a["h"], b["h"]) and np.array_equal(a["w"], b["w"])
    e = np.sum(np.abs(a["h"]) ** 2, axis=-1)
    assert np.allclose(e, 1.0)
    f3 = synth.batch_draws(synth.FP32, frames=[3])
    assert np.array_equal(f3["h"][0], synth.frame_draws(synth.FP32, 3)[1])
    shp = synth.varlen_shapes(64)
    assert np.all(shp[:, 2] * shp[:, 3] <= (1 << shp[:, 1]) - 1)



@pytest.mark.parametrize("L,lnz", [(64, 64), (128, 16), (128, 1), (32, 5)])
def test_sparse_taps_follow_the_section_ii_model(L, lnz):
    """Section II's channel: lnz non-zero taps at distinct positions of an
    L-tap CIR, each CN(0, p), p = 1 / (N_t sqrt(lnz)), positions uniform."""
    n_tx = 16
    shape = (40, 16, 4)
    h = synth.sparse_taps(shape, L, lnz, n_tx, seed=5)
    assert h.shape == shape + (L,) and h.dtype == np.complex128
    assert np.array_equal(h, synth.sparse_taps(shape, L, lnz, n_tx, seed=5))
    nz = h.reshape(-1, L) != 0
    assert np.all(nz.sum(axis=1) == lnz)          # exactly lnz distinct taps per CIR
    v = h.reshape(-1, L)[nz]
    p = 1.0 / (n_tx * np.sqrt(lnz))
    n = v.size
    # E|h|^2 = p, E re^2 = E im^2 = p/2, E re*im = 0; |h|^2/p is Exp(1), so
    # its sample mean has standard deviation 1/sqrt(n): 6 sigma bounds
    assert abs(np.mean(np.abs(v) ** 2) / p - 1.0) < 6.0 / np.sqrt(n)
    assert abs(np.mean(v.real ** 2) / (p / 2) - 1.0) < 6.0 * np.sqrt(2.0 / n)
    assert abs(np.mean(v.imag ** 2) / (p / 2) - 1.0) < 6.0 * np.sqrt(2.0 / n)
    assert abs(np.mean(v.real * v.imag)) / (p / 2) < 6.0 / np.sqrt(n)
    # every position is hit with probability lnz / L
    if lnz < L:
        cirs = nz.shape[0]
        hits = nz.sum(axis=0)
        q = lnz / L
        sd = np.sqrt(cirs * q * (1 - q))
        assert np.all(np.abs(hits - cirs * q) < 6.0 * sd)


# ------------------------------- per-cell sequences and Eq. 8 lag spacing
def _totient(n):
    r, m, p = n, n, 2
    while p * p <= m:
        if m % p == 0:
            while m % p == 0:
                m //= p
            r -= r // p
        p += 1
    if m > 1:
        r -= r // m
    return r


def _is_shift(u, v):
    """True when v is a circular shift of u."""
    return any(np.array_equal(np.roll(u, k), v) for k in range(u.size))


@pytest.mark.parametrize("d", list(range(2, 11)))
def test_primitive_polynomial_count(d):
    """There are phi(2^d - 1)/d primitive binary polynomials of degree d, so
    as many feedback masks give maximal-length sequences."""
    assert len(oracle.primitive_masks(d)) == _totient((1 << d) - 1) // d


@pytest.mark.parametrize("d", [5, 7, 8])
def test_every_primitive_mask_has_two_level_autocorrelation(d):
    """Eq. 1 holds for every cell's sequence, not only the default one."""
    N = (1 << d) - 1
    for m in oracle.primitive_masks(d):
        s = oracle.mseq_mask(d, m).astype(np.float64)
        assert np.sum(s == -1) == (N + 1) // 2
        ac = np.real(np.fft.ifft(np.abs(np.fft.fft(s)) ** 2))
        assert abs(ac[0] - N) < 1e-6 and np.max(np.abs(ac[1:] + 1.0)) < 1e-6


@pytest.mark.parametrize("d", list(range(2, 11)))
def test_default_sequence_is_a_primitive_mask_sequence(d):
    seqs = [oracle.mseq_mask(d, m) for m in oracle.primitive_masks(d)]
    assert any(np.array_equal(oracle.mseq(d), s) for s in seqs)


@pytest.mark.parametrize("d", [5, 7, 10])
def test_reciprocal_polynomial_reverses_the_sequence(d):
    """x^d f(1/x) generates the time-reversed m-sequence (up to a shift)."""
    for m in oracle.primitive_masks(d)[:6]:
        rec = 1 | sum(1 << (d - i) for i in range(1, d) if (m >> i) & 1)
        s, r = oracle.mseq_mask(d, m), oracle.mseq_mask(d, rec)
        assert r is not None and _is_shift(s[::-1].copy(), r)


@pytest.mark.parametrize("d", [5, 7, 9])
def test_decimation_by_three_gives_a_preferred_pair(d):
    """Gold: for odd d the sequence decimated by 3 is another cell's
    m-sequence and the pair's cross-correlation takes only the three values
    -1, -t, t - 2 with t = 2^((d+1)/2) + 1."""
    N = (1 << d) - 1
    s = oracle.mseq(d).astype(np.int64)
    u = s[(3 * np.arange(N)) % N]
    owners = [m for m in oracle.primitive_masks(d)
              if _is_shift(oracle.mseq_mask(d, m).astype(np.int64), u)]
    assert len(owners) == 1 and oracle.mseq_mask(d, owners[0]) is not None
    cc = np.rint(np.real(np.fft.ifft(np.conj(np.fft.fft(s)) * np.fft.fft(u)))).astype(int)
    t = (1 << ((d + 1) // 2)) + 1
    assert set(cc.tolist()) == {-1, -t, t - 2}


def test_mseq_mask_rejects_non_primitive_and_bad_masks():
    assert oracle.mseq_mask(4, 0xF) is None        # x^4+x^3+x^2+x+1: period 5
    assert oracle.mseq_mask(5, 0x0) is None        # x^5: not invertible
    assert oracle.mseq_mask(6, 0x9) is None        # x^6+x^3+1: irreducible, order 9
    with pytest.raises(ValueError):
        oracle.mseq_mask(5, 1 << 5)
    with pytest.raises(ValueError):
        oracle.mseq_mask(1, 1)


@pytest.mark.parametrize("N,T,L", [(31, 3, 7), (127, 4, 16), (1023, 16, 32), (255, 7, 36)])
def test_eq8_lags_are_distinct_blocks_with_guards(N, T, L):
    lag = oracle.lags(N, T, L, "eq8").reshape(T, L)
    D = N // T
    assert np.array_equal(lag[:, 0], D * np.arange(T))
    assert np.array_equal(np.diff(lag, axis=1), np.ones((T, L - 1)))
    assert len(np.unique(lag % N)) == T * L                     # no overlap
    assert np.all(lag[1:, 0] - lag[:-1, -1] - 1 == D - L)        # guard lags
    assert np.array_equal(oracle.lags(N, 1, L, "eq8"), oracle.lags(N, 1, L))
    with pytest.raises(ValueError):
        oracle.lags(N, T, N // T + 1, "eq8")


@pytest.mark.parametrize("d,T,L", [(5, 3, 7), (7, 4, 16), (8, 5, 40)])
def test_correlate_and_adjoint_at_eq8_lags_equal_dense_products(d, T, L):
    """Column k of P is the sequence delayed by lag k (np.roll)."""
    s = oracle.mseq(d)
    N = s.size
    lag = oracle.lags(N, T, L, "eq8")
    P = np.stack([np.roll(s.astype(np.float64), int(k)) for k in lag], axis=1)
    Y = rand_c((2, 3, N), 41)
    G = rand_c((2, 3, T * L), 42)
    assert np.max(np.abs(oracle.correlate(Y, s, T * L, lag) - Y @ P / N)) < 1e-13
    assert np.max(np.abs(oracle.adjoint(G, s, lag) - G @ P.T / N)) < 1e-13


@pytest.mark.parametrize("spacing", ["contiguous", "eq8"])
def test_noiseless_least_squares_recovers_channel_at_any_spacing(spacing):
    """Eq. 9 with each transmitter's shift, then the correlator at the same
    lags and the closed-form inverse of P^T P: the CIRs come back exactly,
    for any set of distinct lags."""
    s = oracle.mseq(7)
    N = s.size
    T, L = 5, 12
    lag = oracle.lags(N, T, L, spacing)
    h = rand_c((1, 3, T, L), 43)
    y, _ = oracle.received(s, h, np.zeros((1, 3, N)), np.array([400.0]),
                           shifts=lag.reshape(T, L)[:, 0])
    x = oracle.ls_closed_form(oracle.correlate(y, s, T * L, lag), N)
    assert np.max(np.abs(x - h.reshape(1, 3, T * L))) < 1e-12


def test_eq8_guard_lags_absorb_channel_tails():
    """A channel longer than L: with adjacent blocks the tail of transmitter
    0 lands on transmitter 1's first taps; with Eq. 8's shifts it falls in
    the guard lags, and transmitter 1 only sees the -1/N floor of Eq. 1."""
    s = oracle.mseq(8)
    N = s.size
    T, L, tail = 4, 16, 8
    h = np.zeros((1, 1, T, L + tail), dtype=np.complex128)
    h[0, 0, 0, L:] = 1.0                                         # taps past L
    for spacing in ("contiguous", "eq8"):
        lag = oracle.lags(N, T, L, spacing)
        y, _ = oracle.received(s, h, np.zeros((1, 1, N)), np.array([400.0]),
                               shifts=lag.reshape(T, L)[:, 0])
        H = oracle.correlate(y, s, T * L, lag).reshape(T, L)
        leak = np.max(np.abs(H[1, :tail]))
        if spacing == "contiguous":                              # the tap, less
            assert abs(leak - (1.0 - (tail - 1) / N)) < 1e-12    # the others' floor
        else:
            assert abs(leak - tail / N) < 1e-12


def test_other_cell_interference_is_bounded_by_cross_correlation():
    """A receiver of cell A hears cell B (a preferred pair): the correlator
    sees B's CIR through the cross-correlation, so each estimated tap is at
    most max|C_AB| / N times the sum of B's tap magnitudes, and equals the
    circular cross-correlation of the two sequences weighted by B's taps."""
    d = 7
    N = (1 << d) - 1
    sa = oracle.mseq(d)
    sb = sa[(3 * np.arange(N)) % N].copy()                       # other cell
    T, L = 4, 8
    hb = rand_c((1, 2, T, L), 44)
    y, _ = oracle.received(sb, hb, np.zeros((1, 2, N)), np.array([400.0]))
    H = oracle.correlate(y, sa, T * L)
    cab = np.real(np.fft.ifft(np.conj(np.fft.fft(sa.astype(float))) * np.fft.fft(sb.astype(float))))
    bound = np.max(np.abs(cab)) / N * np.sum(np.abs(hb), axis=(2, 3))
    assert np.all(np.max(np.abs(H), axis=-1) <= bound + 1e-12)
    # H_A[k] = (1/N) sum_j hb[j] C_AB(k - j)  (j over B's stacked lags)
    hbs = hb.reshape(1, 2, T * L)
    k = np.arange(T * L)
    C = cab[(k[:, None] - k[None, :]) % N]                       # [k, j]
    assert np.max(np.abs(H - hbs @ C.T / N)) < 1e-12

"""The oracle's pins are not vacuous: each plausible mistake below, planted in
the oracle (on the CPU, by replacing one function for the duration of a
test), makes at least one pin of tests/test_oracle_pins.py fail.

The mutants are written here in numpy from each function's definition with
one deliberate error: a flipped lag sign, a missing 1/N, a conjugated input,
an off-by-one lag, the adjoint's shift reversed, a wrong constant in the
least-squares closed form, a transmitter advanced instead of delayed, the
bf16 rounding truncating, Eq. 8's quotient taken up instead of down, the
refinement step subtracting, a flipped sequence bit.
"""
import numpy as np
import pytest

import oracle
import test_oracle_pins as pins

_orig = {name: getattr(oracle, name) for name in
         ("correlate", "adjoint", "ls_closed_form", "received", "lags", "refine", "mseq",
          "_bf16_bits")}


def _corr(Y, s, K, lag, sign=-1, scale=True):
    Y = np.asarray(Y, np.complex128)
    s = np.asarray(s, np.float64)
    N = s.size
    lag = np.arange(K) if lag is None else np.asarray(lag)
    idx = (np.arange(N)[:, None] + sign * lag[None, :]) % N
    H = Y @ s[idx]
    return H / N if scale else H


def m_corr_lag_sign(Y, s, K, lag=None, threads=None):
    return _corr(Y, s, K, lag, sign=+1)


def m_corr_no_norm(Y, s, K, lag=None, threads=None):
    return _corr(Y, s, K, lag, scale=False)


def m_corr_conj(Y, s, K, lag=None, threads=None):
    return _corr(np.conj(np.asarray(Y, np.complex128)), s, K, lag)


def m_corr_off_by_one(Y, s, K, lag=None, threads=None):
    lag = np.arange(K) if lag is None else np.asarray(lag)
    return _corr(Y, s, K, lag + 1)


def m_adjoint_reversed(G, s, lag=None):
    G = np.asarray(G, np.complex128)
    s = np.asarray(s, np.float64)
    N, K = s.size, G.shape[-1]
    lag = np.arange(K) if lag is None else np.asarray(lag)
    idx = (np.arange(N)[None, :] + lag[:, None]) % N       # s[(n + k) mod N]
    return G @ s[idx] / N


def m_ls_constant(H, N):
    H = np.asarray(H, np.complex128)
    K = H.shape[-1]
    return N / (N + 1.0) * (H + H.sum(axis=-1, keepdims=True) / (N - K))


def m_received_advance(s, h, w, snr_db, shifts=None):
    s = np.asarray(s)
    return _orig["received"](np.roll(s, -2), h, w, snr_db, shifts)


def m_bf16_truncate(x32):
    u = np.asarray(x32, np.float32).view(np.uint32)
    return (u >> 16).astype(np.uint16)


def m_lags_ceil(N, T, L, spacing="contiguous"):
    if spacing != "eq8":
        return _orig["lags"](N, T, L, spacing)
    if T * L > N:
        raise ValueError("Eq. 8 spacing needs T*L <= N")
    t = np.repeat(np.arange(T), L)
    l = np.tile(np.arange(L), T)
    return ((-(-N // T)) * t + l).astype(np.int32)


def m_refine_sign(y, s, K, steps, lag=None):
    y = np.asarray(y, np.complex128)
    N = y.shape[2]
    x = oracle.correlate(y, s, K, lag)
    out = [x]
    for _ in range(steps):
        r = y - N * oracle.adjoint(x, s, lag)
        x = x - oracle.correlate(r, s, K, lag)
        out.append(x)
    return out


def m_mseq_bit(d):
    s = _orig["mseq"](d).copy()
    s[len(s) // 2] = -s[len(s) // 2]
    return s


# mutant -> (oracle attribute, replacement, pins that should notice)
MUTANTS = {
    "correlate: lag sign": ("correlate", m_corr_lag_sign, [
        lambda: pins.test_correlate_equals_dense_brute_force(5, 8),
        lambda: pins.test_demultiplex_view()]),
    "correlate: no 1/N": ("correlate", m_corr_no_norm, [
        lambda: pins.test_correlate_equals_fft_cross_correlation(7, 64),
        lambda: pins.test_noiseless_least_squares_recovers_channel()]),
    "correlate: conjugated input": ("correlate", m_corr_conj, [
        lambda: pins.test_correlate_equals_dense_brute_force(5, 8),
        lambda: pins.test_linearity_and_shift_equivariance()]),
    "correlate: lag off by one": ("correlate", m_corr_off_by_one, [
        lambda: pins.test_correlate_equals_dense_brute_force(5, 8),
        lambda: pins.test_demultiplex_view()]),
    "adjoint: shift reversed": ("adjoint", m_adjoint_reversed, [
        lambda: pins.test_adjoint_brute_force_and_dot_identity(5, 8),
        lambda: pins.test_refinement_converges_to_lstsq()]),
    "least squares: N - K for N + 1 - K": ("ls_closed_form", m_ls_constant, [
        lambda: pins.test_noiseless_least_squares_recovers_channel(),
        lambda: pins.test_refinement_converges_to_lstsq()]),
    "receive model: transmitter advanced": ("received", m_received_advance, [
        lambda: pins.test_received_model_equals_dense_product(),
        lambda: pins.test_demultiplex_view()]),
    "bf16 rounding truncates": ("_bf16_bits", m_bf16_truncate, [
        lambda: pins.test_bf16_and_f16_codes_match_torch_rounding()]),
    "Eq. 8 quotient rounded up": ("lags", m_lags_ceil, [
        lambda: pins.test_eq8_lags_are_distinct_blocks_with_guards(127, 4, 16),
        lambda: pins.test_eq8_lags_are_distinct_blocks_with_guards(31, 3, 7)]),
    "refinement step subtracts": ("refine", m_refine_sign, [
        lambda: pins.test_refinement_converges_to_lstsq(),
        lambda: pins.test_refinement_contraction_rates()]),
    "sequence with one bit flipped": ("mseq", m_mseq_bit, [
        lambda: pins.test_mseq_balance_and_two_level_autocorrelation(7),
        lambda: pins.test_mseq_autocorrelation_direct(5)]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_a_pin_catches_the_mutant(name, monkeypatch):
    attr, repl, checks = MUTANTS[name]
    monkeypatch.setattr(oracle, attr, repl)
    caught = 0
    for check in checks:
        try:
            check()
        except (AssertionError, ValueError):
            caught += 1
    assert caught > 0, f"no pin noticed: {name}"


def test_the_unmutated_oracle_passes_the_same_checks():
    for _, _, checks in MUTANTS.values():
        for check in checks:
            check()

"""FP64 oracle for PN-sequence correlation channel estimation (arXiv 2206.05506).

TEST INFRASTRUCTURE. Only ``tests/``, the smoke check and the benchmark's CPU
baseline leg import this package. It shares no code with the GPU library and
never imports it; the GPU library never imports this package.

What it computes, each function citing the passage it follows:

* ``mseq``        m-sequence (Section II-A, Eq. 1) -- C, own LFSR.
* ``mseq_mask`` / ``primitive_masks``  the m-sequence of any feedback
                  polynomial, and every primitive one of a degree (the
                  per-cell sequences of Section II-B) -- C, own LFSR.
* ``lags``        the lag each estimated tap sits at: adjacent blocks of L, or
                  Eq. 8's shifts floor(N/T)*t.
* ``correlate``   correlator at the T*L multiplexed lags (Eq. 3, Eq. 10) -- C.
* ``adjoint``     its transpose, circular convolution with the sequence -- C.
* ``received``    multiplexed receive model y = sum_t s shifted by the
                  transmitter's lag, convolved with h_t, plus noise
                  (Eq. 6 / Eq. 9) -- numpy FFT.
* ``refine``      least-squares refinement iterates built from the two above.
* ``loss_grad``   ||y - P h||^2 and its gradient.
* ``quantize`` / ``dequantize``  the reduced-precision storage of Y with a
                  per-frame power-of-two scale (the half-precision conversion
                  of Section III-B), bit-exact model.
* metrics: ``nmse_db``, ``mae`` (Eq. 12), ``relerr``.

Pins (tests/test_oracle_pins.py) tie every function to something other than
itself: the two-level autocorrelation of Eq. 1, closed forms that follow from
it, a textbook FFT correlation, dense brute force, scipy's circulant and lstsq,
and finite differences. No function here is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    c_dp = ctypes.POINTER(ctypes.c_double)
    c_sp = ctypes.POINTER(ctypes.c_byte)
    c_ip = ctypes.POINTER(ctypes.c_int)
    lib.oracle_mseq.argtypes = [ctypes.c_int, c_sp]
    lib.oracle_mseq.restype = ctypes.c_int
    lib.oracle_mseq_mask.argtypes = [ctypes.c_int, ctypes.c_uint, c_sp]
    lib.oracle_mseq_mask.restype = ctypes.c_int
    for fn in (lib.oracle_correlate, lib.oracle_adjoint):
        fn.argtypes = [c_dp, c_sp, ctypes.c_int, c_ip, ctypes.c_int, ctypes.c_long,
                       ctypes.c_int, c_dp]
        fn.restype = None
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _sp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_byte))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def threads() -> int:
    """OpenMP threads the C oracle uses (the core count of a timed run)."""
    return int(_load().oracle_threads())


# --------------------------------------------------------------------------
# a1: the sequence
# --------------------------------------------------------------------------
def mseq(d: int) -> np.ndarray:
    """m-sequence of length 2^d - 1 as int8 +-1 (Section II-A, Eq. 1)."""
    N = (1 << d) - 1
    s = np.zeros(N, dtype=np.int8)
    got = _load().oracle_mseq(int(d), _sp(s))
    if got != N:
        raise ValueError(f"degree {d} outside [2, 16]")
    return s


def mseq_mask(d: int, mask: int):
    """m-sequence of the feedback polynomial x^d + sum_{bit i of mask} x^i.

    Same recurrence, start state and +-1 mapping as ``mseq``. Returns the
    int8 +-1 sequence of length 2^d - 1, or None when the polynomial is not
    primitive (the bits do not repeat with period exactly 2^d - 1).
    """
    N = (1 << d) - 1
    s = np.zeros(N, dtype=np.int8)
    got = _load().oracle_mseq_mask(int(d), int(mask), _sp(s))
    if got < 0:
        raise ValueError(f"degree {d} outside [2, 16] or mask {mask:#x} has bits >= d")
    return s if got == N else None


def primitive_masks(d: int) -> list:
    """Every feedback mask of degree d whose sequence is maximal length, by
    trying all 2^d masks (the candidate sequences of the cells of Section
    II-B)."""
    return [m for m in range(1 << d) if mseq_mask(d, m) is not None]


def lags(N: int, T: int, L: int, spacing: str = "contiguous") -> np.ndarray:
    """Lag of estimated tap k = t*L + l (transmitter t, tap l), int32 [T*L].

    "contiguous": t*L + l, the transmitters' blocks adjacent.
    "eq8":        floor(N/T)*t + l, the circular shift of Eq. 8 with the
                  non-integer N/T taken down to an integer, which leaves
                  floor(N/T) - L guard lags after every block. Needs
                  T*L <= N (Eq. 7) so that blocks do not overlap.
    """
    t = np.repeat(np.arange(T, dtype=np.int64), L)
    l = np.tile(np.arange(L, dtype=np.int64), T)
    if spacing == "contiguous":
        return (t * L + l).astype(np.int32)
    if spacing == "eq8":
        if T * L > N:
            raise ValueError("Eq. 8 spacing needs T*L <= N")
        return ((N // T) * t + l).astype(np.int32)
    raise ValueError(spacing)


def degree_of(N: int) -> int:
    d = int(N + 1).bit_length() - 1
    if (1 << d) - 1 != N:
        raise ValueError(f"N={N} is not 2^d - 1")
    return d


# --------------------------------------------------------------------------
# a4 / a7: correlator and adjoint
# --------------------------------------------------------------------------
def _as_c128(x, ndim):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    if x.ndim != ndim:
        raise ValueError(f"expected {ndim}-d array, got shape {x.shape}")
    return x


def _lag_array(K: int, lag) -> np.ndarray:
    lag = np.arange(K, dtype=np.int32) if lag is None else np.ascontiguousarray(lag, np.int32)
    if lag.shape != (K,):
        raise ValueError("one lag per estimated tap expected")
    return lag


def correlate(Y, s, K: int, lag=None, threads=None) -> np.ndarray:
    """H[b,r,k] = (1/N) sum_n Y[b,r,n] s[(n-lag[k]) mod N], k < K (Eq. 3, Eq. 10).

    Y: [B, R, N] complex; lag: [K] ints (default k, the adjacent blocks);
    threads: OpenMP threads for this call (default: all). Returns
    [B, R, K] complex128. The CIR of transmitter t sits at
    H[..., t*L:(t+1)*L] (the de-multiplexing of Eq. 10).
    """
    Y = _as_c128(Y, 3)
    s = np.ascontiguousarray(s, dtype=np.int8)
    B, R, N = Y.shape
    if s.shape != (N,):
        raise ValueError("sequence length does not match Y")
    lag = _lag_array(int(K), lag)
    H = np.empty((B, R, K), dtype=np.complex128)
    lib = _load()
    before = lib.oracle_threads()
    if threads:
        lib.oracle_set_threads(int(threads))
    try:
        lib.oracle_correlate(_dp(Y.view(np.float64)), _sp(s), N, _ip(lag), int(K), B, R,
                             _dp(H.view(np.float64)))
    finally:
        if threads:
            lib.oracle_set_threads(before)
    return H


def adjoint(G, s, lag=None) -> np.ndarray:
    """A[b,r,n] = (1/N) sum_k G[b,r,k] s[(n-lag[k]) mod N]: transpose of correlate.

    G: [B, R, K] complex; lag as in ``correlate``. Returns [B, R, N]
    complex128. N * adjoint(h) is the noiseless multiplexed received frame of
    Eq. 9 for stacked CIRs h.
    """
    G = _as_c128(G, 3)
    s = np.ascontiguousarray(s, dtype=np.int8)
    B, R, K = G.shape
    N = s.shape[0]
    lag = _lag_array(K, lag)
    A = np.empty((B, R, N), dtype=np.complex128)
    _load().oracle_adjoint(_dp(G.view(np.float64)), _sp(s), N, _ip(lag), K, B, R,
                           _dp(A.view(np.float64)))
    return A


# --------------------------------------------------------------------------
# Receive model (Eq. 6 / Eq. 9), used to build test inputs
# --------------------------------------------------------------------------
def received(s, h, w, snr_db, shifts=None):
    """Noisy multiplexed frame y = P h_stack + sigma * w  (Eq. 9).

    s: [N] +-1; h: [B, R, T, Lh] complex CIRs; w: [B, R, N] unit-variance
    complex noise; snr_db: [B] receive SNR per frame; shifts: [T] circular
    shift of each transmitter's copy of the sequence (default t*Lh, adjacent
    blocks; Eq. 8's floor(N/T)*t otherwise). Transmitter t sends the sequence
    delayed by shifts[t], so its taps occupy lags shifts[t] ... shifts[t]+Lh-1.
    The clean frame is the sum over transmitters of the circular convolution
    of the delayed sequence with h_t, computed with numpy's FFT. sigma^2 is
    the mean clean power of the frame divided by 10^(SNR/10). Returns
    (y, y_clean), complex128.
    """
    s = np.asarray(s, dtype=np.float64)
    N = s.shape[0]
    h = np.asarray(h, dtype=np.complex128)
    B, R, T, L = h.shape
    if shifts is None:
        shifts = [t * L for t in range(T)]
    hs = np.zeros((B, R, N), dtype=np.complex128)
    # lags beyond N wrap around (they alias when T*L > N)
    for t in range(T):
        for l in range(L):
            hs[:, :, (shifts[t] + l) % N] += h[:, :, t, l]
    y_clean = np.fft.ifft(np.fft.fft(hs, axis=-1) * np.fft.fft(s), axis=-1)
    p = np.mean(np.abs(y_clean) ** 2, axis=(1, 2))
    sigma = np.sqrt(p / 10.0 ** (np.asarray(snr_db, dtype=np.float64) / 10.0))
    y = y_clean + sigma[:, None, None] * np.asarray(w, dtype=np.complex128)
    return y, y_clean


# --------------------------------------------------------------------------
# a6: least-squares refinement, and the loss it descends
# --------------------------------------------------------------------------
def refine(y, s, K: int, steps: int, lag=None):
    """Iterates x_0 = H(y), x_{j+1} = x_j + H(y - N A(x_j)), j < steps.

    H is ``correlate`` and N A(x) = P x is ``adjoint`` times N, so each step
    adds P^T (y - P x) / N: the refinement x <- x + P^T (y - P x)/N, i.e.
    gradient descent on ||y - P x||^2 with step 1/(2N). Returns the list
    [x_0, ..., x_steps] of complex128 arrays [B, R, K].
    """
    y = _as_c128(y, 3)
    N = y.shape[2]
    x = correlate(y, s, K, lag)
    out = [x]
    for _ in range(steps):
        r = y - N * adjoint(x, s, lag)
        x = x + correlate(r, s, K, lag)
        out.append(x)
    return out


def loss_grad(y, s, x, lag=None):
    """Loss ||y - P x||^2 summed over all frames and antennas, and its
    gradient in PyTorch's convention for a real loss of complex x
    (dL/d(re) + i dL/d(im)), which is -2 P^T (y - P x) = -2N H(y - P x)."""
    y = _as_c128(y, 3)
    x = _as_c128(x, 3)
    N = y.shape[2]
    r = y - N * adjoint(x, s, lag)
    loss = float(np.sum(np.abs(r) ** 2))
    grad = -2.0 * N * correlate(r, s, x.shape[2], lag)
    return loss, grad


def ls_closed_form(H, N: int):
    """Least-squares CIR from a correlator output when T*L <= N.

    The sequence's two-level autocorrelation (Eq. 1) gives, for any K
    distinct lags (adjacent or Eq. 8's),
    P^T P = (N+1) I - J (J all-ones), whose inverse is
    (I + J/(N+1-K)) / (N+1). With H = P^T y / N this yields
    x_LS = N/(N+1) * (H + sum(H)/(N+1-K)), the sum over the K lags of a row.
    """
    H = np.asarray(H, dtype=np.complex128)
    K = H.shape[-1]
    if K > N:
        raise ValueError("least squares is not unique when T*L > N")
    tot = H.sum(axis=-1, keepdims=True)
    return N / (N + 1.0) * (H + tot / (N + 1.0 - K))


# --------------------------------------------------------------------------
# a3: reduced-precision storage of Y (bit-exact model)
# --------------------------------------------------------------------------
FORMATS = ("bf16", "f16", "e4m3")
_TARGET = {"bf16": 1.0, "f16": 1.0, "e4m3": 448.0}


def frame_scale(y, fmt: str) -> np.ndarray:
    """Per-frame power-of-two scale: the smallest 2^e with maxabs <= target*2^e,
    and at least 2^-126.

    maxabs is the largest |re| or |im| over the frame's R*N samples; target is
    1 for bf16/f16 and 448 (the largest finite e4m3) for e4m3. A frame of
    zeros, or with a non-finite maxabs, gets scale 1. Returns float32 [B].
    """
    y = np.asarray(y)
    B = y.shape[0]
    v = np.concatenate([np.abs(y.real).reshape(B, -1),
                        np.abs(y.imag).reshape(B, -1)], axis=1)
    mx = v.max(axis=1).astype(np.float64)
    tgt = _TARGET[fmt]
    out = np.ones(B, dtype=np.float32)
    for b in range(B):
        m = mx[b]
        if not np.isfinite(m) or m == 0.0:
            continue
        e = 0
        while m > tgt * 2.0 ** e:
            e += 1
        while m <= tgt * 2.0 ** (e - 1):
            e -= 1
        # never below the smallest normal float32, 2^-126: a frame of
        # subnormal samples would otherwise get a scale whose reciprocal
        # overflows (the paper does not treat such frames)
        e = max(e, -126)
        out[b] = np.float32(2.0 ** e)
    return out


def _bf16_bits(x32: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit pattern, round to nearest even (NaN kept)."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    nan = np.isnan(x32)
    r[nan] = ((u[nan] >> 16).astype(np.uint16) | 0x0040)
    return r


def _e4m3_table() -> np.ndarray:
    """Values of the 127 non-negative finite OCP e4m3fn codes 0x00..0x7E."""
    v = np.zeros(127, dtype=np.float64)
    for c in range(127):
        E, m = c >> 3, c & 7
        v[c] = (m / 8.0) * 2.0 ** -6 if E == 0 else (1 + m / 8.0) * 2.0 ** (E - 7)
    return v


_E4M3 = _e4m3_table()


def _e4m3_bits(x32: np.ndarray) -> np.ndarray:
    """float32 -> OCP e4m3fn code, round to nearest even, saturating at +-448.

    Infinities saturate to +-448; NaN maps to 0x7F with its sign bit.
    """
    x = x32.astype(np.float64)
    a = np.abs(x)
    sign = (np.signbit(x)).astype(np.uint8) << 7
    a_c = np.minimum(np.nan_to_num(a, nan=0.0, posinf=448.0), 448.0)
    hi = np.searchsorted(_E4M3, a_c, side="left")       # first value >= a
    hi = np.minimum(hi, 126)
    lo = np.maximum(hi - 1, 0)
    dlo = a_c - _E4M3[lo]
    dhi = _E4M3[hi] - a_c
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo).astype(np.uint8)
    code = np.where(a_c == _E4M3[hi], hi, code).astype(np.uint8)
    out = code | sign
    out[np.isnan(x)] = 0x7F | sign[np.isnan(x)]
    return out


def quantize(y, fmt: str):
    """Reduced-precision copy of a complex64 frame batch.

    y: [B, R, N] complex64. Each value is multiplied (in float32) by 1/scale_b
    and rounded to nearest even into ``fmt``. Layout of the result, per frame
    and antenna: the real plane then the imaginary plane, each padded from N
    to Np = N + 1 samples with a zero. Returns (codes, scales): codes is
    uint16 [B, R, 2, Np] for bf16/f16 and uint8 [B, R, 2, Np] for e4m3.
    """
    y = np.asarray(y, dtype=np.complex64)
    B, R, N = y.shape
    sc = frame_scale(y, fmt)
    inv = (np.float32(1.0) / sc).astype(np.float32)
    planes = np.stack([y.real, y.imag], axis=2).astype(np.float32)  # [B,R,2,N]
    v = (planes * inv[:, None, None, None]).astype(np.float32)
    if fmt == "bf16":
        c = _bf16_bits(v)
        dt = np.uint16
    elif fmt == "f16":
        c = v.astype(np.float16).view(np.uint16)
        dt = np.uint16
    elif fmt == "e4m3":
        c = _e4m3_bits(v)
        dt = np.uint8
    else:
        raise ValueError(fmt)
    out = np.zeros((B, R, 2, N + 1), dtype=dt)
    out[..., :N] = c
    return out, sc


def decode(codes, fmt: str) -> np.ndarray:
    """Exact float64 value of each stored code."""
    c = np.asarray(codes)
    if fmt == "bf16":
        return (c.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    if fmt == "f16":
        return c.astype(np.uint16).view(np.float16).astype(np.float64)
    if fmt == "e4m3":
        mag = c & 0x7F
        val = np.where(mag == 0x7F, np.nan, _E4M3[np.minimum(mag, 126)])
        return np.where(c & 0x80, -val, val)
    raise ValueError(fmt)


def dequantize(codes, scales, fmt: str, N: int) -> np.ndarray:
    """complex128 [B, R, N] value of a quantized batch: code * scale (exact)."""
    v = decode(codes, fmt)[..., :N] * np.asarray(scales, np.float64)[:, None, None, None]
    return v[:, :, 0, :] + 1j * v[:, :, 1, :]


# --------------------------------------------------------------------------
# Metrics (Section IV)
# --------------------------------------------------------------------------
def nmse_db(h_hat, h) -> float:
    """Per-frame sum|h_hat-h|^2 / sum|h|^2, averaged over frames, in dB."""
    h_hat = np.asarray(h_hat)
    h = np.asarray(h)
    B = h.shape[0]
    e = np.sum(np.abs(h_hat - h).reshape(B, -1) ** 2, axis=1)
    p = np.sum(np.abs(h).reshape(B, -1) ** 2, axis=1)
    return float(10.0 * np.log10(np.mean(e / p)))


def mae(h_hat, h) -> float:
    """Mean absolute tap error over all taps, antennas and transmitters (Eq. 12)."""
    return float(np.mean(np.abs(np.asarray(h_hat) - np.asarray(h))))


def relerr(x, ref) -> float:
    """max over frames of ||x - ref||_F / ||ref||_F (frame = leading axis)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    B = ref.shape[0]
    num = np.sqrt(np.sum(np.abs(x - ref).reshape(B, -1) ** 2, axis=1))
    den = np.sqrt(np.sum(np.abs(ref).reshape(B, -1) ** 2, axis=1))
    return float(np.max(num / np.where(den == 0, 1.0, den)))

"""Shared helpers of the GPU parity tests (inputs and comparisons only)."""
import numpy as np
import torch

import oracle
import synth


def dev(x, dtype=torch.complex64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def host(t):
    return t.detach().cpu().numpy()


def frames(cfg, nframes=None, seed_offset=0):
    """(y complex64 host [F,R,N], h [F,R,T,L], s) of the first frames of cfg,
    built by the oracle's receive model from the seeded draws."""
    F = cfg.B if nframes is None else nframes
    d = synth.batch_draws(cfg, frames=range(seed_offset, seed_offset + F))
    s = oracle.mseq(cfg.d)
    y, _ = oracle.received(s, d["h"], d["w"], d["snr_db"])
    return y.astype(np.complex64), d["h"], s


def bf16_round(y):
    """complex64 -> complex128 with re and im rounded to bf16 (nearest even),
    the values a bf16 matrix-core operand holds."""
    y = np.asarray(y, dtype=np.complex64)
    re = oracle.decode(oracle._bf16_bits(y.real.astype(np.float32)), "bf16")
    im = oracle.decode(oracle._bf16_bits(y.imag.astype(np.float32)), "bf16")
    return re + 1j * im


def device_frames(cfg, s):
    """Large seeded workloads built on the GPU without the library: seeded
    torch draws, then y = P h + sigma w by torch's FFT circular convolution
    with the oracle's sequence s (the receive model of Eq. 9).
    Returns (y complex64 [B,R,N], h complex64 [B,R,T,L]) on the device."""
    d = synth.device_draws(cfg, torch)
    h = d["h"]
    B, R, T, L = h.shape
    K = T * L
    N = cfg.N
    hs = torch.zeros((B, R, N), dtype=torch.complex64, device="cuda")
    idx = torch.arange(K, device="cuda") % N
    hs.index_add_(2, idx, h.reshape(B, R, K))
    S = torch.fft.fft(torch.from_numpy(s.astype(np.float32)).cuda().to(torch.complex64))
    y = torch.empty((B, R, N), dtype=torch.complex64, device="cuda")
    for b0 in range(0, B, 64):
        b1 = min(B, b0 + 64)
        yc = torch.fft.ifft(torch.fft.fft(hs[b0:b1], dim=-1) * S, dim=-1)
        p = (yc.abs() ** 2).mean(dim=(1, 2))
        sigma = torch.sqrt(p / 10.0 ** (d["snr_db"][b0:b1] / 10.0))
        y[b0:b1] = yc + sigma[:, None, None] * d["w"][b0:b1]
    del hs, d
    return y.contiguous(), h


def perr(x, ref) -> float:
    """Parity error of a float result against the oracle: per frame (leading
    axis) the larger of the normwise relative error ||x - ref||_F / ||ref||_F
    and the element-wise max|x - ref| / max|ref|, maximised over frames. One
    tolerance bounds both, so neither a frame-wide drift nor a single wrong
    element (a lag column, an antenna) can hide under the other."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    B = ref.shape[0]
    d = np.abs(x - ref).reshape(B, -1)
    a = np.abs(ref).reshape(B, -1)
    nw = np.sqrt(np.sum(d ** 2, axis=1)) / np.where(np.any(a > 0, axis=1),
                                                     np.sqrt(np.sum(a ** 2, axis=1)), 1.0)
    mx = a.max(axis=1) if a.size else np.zeros(B)
    ew = (d.max(axis=1) if d.size else np.zeros(B)) / np.where(mx == 0, 1.0, mx)
    return float(max(np.max(nw), np.max(ew)))


def tol_sum(tol, n_terms):
    """Parity bound for FP32 sums of n_terms terms: tol up to 4096 terms (every
    reduction of the workloads: sequences up to 4095, lag stacks up to 4096),
    scaled by sqrt(n_terms / 4096) beyond, as the rounding error of an FP32
    sum of random-sign terms grows like the square root of their number."""
    return tol * max(1.0, (n_terms / 4096.0) ** 0.5)


def rows_of(x, rows):
    """Gather (frame, antenna) rows of a [B, R, ...] array into [1, n, ...]."""
    return np.stack([x[b, r] for b, r in rows])[None]

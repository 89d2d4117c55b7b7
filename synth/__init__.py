"""Seeded synthetic inputs shaped like the paper's sweeps (Table I).

This module only draws random numbers; it holds none of the estimator's
arithmetic and imports neither the GPU library nor the oracle, so both sides
of every parity check can consume the same arrays.

Draws per frame b of a configuration with seed S come from their own stream,
``numpy.random.default_rng([S, b])`` (PCG64), in this order:

1. the receive SNR in dB, uniform on the configuration's range;
2. the CIR taps h[r, t, l] ~ CN(0, exp(-l / tau)) (real parts for all
   (r, t, l), then imaginary parts), each (r, t) vector then scaled to unit
   energy (exponential power-delay profile standing in for the paper's
   sparse-tap model of Section II);
3. unit-variance complex white noise w[r, n] (real parts, then imaginary),
   each part N(0, 1/2).

Per-frame streams let a test draw any subset of a large batch.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Config:
    name: str
    d: int          # sequence degree, N = 2^d - 1
    T: int          # multiplexed transmitters
    L: int          # CIR taps per transmitter
    R: int          # receive antennas
    B: int          # frames in the batch
    tau: float      # power-delay-profile decay in taps
    snr_lo: float   # receive SNR range in dB
    snr_hi: float
    seed: int

    @property
    def N(self) -> int:
        return (1 << self.d) - 1

    @property
    def K(self) -> int:
        return self.T * self.L


# The workloads: a plain CPU-checkable case, the FP32 baseline, the precision
# study, the differentiation case and the tiny gradient-check instance.
PLAIN = Config("plain_N127_T4_L16_R16_B1", 7, 4, 16, 16, 1, 4.0, 10.0, 10.0, 0)
FP32 = Config("fp32_N1023_T16_L32_R64_B256", 10, 16, 32, 64, 256, 8.0, 0.0, 20.0, 1)
PRECISION = Config("precision_N4095_T32_L64_R256_B512", 12, 32, 64, 256, 512, 8.0, -5.0, 25.0, 2)
DIFF = Config("diff_N1023_T16_L64_R128_B1024", 10, 16, 64, 128, 1024, 8.0, 0.0, 20.0, 4)
GRADCHECK = Config("gradcheck_N31_T2_L4_R2_B1", 5, 2, 4, 2, 1, 4.0, 10.0, 10.0, 5)

CONFIGS = {c.name: c for c in (PLAIN, FP32, PRECISION, DIFF, GRADCHECK)}


def frame_draws(cfg: Config, b: int):
    """(snr_db, h [R,T,L] complex128, w [R,N] complex128) of frame b."""
    rng = np.random.default_rng([cfg.seed, b])
    snr = rng.uniform(cfg.snr_lo, cfg.snr_hi) if cfg.snr_hi > cfg.snr_lo else cfg.snr_lo
    shape = (cfg.R, cfg.T, cfg.L)
    pdp = np.exp(-np.arange(cfg.L) / cfg.tau)
    hr = rng.standard_normal(shape)
    hi = rng.standard_normal(shape)
    h = (hr + 1j * hi) * np.sqrt(pdp / 2.0)
    h /= np.sqrt(np.sum(np.abs(h) ** 2, axis=-1, keepdims=True))
    wr = rng.standard_normal((cfg.R, cfg.N))
    wi = rng.standard_normal((cfg.R, cfg.N))
    w = (wr + 1j * wi) / np.sqrt(2.0)
    return float(snr), h, w


def batch_draws(cfg: Config, frames=None):
    """Stack ``frame_draws`` over ``frames`` (default: all B frames).

    Returns dict(snr_db [F], h [F,R,T,L], w [F,R,N]) as float64/complex128.
    """
    if frames is None:
        frames = range(cfg.B)
    frames = list(frames)
    F = len(frames)
    snr = np.empty(F)
    h = np.empty((F, cfg.R, cfg.T, cfg.L), dtype=np.complex128)
    w = np.empty((F, cfg.R, cfg.N), dtype=np.complex128)
    for i, b in enumerate(frames):
        snr[i], h[i], w[i] = frame_draws(cfg, b)
    return {"snr_db": snr, "h": h, "w": w}


def gaussian(shape, seed: int, dtype=np.complex128):
    """Plain seeded complex Gaussian array (unit variance), for parity inputs
    that need no channel structure."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    return x.astype(dtype)


# Batching workload: frames of uneven shape, drawn per frame, redrawn while
# T*L exceeds N (the multiplexing bound of Eq. 7 with C = L).
VARLEN_R = (32, 64, 128, 256)
VARLEN_D = (8, 9, 10, 11)          # N = 255, 511, 1023, 2047
VARLEN_T = (4, 8, 16)
VARLEN_L = (16, 32, 64)


def varlen_shapes(nframes: int = 4096, seed: int = 3):
    """Per-frame (R, d, T, L) of the uneven batch, as an int array [F, 4]."""
    rng = np.random.default_rng(seed)
    out = np.empty((nframes, 4), dtype=np.int64)
    for f in range(nframes):
        while True:
            R = VARLEN_R[rng.integers(4)]
            d = VARLEN_D[rng.integers(4)]
            T = VARLEN_T[rng.integers(3)]
            L = VARLEN_L[rng.integers(3)]
            if T * L <= (1 << d) - 1:
                break
        out[f] = (R, d, T, L)
    return out


def device_draws(cfg: Config, torch, device="cuda", frames=None, seed_offset=1000):
    """Seeded draws made on the GPU with torch's generator, for workloads too
    large to draw on the host (the precision study holds 537M samples).
    Same distributions as ``frame_draws``; a different stream (seed
    cfg.seed + seed_offset). Returns dict(snr_db [F], h [F,R,T,L], w [F,R,N])
    as float32 / complex64 device tensors."""
    F = cfg.B if frames is None else frames
    g = torch.Generator(device=device)
    g.manual_seed(cfg.seed + seed_offset)
    snr = cfg.snr_lo + (cfg.snr_hi - cfg.snr_lo) * torch.rand(F, generator=g, device=device)
    pdp = torch.exp(-torch.arange(cfg.L, device=device, dtype=torch.float32) / cfg.tau)
    h = torch.complex(torch.randn((F, cfg.R, cfg.T, cfg.L), generator=g, device=device),
                      torch.randn((F, cfg.R, cfg.T, cfg.L), generator=g, device=device))
    h = h * torch.sqrt(pdp / 2.0)
    h = h / torch.sqrt((h.abs() ** 2).sum(dim=-1, keepdim=True))
    w = torch.complex(torch.randn((F, cfg.R, cfg.N), generator=g, device=device),
                      torch.randn((F, cfg.R, cfg.N), generator=g, device=device))
    w = w / (2.0 ** 0.5)
    return {"snr_db": snr, "h": h, "w": w}


def sparse_taps(shape, L: int, lnz: int, n_tx: int, seed: int) -> np.ndarray:
    """The sparse-tap channel of Section II: within an L-tap CIR, lnz taps at
    positions drawn uniformly without replacement, each CN(0, p) with
    p = 1 / (n_tx * sqrt(lnz)), the others zero. shape = leading dims
    (e.g. [frames, R, T]); returns complex128 [*shape, L]. Draw order: the
    positions of every CIR, then real parts, then imaginary parts."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    keys = rng.random((n, L))
    pos = np.argsort(keys, axis=1)[:, :lnz]          # lnz distinct positions per CIR
    p = 1.0 / (n_tx * np.sqrt(lnz))
    vals = (rng.standard_normal((n, lnz)) + 1j * rng.standard_normal((n, lnz))) * np.sqrt(p / 2)
    h = np.zeros((n, L), dtype=np.complex128)
    np.put_along_axis(h, pos, vals, axis=1)
    return h.reshape(*shape, L)

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

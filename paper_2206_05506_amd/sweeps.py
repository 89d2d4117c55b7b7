"""Accuracy sweeps of Section IV on synthetic channels, run on the GPU.

MAE of Eq. 12 (mean |h_hat - h| over every tap of every (r, t) pair) against
SNR for the estimator's precisions, with and without the closed-form
least-squares rows:

  fig4: PN length M in {511, 2047}, multiplexed transmitters per pilot
        block N_batch in {1, 2, 4}, L = L_nz = 64, N_t = N_r = 16;
  fig5: M = 2047, N_batch = 4, L = 128, L_nz in {1, 4, 16, 64, 128}.

Each point averages `iters` realisations (Table I: 50). One realisation of an
N_t x N_r system sends N_t / N_batch multiplexed pilot blocks; each block is
one frame of the estimator with T = N_batch. Channels follow the sparse-tap
model of Section II (synth.sparse_taps). Frames are y = P h + sigma w built
by torch's FFT circular convolution with the plan's sequence (the receive
model of Eq. 9, outside the library), sigma per frame from the receive SNR.
Every estimate runs in libpnce's kernels; torch only composes the frames,
draws the noise and averages the errors.

Usage: python -m paper_2206_05506_amd.sweeps [--iters 50] [--out FILE.json]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from .api import Plan

SNRS = (-10, -5, 0, 5, 10, 15, 20, 25, 30)
N_T = N_R = 16
METHODS = ("fp32", "bf16", "f16", "e4m3", "fp32_ls", "bf16_ls")


def compose(plan: Plan, h: torch.Tensor, snr_db: float, gen: torch.Generator) -> torch.Tensor:
    """y = P h + sigma w on the device for channels h [F, R, K] (column k at
    the plan's lag k): the taps placed at their lags and circularly convolved
    with the plan's sequence by torch's FFT, w complex Gaussian of unit
    variance drawn from gen, sigma^2 = mean clean power / 10^(SNR/10) per
    frame. Returns complex64 [F, R, N]."""
    F, R, K = h.shape
    N = plan.N
    S = torch.fft.fft(torch.from_numpy(plan.sequence().astype(np.float64)).to(h.device)
                      .to(torch.complex128))
    lag = torch.from_numpy(plan.lags().astype(np.int64) % N).to(h.device)
    g = torch.zeros((F, R, N), dtype=torch.complex128, device=h.device)
    g.index_add_(2, lag, h.to(torch.complex128))
    y0 = torch.fft.ifft(torch.fft.fft(g, dim=-1) * S, dim=-1)
    p = (y0.abs() ** 2).mean(dim=(1, 2))
    sigma = torch.sqrt(p / 10.0 ** (snr_db / 10.0))
    w = torch.complex(torch.randn((F, R, N), generator=gen, device=h.device, dtype=torch.float64),
                      torch.randn((F, R, N), generator=gen, device=h.device, dtype=torch.float64))
    y = y0 + sigma[:, None, None] * w / np.sqrt(2.0)
    return y.to(torch.complex64).contiguous()


def estimates(plan: Plan, y: torch.Tensor) -> dict:
    """Every method's CIR stack [F, R, K] (complex64) from frames y."""
    est = {
        "fp32": plan.estimate(y, "f32s"),
        "bf16": plan.estimate(y, "bf16"),
        "fp32_ls": plan.estimate_ls(y, "f32s"),
        "bf16_ls": plan.estimate_ls(y, "bf16"),
    }
    for fmt in ("f16", "e4m3"):
        q, sc = plan.pack(y, fmt)
        est[fmt] = plan.estimate_packed(q, sc, fmt)
    return est


def mae_point(plan: Plan, y: torch.Tensor, h: torch.Tensor) -> dict:
    """Eq. 12's MAE of every method on frames y [F, R, N] of channels h [F, R, K]."""
    est = estimates(plan, y)
    return {m: float((est[m].to(torch.complex128) - h.to(torch.complex128)).abs().mean())
            for m in METHODS}


def _curve(M: int, nb: int, L: int, lnz: int, iters: int, seed: int) -> dict:
    import synth
    F = iters * (N_T // nb)
    h_np = synth.sparse_taps((F, N_R, nb), L, lnz, N_T, seed)
    h = torch.from_numpy(h_np.reshape(F, N_R, nb * L)).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    with Plan(M, nb, L, N_R) as plan:
        pts = {str(s): mae_point(plan, compose(plan, h, float(s), gen), h) for s in SNRS}
    return {"M": M, "N_batch": nb, "L": L, "L_nz": lnz, "frames": F, "mae": pts}


# (M, N_batch, L, L_nz) of every curve
FIG4_CURVES = [(M, nb, 64, 64) for M in (511, 2047) for nb in (1, 2, 4)]
FIG5_CURVES = [(2047, 4, 128, lnz) for lnz in (1, 4, 16, 64, 128)]
DEFAULT_ITERS = 50  # realisations per point (Table I)


def fig4(iters: int) -> list:
    return [_curve(M, nb, L, lnz, iters, 100 + 10 * nb + M % 7) for M, nb, L, lnz in FIG4_CURVES]


def fig5(iters: int) -> list:
    return [_curve(M, nb, L, lnz, iters, 200 + lnz) for M, nb, L, lnz in FIG5_CURVES]


def table(curves: list, label) -> str:
    """Markdown: one row per (curve, method), one column per SNR."""
    head = "| " + " | ".join(["curve", "method"] + [f"{s} dB" for s in SNRS]) + " |"
    sep = "|" + "---|" * (len(SNRS) + 2)
    rows = [head, sep]
    for c in curves:
        for m in METHODS:
            vals = [f"{c['mae'][str(s)][m]:.2e}" for s in SNRS]
            rows.append("| " + " | ".join([label(c), m] + vals) + " |")
    return "\n".join(rows)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--iters", type=int, default=DEFAULT_ITERS)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    res = {"fig4": fig4(args.iters), "fig5": fig5(args.iters), "iters": args.iters,
           "snr_db": list(SNRS), "methods": list(METHODS)}
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text, flush=True)
    print(table(res["fig4"], lambda c: f"M={c['M']} Nb={c['N_batch']}"), file=sys.stderr)
    print(table(res["fig5"], lambda c: f"Lnz={c['L_nz']}"), file=sys.stderr)


if __name__ == "__main__":
    main()

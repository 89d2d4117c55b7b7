"""Least-squares CIRs in closed form (pnce_debias, pnce_estimate_ls).

From the two-level autocorrelation (Eq. 1), P^T P = (N+1) I - J, so the LS
solution is N/(N+1) (H + sum(H)/(N+1-K)) per row of correlator outputs H.
Checked against the oracle's closed form (itself pinned to numpy.linalg.lstsq
on the CPU) within 1e-5, and by exact recovery of noiseless channels: the
correlator alone leaves the -sum(h)/N bias, the LS rows remove it.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import bf16_round, dev, frames, host, perr

pytestmark = pytest.mark.gpu

# fused epilogue (one column group), two-launch fallback (one frame: narrow
# tiles; K > 512), ragged R, tiny shapes
SHAPES = [
    (31, 2, 4, 3, 2),
    (127, 4, 16, 16, 1),
    (255, 4, 32, 40, 3),
    (1023, 16, 32, 64, 256),
    (2047, 16, 64, 32, 1),
    (4095, 32, 64, 8, 2),
]


def _plan(N, T, L, R):
    from paper_2206_05506_amd import Plan
    return Plan(N, T, L, R)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "N%d_T%d_L%d_R%d_B%d" % s)
@pytest.mark.parametrize("prec", ["f32s", "bf16", "f32"])
def test_estimate_ls_matches_oracle_closed_form(shape, prec):
    N, T, L, R, B = shape
    K = T * L
    y = synth.gaussian((B, R, N), N + R).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        yd = dev(y)
        X = p.estimate_ls(yd, prec)
        H = p.estimate(yd, prec)
        p.debias(H)
        Xh, Hh = host(X), host(H)
    pick = list(range(B)) if B <= 8 else [0, 77, B - 1]
    x = bf16_round(y[pick]) if prec == "bf16" else y[pick].astype(np.complex128)
    ref = oracle.ls_closed_form(oracle.correlate(x, s, K), N)
    assert perr(Xh[pick], ref) <= 1e-5
    assert perr(Hh[pick], ref) <= 1e-5


def test_noiseless_channels_are_recovered():
    """y = P h exactly: the correlator is off by the -sum(h)/N bias, the LS
    rows recover h to FP32 rounding."""
    cfg = synth.Config("ls", 10, 16, 32, 64, 4, 8.0, 0.0, 20.0, 11)
    d = synth.batch_draws(cfg)
    s = oracle.mseq(cfg.d)
    y, _ = oracle.received(s, d["h"], np.zeros_like(d["w"]), np.full(cfg.B, 300.0))
    h = d["h"].reshape(cfg.B, cfg.R, cfg.K)
    with _plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
        yd = dev(y.astype(np.complex64))
        H = host(p.estimate(yd, "f32s"))
        X = host(p.estimate_ls(yd, "f32s"))
    bias = perr(H, h)
    err = perr(X, h)
    print(f"correlator vs h {bias:.2e}, least squares vs h {err:.2e}")
    assert bias > 1e-3          # the -sum(h)/N floor of the plain correlator
    assert err <= 2e-6


def test_lag_alias_is_refused():
    from paper_2206_05506_amd import PnceError
    N, T, L, R = 63, 5, 16, 4    # T*L = 80 > N
    with _plan(N, T, L, R) as p:
        y = dev(synth.gaussian((1, R, N), 1).astype(np.complex64))
        with pytest.raises(PnceError):
            p.estimate_ls(y, "f32s")
        H = p.estimate(y, "f32s")
        with pytest.raises(PnceError):
            p.debias(H)

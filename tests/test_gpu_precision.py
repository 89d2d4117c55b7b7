"""Precision form on the full precision-study workload (N=4095, T=32, L=64,
R=256, 512 frames): Y stored as bf16 / f16 / e4m3 with a per-frame scale,
correlated with FP32 accumulation, then FP32 least-squares refinement.

Checked against the FP64 oracle on sampled (frame, antenna) rows: the oracle
iterate with the same step count k, started from the FP64 correlation of the
original complex64 frame. The quantiser's codes and scales of the first and
last frames are bit-exact, and the packed estimates of their sampled rows
match the oracle's correlation of the same dequantised codes (<= 1e-5).
Bars: FP32-accurate correlation <= 1e-5; bf16 and f16 + refinement <= 1e-5
after 5 steps; every format's error shrinks
monotonically for the first steps. NMSE of the bf16 estimate (no refinement)
against the true channels within 0.05 dB of the FP32-accurate estimate.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import device_frames, host, perr

pytestmark = pytest.mark.gpu

ROWS = [(0, 0), (0, 255), (97, 17), (255, 128), (400, 3), (511, 255)]


def _rows(x):
    return np.stack([host(x[b, r]) for b, r in ROWS])[:, None, :]


def _nmse_db(H, h):
    B = h.shape[0]
    hs = h.reshape(H.shape)
    e = ((H - hs).abs() ** 2).reshape(B, -1).sum(1).double()
    p = (hs.abs() ** 2).reshape(B, -1).sum(1).double()
    return float(10.0 * torch.log10((e / p).mean()))


def test_precision_study_full_workload():
    from paper_2206_05506_amd import Plan
    cfg = synth.PRECISION
    s = oracle.mseq(cfg.d)
    y, h = device_frames(cfg, s)
    with Plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
        assert np.array_equal(p.sequence(), s)
        yr = _rows(y).astype(np.complex128)
        its = oracle.refine(yr, s, cfg.K, 5)

        H32 = p.estimate(y, "f32s")
        e32 = perr(_rows(H32), its[0])
        print(f"f32s correlation relerr {e32:.2e}")
        assert e32 <= 1e-5

        work = torch.empty_like(y)
        report = {}
        nmse = {"f32s": _nmse_db(H32, h)}
        for fmt in ("bf16", "f16", "e4m3"):
            q, sc = p.pack(y, fmt)
            X0 = p.estimate_packed(q, sc, fmt)
            nmse[fmt] = _nmse_db(X0, h)
            # the launches the benchmark times, at full size: codes and
            # scales of the first and last frames bit-exact, and the packed
            # correlation of their sampled rows against the oracle's
            # correlation of the same dequantised codes
            for b in (0, cfg.B - 1):
                ref_q, ref_s = oracle.quantize(host(y[b:b + 1]), fmt)
                assert np.array_equal(host(sc[b:b + 1]), ref_s), (fmt, b)
                assert np.array_equal(host(q[b:b + 1]).view(ref_q.dtype), ref_q), (fmt, b)
                x = oracle.dequantize(ref_q, ref_s, fmt, cfg.N)
                for bb, r in ROWS:
                    if bb == b:
                        got = host(X0[b, r])[None, None]
                        assert perr(got, oracle.correlate(x[:, r:r + 1], s, cfg.K)) <= 1e-5
            errs = []
            for k in range(6):
                X = X0.clone()
                p.refine(y, X, k, work=work)
                errs.append(perr(_rows(X), its[k]))
            report[fmt] = errs
            del q, X0, X
        torch.cuda.synchronize()
    for fmt, errs in report.items():
        print(fmt, " ".join(f"{e:.2e}" for e in errs), f"nmse {nmse[fmt]:.3f} dB")
    print(f"f32s nmse {nmse['f32s']:.3f} dB")
    assert report["bf16"][5] <= 1e-5
    assert report["f16"][5] <= 1e-5
    for errs in report.values():
        assert errs[1] < errs[0] and errs[2] < errs[1]
    assert abs(nmse["bf16"] - nmse["f32s"]) <= 0.05
    assert abs(nmse["f16"] - nmse["f32s"]) <= 0.05

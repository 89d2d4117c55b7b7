"""Benchmark: CIR estimates per second of PN-correlation channel estimation on
one MI355X, BF16 matrix-core path against the FP32 paths at matched NMSE, plus
p50 single-frame latency.

Headline workload (precision study): N = 4095 (degree-12 m-sequence), T = 32
multiplexed transmitters, L = 64 taps (T*L = 2048 lags), R = 256 antennas,
512 frames, exponential power-delay profile (decay 8 taps), SNR uniform in
[-5, 25] dB per frame. Synthetic frames: seeded draws (synth) composed into
y = P h + noise by torch's FFT circular convolution (no library kernel), then
stored as bf16 codes with a per-frame power-of-two scale.

A timed step is one estimation pass over the 512 frames resident in HBM:
  pnce_estimate_packed(format=BF16) -- bf16 codes read once, +-1 operand
  expanded on chip, bf16 matrix cores, FP32 accumulation, c64 CIRs written.
The conversion of the complex64 frames into stored bf16 codes is not inside
the step (the frames are held as bf16, as the workload states); it is timed
beside it, and so is the variant that reads the complex64 frames and rounds
them in registers. The FP32-accurate (3-way bf16 split) and FP32-matrix
paths are timed on the same complex64 frames, each with its NMSE against the
true channels.

Besides the headline the line carries the FP32-baseline workload (N = 1023,
T*L = 512, R = 64, 256 frames: the HBM-bound shape), timings of every other
form of the path (adjoint, refinement, least squares, Eq. 8 lags, the
4096-frame uneven batch, the front end) and the differentiation workload
(N = 1023, T*L = 1024, R = 128, 1024 frames: forward + backward through
autograd), and the frame latencies of Figs. 6 and 7 (copies from and to pinned
host memory included) beside the pilot airtime of Eq. 11.

Prints one JSON line (rank 0). Usage:
  python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--no-cpu] [--no-rows]
                  [--no-workloads]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
ROTATE_COPIES = 5              # frame / CIR buffer copies the FP32-baseline steps rotate over

# HBM bytes per launch of the headline kernel measured with rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE (scaled by a plain copy of known size), valid only
# for the kernel source with this sha256; any other source reports null.
TRAFFIC = {"source_sha256": "f0338a9c6819640b641b336567326292ecd7793258f3482507f49e88f7b7bbfe",
           "bytes_per_launch": 4295642035}
BF16_PEAK_TFLOPS = 2516.6      # dense bf16 / f16 matrix
FP8_PEAK_TFLOPS = 5033.2       # dense fp8 matrix
FP32_PEAK_TFLOPS = 157.3       # dense fp32 matrix
FP64_PEAK_TFLOPS = 78.6        # dense fp64 matrix
INT8_PEAK_TOPS = 5033.2         # dense int8 matrix


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--latency-iters", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only 3 headline launches (packed bf16 estimate, 512 precision-study "
                         "frames) and 3 plain copies of the code buffer, for rocprofv3 --pmc "
                         "byte counters and their copy-kernel calibration")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="only 3 launches each of the matrix-bound kernels (the headline "
                         "packed bf16 estimate on all 512 precision-study frames, the e4m3 one, "
                         "the FP32-accurate estimate of the same frames), for rocprofv3 --pmc "
                         "counters of matrix-core activity")
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="only 3 launches each of the FP32-accurate adjoint on the FP32-baseline "
                         "shape (256 frames, T*L=512 -> N=1023) and on the differentiation shape "
                         "(1024 frames, T*L=1024 -> N=1023), and of the FP32-accurate estimate of "
                         "the FP32-baseline shape, for rocprofv3 counters")
    ap.add_argument("--exact-probe", action="store_true",
                    help="only 3 launches each of the refinement residual r = y - P x on "
                         "the 512 precision-study frames with exact sums (eight int8 digits), "
                         "FP64 sums (FP64 matrix cores), four int8 digits and the bf16 split, "
                         "for rocprofv3 counters")
    ap.add_argument("--varlen-probe", action="store_true",
                    help="only 3 persistent launches of the 4096-frame uneven batch (default "
                         "schedule) and 3 plain copies of its code buffer, for rocprofv3 counters")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the adjoint/refinement/uneven-batch/front-end timings")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the FP32-baseline and differentiation workloads")
    return ap.parse_args()


def measured_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2206_05506_amd", "csrc", "pnce_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return TRAFFIC["bytes_per_launch"] if sha == TRAFFIC["source_sha256"] else None


def compose(plan, h, w, snr_db, torch, chunk=32):
    """y = P h + sigma w on the GPU without the library: the stacked taps
    (column k of H at the plan's lag k) circularly convolved with the plan's
    sequence by torch's FFT (the receive model of Eq. 9), noise scaled per
    frame to the drawn receive SNR (sigma^2 = mean clean power / 10^(SNR/10)).
    h [F, R, K], w [F, R, N] complex64 and snr_db [F] on the device."""
    F, R, K = h.shape
    N = plan.N
    S = torch.fft.fft(torch.from_numpy(plan.sequence().astype(np.float32)).cuda()
                      .to(torch.complex64))
    lag = torch.from_numpy(plan.lags().astype(np.int64) % N).cuda()
    y = torch.empty((F, R, N), dtype=torch.complex64, device="cuda")
    for f0 in range(0, F, chunk):
        f1 = min(F, f0 + chunk)
        g = torch.zeros((f1 - f0, R, N), dtype=torch.complex64, device="cuda")
        g.index_add_(2, lag, h[f0:f1])
        yc = torch.fft.ifft(torch.fft.fft(g, dim=-1) * S, dim=-1)
        p = (yc.abs() ** 2).mean(dim=(1, 2)).double()
        sigma = torch.sqrt(p / 10.0 ** (snr_db[f0:f1].double() / 10.0)).float()
        y[f0:f1] = yc + sigma[:, None, None] * w[f0:f1]
        del g, yc
    torch.cuda.synchronize()
    return y


def make_inputs(plan, cfg, torch):
    """Seeded host draws of every frame of cfg, composed on the GPU."""
    import synth
    d = synth.batch_draws(cfg)
    h = torch.from_numpy(d["h"].reshape(cfg.B, cfg.R, cfg.K)).to(torch.complex64).cuda()
    w = torch.from_numpy(d["w"]).to(torch.complex64).cuda()
    snr = torch.from_numpy(d["snr_db"]).cuda()
    y = compose(plan, h, w, snr, torch)
    del w
    return y, h


def make_device_inputs(plan, cfg, torch, frames=None):
    """Seeded device draws (the precision study's 537 M samples are drawn on
    the GPU), composed on the GPU."""
    import synth
    d = synth.device_draws(cfg, torch, frames=frames)
    F = d["h"].shape[0]
    h = d["h"].reshape(F, cfg.R, cfg.K)
    y = compose(plan, h, d["w"], d["snr_db"], torch)
    del d
    return y, h.contiguous()


def nmse_db(H, h):
    B = h.shape[0]
    e = ((H - h).abs() ** 2).reshape(B, -1).sum(1).double()
    p = (h.abs() ** 2).reshape(B, -1).sum(1).double()
    return float(10.0 * np.log10((e / p).mean().item()))


def spin_up(fn, seconds, torch):
    """Untimed: keep the GPU busy with the step itself for `seconds` so that
    its clocks have left the idle state before warm-up and timing (a few
    dozen microsecond launches alone do not get them there)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            fn()
        torch.cuda.synchronize()


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3


def p50_latency_us(fn, iters, torch):
    st = torch.cuda.current_stream()
    for _ in range(10):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(iters):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fn()
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e3)
    return statistics.median(ts)


def p50_wall_us(fn, iters, torch):
    """Median host wall-clock time of fn followed by a device synchronize:
    the latency a host thread sees, enqueue and completion signal included."""
    for _ in range(10):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(iters):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e6)
    return statistics.median(ts)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _elementwise(x, ref):
    """max over frames of max|x - ref| / max|ref| (frame = leading axis)."""
    B = ref.shape[0]
    d = np.abs(x - ref).reshape(B, -1).max(axis=1)
    m = np.abs(ref).reshape(B, -1).max(axis=1)
    return float(np.max(d / np.where(m == 0, 1.0, m)))


def cpu_baseline(plan, cfg, y_dev, q_dev, sc_dev, H_dev, target_s, torch):
    """The FP64 oracle on the host's cores (OpenMP) over a bounded sample of
    the headline frames: whole passes over the first n complex64 frames,
    repeated until at least target_s seconds of work (one pass is at most
    about target_s), then one frame on one thread. The same leg checks the
    timed output against the oracle on a few of those frames (the correlation
    of the dequantised bf16 codes), and the refinement iterates from each
    packed start against the oracle's FP64 iterates with the same step count.
    Returns the cpu_baseline object of the JSON line."""
    import oracle
    s = oracle.mseq(cfg.d)
    if not np.array_equal(s, plan.sequence()):
        raise RuntimeError("library sequence differs from the oracle's")
    K = cfg.K
    y1 = y_dev[:1].cpu().numpy()
    oracle.correlate(y1, s, K)                               # warm-up (threads, pages)
    t0 = time.perf_counter()
    oracle.correlate(y1, s, K)
    per_frame = time.perf_counter() - t0
    n = int(max(1, min(cfg.B, round(target_s / max(per_frame, 1e-4)))))
    y = y_dev[:n].cpu().numpy()
    reps = 0
    t0 = time.perf_counter()
    while True:                                  # whole passes until target_s is reached
        oracle.correlate(y, s, K)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= target_s:
            break
    t0 = time.perf_counter()
    oracle.correlate(y1, s, K, threads=1)
    dt1 = time.perf_counter() - t0

    # the headline output of the first frames against the oracle on the same codes
    nchk = min(4, cfg.B)
    ref = oracle.correlate(oracle.dequantize(q_dev[:nchk].cpu().numpy(),
                                             sc_dev[:nchk].cpu().numpy(), "bf16", cfg.N), s, K)
    got = H_dev[:nchk].cpu().numpy()
    check = {"frames": nchk, "relerr_max": oracle.relerr(got, ref),
             "elementwise_max": _elementwise(got, ref), "bound": 1e-5,
             "what": "headline CIRs of the first frames vs the FP64 oracle correlation of "
                     "the same dequantised bf16 codes (normwise per frame, and max|dH| / "
                     "max|H_ref| per frame)"}
    check["pass"] = bool(check["relerr_max"] <= 1e-5 and check["elementwise_max"] <= 1e-5)

    # refinement from each packed start against the oracle's FP64 iterates
    nacc = min(2, cfg.B)
    its = oracle.refine(y[:nacc].astype(np.complex128), s, K, 5)
    ya = y_dev[:nacc].contiguous()
    work = torch.empty_like(ya)
    acc = {"frames": nacc,
           "reference": "oracle FP64 iterate with the same k, from the FP64 correlation of "
                        "the same complex64 frames"}
    for fmt in ("bf16", "f16", "e4m3"):
        qa, sa = plan.pack(ya, fmt)
        x0 = plan.estimate_packed(qa, sa, fmt)
        rows = []
        for k in range(6):
            X = x0.clone()
            if k:
                plan.refine(ya, X, k, work=work)
            xh = X.cpu().numpy()
            rows.append({"k": k, "relerr_vs_fp64": oracle.relerr(xh, its[k]),
                         "elementwise_vs_fp64": _elementwise(xh, its[k])})
        acc[fmt] = rows
    del ya, work
    return {"value": reps * n * cfg.R * cfg.T / dt, "unit": "CIR estimates/s",
            "one_thread_value": cfg.R * cfg.T / dt1, "cpu_model": cpu_model(),
            "nproc": os.cpu_count(), "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{reps} pass(es) over {n} of {cfg.B} frames of the headline workload "
                      f"(N={cfg.N}, T*L={K}, R={cfg.R}), FP64 direct correlation of the "
                      f"complex64 frames, {dt:.1f} s; one-thread value from one frame",
            "oracle_check": check, "accuracy_vs_oracle_fp64": acc}


def headline(torch, args):
    """The precision-study workload: the timed step (packed bf16 estimate of
    512 frames), the other precisions on the same frames with their NMSE, the
    quantiser, refinement and one-frame latencies. Returns (line, ctx): the
    JSON fields of the headline and the tensors the CPU leg checks."""
    import synth
    from paper_2206_05506_amd import Plan
    cfg = synth.PRECISION
    B, R, N, K, T = cfg.B, cfg.R, cfg.N, cfg.K, cfg.T
    plan = Plan(N, T, cfg.L, R)
    y, h = make_device_inputs(plan, cfg, torch)
    q, sc = plan.pack(y, "bf16")
    H = torch.empty((B, R, K), dtype=torch.complex64, device="cuda")

    def step():
        plan.estimate_packed(q, sc, "bf16", out=H)

    spin_up(step, 0.3, torch)
    ms_bf, wall_bf = time_steps(step, args.steps, args.warmup, torch)
    nmse = {"bf16": nmse_db(H, h)}

    few = max(3, args.steps // 10)
    H2 = torch.empty_like(H)
    # the same estimate read straight from the complex64 frames (each sample
    # rounded to bf16 in registers; no stored copy, no scale)
    ms_c64, _ = time_steps(lambda: plan.estimate(y, "bf16", out=H2), few, 2, torch)
    nmse["bf16_from_c64"] = nmse_db(H2, h)
    # the conversion that produces the stored codes (Section III-B)
    # (pnce_pack_ws: every frame read from HBM once), and the two-pass
    # conversion without a workspace (a max pass, then a conversion pass)
    work = torch.empty((1024 * B + 1,), dtype=torch.int32, device="cuda")
    ms_pack, _ = time_steps(lambda: plan.pack(y, "bf16", out=q, scales=sc, work=work), few, 1,
                            torch)
    ms_pack2, _ = time_steps(lambda: plan.pack_two_pass(y, "bf16", out=q, scales=sc), few, 1,
                             torch)
    frame_b = B * R * N * 8
    code_b = q.numel() * q.element_size()
    formats = {}
    for fmt, peak in (("f16", BF16_PEAK_TFLOPS), ("e4m3", FP8_PEAK_TFLOPS)):
        qf, sf = plan.pack(y, fmt)
        ms_p, _ = time_steps(lambda: plan.pack(y, fmt, out=qf, scales=sf, work=work), few, 1,
                             torch)
        ms_e, _ = time_steps(lambda: plan.estimate_packed(qf, sf, fmt, out=H2), few, 1, torch)
        nmse[fmt] = nmse_db(H2, h)
        cb = qf.numel() * qf.element_size()
        formats[fmt] = {"estimate_ms": ms_e, "CIR/s": B * R * T / (ms_e * 1e-3),
                        "mfma_frac": 4.0 * B * R * N * K / ms_e / 1e9 / peak,
                        "pack_ms": ms_p, "pack_GB/s": (frame_b + cb) / ms_p / 1e6,
                        "pack_hbm_frac": (frame_b + cb) / ms_p / 1e6 / HBM_PEAK_GBS}
        del qf, sf
    ms_32, _ = time_steps(lambda: plan.estimate(y, "f32s", out=H2), few, 2, torch)
    nmse["fp32_accurate"] = nmse_db(H2, h)
    ms_x32, _ = time_steps(lambda: plan.estimate(y, "exact32", out=H2), few, 2, torch)
    nmse["fp32_int8_digits"] = nmse_db(H2, h)
    ms_mf, _ = time_steps(lambda: plan.estimate(y, "f32", out=H2), 3, 1, torch)
    nmse["fp32_mfma"] = nmse_db(H2, h)

    # least-squares refinement from the bf16 estimate (original c64 frames)
    work = torch.empty_like(y)
    X = H.clone()
    ref_ms = {}
    for k in (1, 2, 5):
        ref_ms[k], _ = time_steps(lambda: plan.refine(y, X, k, work=work), 2, 1, torch)
    # its residual r = y - P x: the last step's both ways, exact sums on int8
    # digits (the one refinement runs) and FP64 sums on the FP64 matrix
    # cores; the inner steps' on four int8 digits (the one refinement runs)
    # and as the FP32-accurate bf16 split
    resid = {}
    for prec in ("exact", "f64acc", "exact32", "f32s"):
        resid[prec], _ = time_steps(
            lambda: plan.adjoint(X, prec, alpha=-1.0, beta=1.0, C=y, out=work), 2, 1, torch)
    del X, work, H2
    torch.cuda.empty_cache()

    # one frame: kernel-only p50 latency, and with the frame's copy from
    # pinned host memory (the paper's latency includes the transfer)
    lat = {}
    if args.latency_iters > 0:
        y1, q1, s1 = y[:1].contiguous(), q[:1].contiguous(), sc[:1].contiguous()
        H1 = torch.empty((1, R, K), dtype=torch.complex64, device="cuda")
        it = args.latency_iters
        lat["bf16"] = p50_latency_us(lambda: plan.estimate_packed(q1, s1, "bf16", out=H1), it,
                                     torch)
        lat["bf16_from_c64"] = p50_latency_us(lambda: plan.estimate(y1, "bf16", out=H1), it,
                                              torch)
        lat["fp32_accurate"] = p50_latency_us(lambda: plan.estimate(y1, "f32s", out=H1), it,
                                              torch)
        q1h = torch.empty(q1.shape, dtype=q1.dtype, pin_memory=True)
        q1h.copy_(q1.cpu())
        q1d = torch.empty_like(q1)
        y1h = torch.empty(y1.shape, dtype=y1.dtype, pin_memory=True)
        y1h.copy_(y1.cpu())
        y1d = torch.empty_like(y1)

        def codes_in():
            q1d.copy_(q1h, non_blocking=True)
            plan.estimate_packed(q1d, s1, "bf16", out=H1)

        def c64_in():
            y1d.copy_(y1h, non_blocking=True)
            plan.estimate(y1d, "bf16", out=H1)

        lat["bf16_with_h2d_copy_of_codes"] = p50_latency_us(codes_in, it, torch)
        lat["bf16_from_c64_with_h2d_copy"] = p50_latency_us(c64_in, it, torch)
        pc = synth.PLAIN
        pp = Plan(pc.N, pc.T, pc.L, pc.R)
        yp = _randn_c64((1, pc.R, pc.N), 13, torch)
        Hp = torch.empty((1, pc.R, pc.K), dtype=torch.complex64, device="cuda")
        lat["plain_workload"] = {prec: p50_latency_us(lambda: pp.estimate(yp, prec, out=Hp), it,
                                                      torch) for prec in ("bf16", "f32s")}
        pp.close()
        del y1h, q1h, y1d, q1d, H1

    cirs = B * R * T
    flops = 4.0 * B * R * N * K
    out_b = B * R * K * 8
    ach = flops / (ms_bf * 1e-3) / 1e12
    line = {
        "metric": "CIR estimates/s + p50 frame latency; BF16-MFMA vs FP32 at matched NMSE",
        "value": cirs / (ms_bf * 1e-3),
        "frames_per_s": B / (ms_bf * 1e-3),
        "unit": "CIR estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_bf,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded device draws; y = P h + noise by torch FFT circular "
                "convolution; stored as bf16 codes with a per-frame power-of-two scale)",
        "config": {"workload": cfg.name, "N": N, "T": T, "L": cfg.L, "R": R, "frames": B,
                   "input": "bf16 codes [B][R][2][N+1] + per-frame scale, resident in HBM",
                   "snr_db": [cfg.snr_lo, cfg.snr_hi],
                   "step": "one pnce_estimate_packed(bf16) launch over all frames; the "
                           "conversion to bf16 codes is not in the step (timed in "
                           "pack_bf16_ms)"},
        "p50_frame_latency_us": lat,
        "fp32_path": {"value": cirs / (ms_32 * 1e-3), "ms_per_step": ms_32,
                      "precision": "f32s: FP32-accurate, each FP32 sample split exactly into "
                                   "three bf16 parts, three bf16 matrix-core products",
                      "input": "complex64 frames"},
        "fp32_int8_digits_path": {"value": cirs / (ms_x32 * 1e-3), "ms_per_step": ms_x32,
                                  "precision": "exact32: each FP32 row in 30-bit fixed point, "
                                               "four int8 digits, exact int32 sums, FP32 "
                                               "epilogue (no FP64); the fastest FP32-class path",
                                  "input": "complex64 frames"},
        "fp32_mfma_path": {"value": cirs / (ms_mf * 1e-3), "ms_per_step": ms_mf,
                           "precision": "f32: v_mfma_f32_32x32x2_f32",
                           "mfma_frac": flops / ms_mf / 1e9 / FP32_PEAK_TFLOPS},
        "bf16_speedup_vs_fp32": {"fp32_accurate": ms_32 / ms_bf, "fp32_mfma": ms_mf / ms_bf,
                                 "fp32_int8_digits": ms_x32 / ms_bf,
                                 "delta_nmse_db_vs_fp32_accurate":
                                     nmse["bf16"] - nmse["fp32_accurate"],
                                 "matched_nmse": abs(nmse["bf16"] - nmse["fp32_accurate"])
                                 <= 0.05,
                                 "note": "same frames; matched NMSE = within 0.05 dB"},
        "nmse_db": nmse,
        "bf16_from_c64": {"ms_per_step": ms_c64, "CIR/s": cirs / (ms_c64 * 1e-3),
                          "mfma_frac": flops / ms_c64 / 1e9 / BF16_PEAK_TFLOPS,
                          "note": "pnce_estimate(bf16) on the complex64 frames: each sample "
                                  "rounded to bf16 in registers, no stored copy"},
        "pack_bf16_ms": ms_pack,
        "pack_bf16_GB/s": (frame_b + code_b) / ms_pack / 1e6,
        "pack_bf16_hbm_frac": (frame_b + code_b) / ms_pack / 1e6 / HBM_PEAK_GBS,
        "pack_bf16_two_pass_ms": ms_pack2,
        "pack_plus_estimate_ms": ms_pack + ms_bf,
        "other_formats": formats,
        "refine_ms": {f"{k}_steps": v for k, v in ref_ms.items()},
        "final_residual_ms": {
            "exact_int8_digits": resid["exact"], "fp64_matrix_cores": resid["f64acc"],
            "speedup": resid["f64acc"] / resid["exact"],
            "int8_frac": 8.0 * flops / resid["exact"] / 1e9 / INT8_PEAK_TOPS,
            "fp64_frac": flops / resid["f64acc"] / 1e9 / FP64_PEAK_TFLOPS,
            "note": "r = y - P x over all frames; exact: every value in 62-bit fixed point "
                    "cut into eight int8 digits, exact int32 sums on v_mfma_i32_32x32x32_i8 "
                    "(8x the contraction's operations), result correctly rounded to FP32"},
        "inner_residual_ms": {
            "four_int8_digits": resid["exact32"], "bf16_split": resid["f32s"],
            "speedup": resid["f32s"] / resid["exact32"],
            "int8_frac": 4.0 * flops / resid["exact32"] / 1e9 / INT8_PEAK_TOPS,
            "note": "r = y - P x of the inner refinement steps: four int8 digits of a 30-bit "
                    "fixed-point value (exact to 2^-30 of each row's largest element, then an "
                    "FP32 epilogue; no FP64) against three bf16 parts with FP32 accumulation"},
        "bf16_plus_2_refine_steps": {
            "ms": ms_bf + ref_ms[2], "CIR/s": cirs / ((ms_bf + ref_ms[2]) * 1e-3),
            "note": "bf16 estimate then 2 refinement steps (sums on four int8 digits, the "
                    "last residual exact): within 1e-5 of the FP64 iterate "
                    "(accuracy_vs_oracle_fp64)"},
        "wall_ms_per_step": wall_bf,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / BF16_PEAK_TFLOPS,
                     "traffic": measured_traffic(),
                     "kernel": "tg_kernel<BF16, bf16 codes, NC=4>",
                     "flops_per_launch": flops,
                     "algorithmic_bytes_per_launch": code_b + out_b,
                     "hbm_GB/s": (code_b + out_b) / (ms_bf * 1e-3) / 1e9},
    }
    ctx = {"plan": plan, "cfg": cfg, "y": y, "q": q, "sc": sc, "H": H}
    del h
    return line, ctx


def other_rows(plan, cfg, y, H, torch, args):
    """Timings of the other forms of the path on the same frames (and, for
    the uneven batch, on its own 4096-frame workload)."""
    B, R, N, K = cfg.B, cfg.R, cfg.N, cfg.K
    res = {}
    q = torch.empty((B, R, 2, N + 1), dtype=torch.int16, device="cuda")
    sc = torch.empty((B,), dtype=torch.float32, device="cuda")
    ms, _ = time_steps(lambda: plan.pack(y, "bf16", out=q, scales=sc), args.steps, 2, torch)
    byt = B * R * N * 8 + B * R * 2 * (N + 1) * 2
    res["pack_bf16"] = {"ms": ms, "GB/s": byt / ms / 1e6,
                        "note": "algorithmic bytes (frames read once, codes written once); one "
                                "launch, a workgroup per frame, whose second read of the frame "
                                "is served by the Infinity Cache"}
    Hq = torch.empty_like(H)
    ms, _ = time_steps(lambda: plan.estimate_packed(q, sc, "bf16", out=Hq), args.steps, 2, torch)
    byt = B * R * 2 * (N + 1) * 2 + B * R * K * 8
    res["estimate_packed_bf16"] = {"ms": ms, "GB/s": byt / ms / 1e6}
    A = torch.empty_like(y)
    ms, _ = time_steps(lambda: plan.adjoint(H, "f32s", out=A), args.steps, 2, torch)
    res["adjoint_f32s"] = {"ms": ms, "TFLOP/s": 4.0 * B * R * N * K / ms / 1e9}
    Hls = torch.empty_like(H)
    ms_f, _ = time_steps(lambda: plan.estimate_ls(y, "bf16", out=Hls), args.steps, 2, torch)
    ms_d, _ = time_steps(lambda: plan.debias(Hls), args.steps, 2, torch)
    res["least_squares"] = {"estimate_ls_bf16_ms": ms_f, "debias_ms": ms_d,
                            "debias_GB/s": 2 * B * R * K * 8 / ms_d / 1e6,
                            "note": "closed-form LS rows: fused into the correlator epilogue "
                                    "(one column group per row here); debias alone reads and "
                                    "writes the CIRs"}
    del Hls
    X = H.clone()
    work = torch.empty_like(y)
    ms, _ = time_steps(lambda: plan.refine(y, X, 1, work=work), max(2, args.steps // 4), 1, torch)
    res["refine_1_step"] = {"ms": ms, "note": "exact-sum residual + four-digit (exact32) correlation"}
    del q, Hq, A, X, work
    res["eq8_lags"] = eq8_lags(cfg, y, H, res, torch, args)
    res["uneven_batch"] = uneven_batch(torch, args)
    res["frames_per_launch"] = frames_per_launch(plan, cfg, torch)
    return res


def frames_per_launch(plan, cfg, torch):
    """The same bf16 estimate with 16 to 4096 frames per launch, frames
    rotated over buffers of at least 1 GB in total (streamed from HBM): time
    per launch and the fraction of the 8 TB/s HBM peak reached. A launch of
    256 frames is one round of tiles (two per CU) whose start and end phases
    overlap nothing; longer launches overlap them with other tiles' streaming."""
    R, N, K = cfg.R, cfg.N, cfg.K
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    out = {}
    for B in (16, 64, 256, 1024, 4096):
        per = B * R * N * 8
        nrot = max(2, min(64, (1 << 30) // per + 1))
        ys = [torch.complex(torch.randn((B, R, N), generator=g, device="cuda"),
                            torch.randn((B, R, N), generator=g, device="cuda")).contiguous()
              for _ in range(nrot)]
        Hs = [torch.empty((B, R, K), dtype=torch.complex64, device="cuda") for _ in range(nrot)]
        c = [0]

        def step():
            c[0] = (c[0] + 1) % nrot
            plan.estimate(ys[c[0]], "bf16", out=Hs[c[0]])

        ms, _ = time_steps(step, 200 if B < 256 else 50, 10, torch)
        gbs = B * R * (N + K) * 8 / ms / 1e6
        out[str(B)] = {"us_per_launch": ms * 1e3, "CIR/s": B * R * cfg.T / (ms * 1e-3),
                       "GB/s": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
        del ys, Hs
        torch.cuda.empty_cache()
    return out


def eq8_lags(cfg, y, H, res, torch, args):
    """The same frames on a plan with Eq. 8's lags (transmitter t at
    floor(N/T)*t) and another cell's m-sequence: correlator, LS rows and
    adjoint, against the adjacent-lag plan's rows above."""
    from paper_2206_05506_amd import Plan
    d = cfg.d
    fb = next(m for m in range((1 << d) - 1, 0, -1)
              if m & 1 and _is_primitive(d, m))
    p8 = Plan(cfg.N, cfg.T, cfg.L, cfg.R, feedback=fb, spacing="eq8")
    Hb = torch.empty_like(H)
    ms_b, _ = time_steps(lambda: p8.estimate(y, "bf16", out=Hb), args.steps, 2, torch)
    ms_l, _ = time_steps(lambda: p8.estimate_ls(y, "bf16", out=Hb), args.steps, 2, torch)
    A = torch.empty_like(y)
    ms_a, _ = time_steps(lambda: p8.adjoint(H, "f32s", out=A), args.steps, 2, torch)
    lag = p8.lags()
    p8.close()
    del Hb, A
    return {"feedback": fb, "lag_step": int(lag[cfg.L]) if cfg.T > 1 else 0,
            "estimate_bf16_ms": ms_b, "estimate_ls_bf16_ms": ms_l, "adjoint_f32s_ms": ms_a,
            "adjoint_vs_adjacent": ms_a / res["adjoint_f32s"]["ms"],
            "note": "adjoint reduces over the lag span (T-1)*floor(N/T)+L with zeros in the "
                    "guard lags: same HBM bytes, more matrix work"}


def _is_primitive(d, mask):
    """Maximal-length test of a feedback mask (the LFSR state returns to its
    start after exactly 2^d - 1 steps), for choosing a cell's polynomial."""
    N = (1 << d) - 1
    w = 1
    for n in range(1, N + 1):
        fb = bin(w & mask).count("1") & 1
        w = (w >> 1) | (fb << (d - 1))
        if w == 1:
            return n == N
    return False


def _varlen_model_cost(N, K, nc):
    """The uneven batch's default cost model of one (frame, 32-antenna) unit
    at column width 128 * nc (streaming ~N samples plus matrix work over the
    padded lag width), used to schedule the fixed-width candidates."""
    w = 128 * nc
    groups = (K + w - 1) // w
    return N * (1.0 + groups * w / 256.0) * 1e-3


def uneven_batch(torch, args):
    """4096 frames of uneven (R, N, T, L) (seed 3), bf16 codes: one persistent
    launch, under the autotuned, the default and three fixed-width schedules
    (timed in interleaved rounds after a clock spin-up, so that clock drift
    hits every schedule alike), eager against a HIP graph replay (also
    interleaved), and against one launch per frame."""
    import synth
    from paper_2206_05506_amd import VarlenPlan
    shapes = [(int(R), (1 << int(d)) - 1, int(T), int(L))
              for R, d, T, L in synth.varlen_shapes(4096, 3)]
    vp = VarlenPlan(shapes)
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    Yq = torch.randn((vp.n_codes,), generator=g, device="cuda").to(torch.bfloat16)
    Yq = Yq.view(torch.int16).contiguous()
    H = torch.empty((vp.n_out,), dtype=torch.complex64, device="cuda")

    def step():
        vp.estimate(Yq, None, out=H)

    default = vp.tuning()
    spin_up(step, 0.3, torch)
    vp.tune(Yq, None, out=H, reps=3)
    tuned = vp.tuning()
    schedules = {"tuned": tuned, "default_model": default}
    for nc in (1, 2, 4):
        schedules[f"all_width_{128 * nc}"] = [(N, K, nc, _varlen_model_cost(N, K, nc))
                                              for N, K, _, _ in default]
    n_t = max(5, args.steps // 2)
    times = {k: [] for k in schedules}
    for _ in range(3):
        for k, sch in schedules.items():
            vp.set_tuning(sch)
            times[k].append(time_steps(step, n_t, 2, torch)[0])
    sched_ms = {k: statistics.median(v) for k, v in times.items()}
    vp.set_tuning(tuned)
    ms_p = sched_ms["tuned"]
    ms_e, _ = time_steps(lambda: vp.estimate_each(Yq, None, out=H), 3, 1, torch)
    # the persistent launch captured once in a HIP graph and replayed,
    # interleaved with eager launches of the same schedule
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    spin_up(step, 0.2, torch)
    eager_t, graph_t = [], []
    for _ in range(3):
        eager_t.append(time_steps(step, n_t, 2, torch)[0])
        graph_t.append(time_steps(graph.replay, n_t, 2, torch)[0])
    del graph
    cirs = sum(R * T for R, N, T, L in shapes)
    byt = vp.n_codes * 2 + vp.n_out * 8
    flops = sum(4.0 * R * N * T * L for R, N, T, L in shapes)
    # per frame the tighter of the two roofs: short-lag frames are bound by
    # HBM, long-lag ones (AI up to ~1000) by the matrix cores
    roof_us = sum(max((R * 2 * (N + 1) * 2 + R * T * L * 8) / (HBM_PEAK_GBS * 1e3),
                      4.0 * R * N * T * L / (BF16_PEAK_TFLOPS * 1e6))
                  for R, N, T, L in shapes)
    st = vp.stats()
    vp.close()
    return {"frames": len(shapes), "persistent_ms": ms_p,
            "untuned_ms": sched_ms["default_model"],
            "schedules_ms": sched_ms,
            "tuned_widths": sorted({(N, K, nc) for N, K, nc, _ in tuned}),
            "eager_ms_interleaved": statistics.median(eager_t),
            "graph_replay_ms": statistics.median(graph_t),
            "per_frame_launches_ms": ms_e,
            "speedup": ms_e / ms_p, "CIR/s": cirs / (ms_p * 1e-3),
            "GB/s": byt / ms_p / 1e6, "hbm_frac": byt / ms_p / 1e6 / HBM_PEAK_GBS,
            "mfma_frac": flops / ms_p / 1e9 / BF16_PEAK_TFLOPS,
            "per_frame_roofline_us": roof_us, "per_frame_roofline_frac": roof_us / (ms_p * 1e3),
            "workgroups": st["workgroups"], "tiles": st["tiles"],
            "note": "schedules_ms: medians of 3 interleaved rounds; tuned = the schedule "
                    "pnce_varlen_tune keeps (the fastest of five candidates timed end to end); "
                    "all_width_W: every class at W lags per tile, scheduled by the cost model"}


def _randn_c64(shape, seed, torch):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    re = torch.randn(shape, generator=g, device="cuda")
    im = torch.randn(shape, generator=g, device="cuda")
    return torch.complex(re, im).contiguous()


def fp32_baseline_workload(torch, args):
    """The FP32-baseline shape (N = 1023, T*L = 512, R = 64, 256 frames),
    HBM-bound for bf16 (AI 171 < ridge 315): the bf16 estimate with frames
    streamed from HBM (rotated buffers) and cache-resident, pipelined over two
    streams, the FP32 paths, p50 latency, and the other rows of the path on
    these frames."""
    import synth
    from paper_2206_05506_amd import Plan
    cfg = synth.FP32
    plan = Plan(cfg.N, cfg.T, cfg.L, cfg.R)
    y, h = make_inputs(plan, cfg, torch)
    H_bf = torch.empty((cfg.B, cfg.R, cfg.K), dtype=torch.complex64, device="cuda")
    H_32 = torch.empty_like(H_bf)
    H_mf = torch.empty_like(H_bf)

    # The 201 MB working set of one step fits in the 256 MB Infinity Cache, so
    # a step that re-reads the frames of the previous step is served partly
    # from that cache. Timed steps therefore rotate over ROT copies of the
    # frames and of the CIR buffers (ROT * 201 MB > 4x the cache): every step
    # streams its frames from HBM, as fresh frames would. The same data is in
    # every copy.
    n_rot = ROTATE_COPIES
    ys = [y] + [y.clone() for _ in range(n_rot - 1)]
    Hs = [H_bf] + [torch.empty_like(H_bf) for _ in range(n_rot - 1)]
    ctr = [0]

    def rot():
        ctr[0] = (ctr[0] + 1) % n_rot
        return ctr[0]

    def step(prec):
        i = rot()
        plan.estimate(ys[i], prec, out=Hs[i])

    spin_up(lambda: step("bf16"), 0.3, torch)
    ms_bf, _ = time_steps(lambda: step("bf16"), args.steps, args.warmup, torch)
    # context for the roofline: a plain device copy of the same frame buffers
    # (rotated likewise), read + write bytes over its time
    ms_cp, _ = time_steps(lambda: ys[rot()].copy_(ys[(ctr[0] + 2) % n_rot]), args.steps, 2, torch)
    ms_bf_cached, _ = time_steps(lambda: plan.estimate(y, "bf16", out=H_bf), args.steps,
                                 args.warmup, torch)
    ms_32, _ = time_steps(lambda: step("f32s"), args.steps, args.warmup, torch)
    H_32.copy_(Hs[ctr[0]])
    ms_mf, _ = time_steps(lambda: step("f32"), max(2, args.steps // 4), 2, torch)
    H_mf.copy_(Hs[ctr[0]])
    # Independent batches pipelined over two streams (default priority), as a
    # serving loop would issue them: step k runs on stream k % 2 with buffer
    # k % 6, so each buffer always belongs to the same stream and its reuse is
    # ordered. One launch's end phase then overlaps the next one's start.
    ys.append(y.clone())
    Hs.append(torch.empty_like(H_bf))
    pipe = [torch.cuda.Stream(), torch.cuda.Stream()]

    def pipelined(k0, n):
        for k in range(k0, k0 + n):
            with torch.cuda.stream(pipe[k % 2]):
                plan.estimate(ys[k % 6], "bf16", out=Hs[k % 6])

    cur = torch.cuda.current_stream()
    for st in pipe:
        st.wait_stream(cur)
    spin_up(lambda: pipelined(0, 2), 0.2, torch)
    pipelined(0, args.warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for st in pipe:
        st.wait_stream(cur)
    pipelined(args.warmup, args.steps)
    for st in pipe:
        cur.wait_stream(st)
    e1.record(cur)
    torch.cuda.synchronize()
    ms_pipe = e0.elapsed_time(e1) / args.steps
    plan.estimate(y, "bf16", out=H_bf)
    del ys, Hs

    lat = {}
    lat_h2d = None
    if args.latency_iters > 0:
        y1 = y[:1].contiguous()
        H1 = torch.empty((1, cfg.R, cfg.K), dtype=torch.complex64, device="cuda")
        lat["bf16"] = p50_latency_us(lambda: plan.estimate(y1, "bf16", out=H1),
                                     args.latency_iters, torch)
        lat["fp32_accurate"] = p50_latency_us(lambda: plan.estimate(y1, "f32s", out=H1),
                                              args.latency_iters, torch)
        y1_host = torch.empty(y1.shape, dtype=y1.dtype, pin_memory=True)
        y1_host.copy_(y1.cpu())
        y1_dev = torch.empty_like(y1)

        def h2d_then_estimate():
            y1_dev.copy_(y1_host, non_blocking=True)
            plan.estimate(y1_dev, "bf16", out=H1)

        lat_h2d = lat["bf16_with_h2d_copy"] = p50_latency_us(h2d_then_estimate,
                                                             args.latency_iters, torch)

    cirs = cfg.B * cfg.R * cfg.T
    bytes_ = cfg.B * (cfg.R * cfg.N * 8 + cfg.R * cfg.K * 8)
    ach_gbs = bytes_ / (ms_bf * 1e-3) / 1e9
    res = {
        "workload": cfg.name, "frames": cfg.B, "input": "complex64",
        "bf16_ms_per_step": ms_bf, "bf16_CIR/s": cirs / (ms_bf * 1e-3),
        "fp32_accurate_ms_per_step": ms_32, "fp32_mfma_ms_per_step": ms_mf,
        "bf16_speedup_vs_fp32": {"fp32_accurate": ms_32 / ms_bf, "fp32_mfma": ms_mf / ms_bf},
        "nmse_db": {"bf16": nmse_db(H_bf, h), "fp32_accurate": nmse_db(H_32, h),
                    "fp32_mfma": nmse_db(H_mf, h)},
        "p50_frame_latency_us": lat,
        "roofline_hbm": {"achieved_GB/s": ach_gbs, "peak_GB/s": HBM_PEAK_GBS,
                         "frac": ach_gbs / HBM_PEAK_GBS,
                         "kernel": "tg_kernel<BF16, c64 in, NC=4>",
                         "algorithmic_bytes_per_launch": bytes_},
        "timing": {"rotated_buffers": ROTATE_COPIES,
                   "note": "each timed step reads its own copy of the frames and writes its own "
                           "CIR buffer (5 x 201 MB > the 256 MB Infinity Cache), so frames stream "
                           "from HBM",
                   "cache_resident_ms_per_step": ms_bf_cached,
                   "hbm_copy_GB/s": 2 * y.numel() * 8 / (ms_cp * 1e-3) / 1e9},
        "pipelined_two_streams": {
            "ms_per_step": ms_pipe, "CIR/s": cirs / (ms_pipe * 1e-3),
            "hbm_frac": bytes_ / (ms_pipe * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "note": "the same steps issued alternately on two streams, as a serving loop "
                    "pipelines independent batches"},
    }
    if not args.no_rows:
        res["rows"] = other_rows(plan, cfg, y, H_32, torch, args)
        res["rows"]["front_end"] = front_end(plan, cfg, y, torch, lat_h2d, args)
    plan.close()
    del y, h, H_bf, H_32, H_mf
    torch.cuda.empty_cache()
    return res


def differentiation_workload(torch, args):
    """Differentiation shape (N=1023, T=16, L=64, R=128, 1024 frames): one
    forward correlation and its backward (adjoint) through autograd, then five
    least-squares refinement steps through autograd and through the library."""
    import synth
    from paper_2206_05506_amd import Plan
    from paper_2206_05506_amd.autograd import correlate, refine_by_gradient
    cfg = synth.DIFF
    B, R, N, K = cfg.B, cfg.R, cfg.N, cfg.K
    plan = Plan(N, cfg.T, cfg.L, R)
    y = _randn_c64((B, R, N), 22, torch).requires_grad_(True)
    G = _randn_c64((B, R, K), 23, torch)

    def fwd_bwd():
        H = correlate(y, plan, "f32s")
        (g,) = torch.autograd.grad(H, y, grad_outputs=G)
        return g

    ms, _ = time_steps(fwd_bwd, max(2, args.steps // 4), 1, torch)
    flops = 2 * 4.0 * B * R * N * K
    del G

    # Five least-squares refinement steps, once as gradient descent through
    # autograd (the loss and the update in torch, every product in the
    # library) and once as the library's own refinement entry point.
    y0 = y.detach()
    res = {}

    def by_autograd():
        res["xs"], res["losses"] = refine_by_gradient(y0, plan, 5, "f32s")

    X0 = plan.estimate(y0, "f32s")
    X = torch.empty_like(X0)
    work = torch.empty_like(y0)

    def by_library():
        X.copy_(X0)
        plan.refine(y0, X, 5, work)

    auto_ms, auto_wall = time_steps(by_autograd, 2, 1, torch)
    lib_ms, _ = time_steps(by_library, 3, 1, torch)
    x5 = res["xs"][-1]
    agree = float((torch.linalg.vector_norm(x5 - X) / torch.linalg.vector_norm(X)).item())
    l0 = res["losses"][0]
    out = {"workload": cfg.name, "frames": B, "forward_backward_ms": ms,
           "TFLOP/s": flops / ms / 1e9,
           "refine5_autograd_ms": auto_ms, "refine5_autograd_wall_ms": auto_wall,
           "refine5_library_ms": lib_ms,
           "refine5_loss_over_initial": [v / l0 for v in res["losses"]],
           "refine5_autograd_vs_library_relerr": agree,
           "note": "FP32-accurate forward and adjoint kernels; 3 bf16 matrix-core products "
                   "per term, so matrix-core rate = 3x the TFLOP/s shown. Refinement: 1 "
                   "correlation + 5 steps of (receive model, adjoint) plus the final loss; "
                   "the autograd run syncs once per step to read the loss"}
    plan.close()
    del y, y0, X0, X, work, res, x5
    torch.cuda.empty_cache()
    return out


def front_end(plan, cfg, y, torch, lat_h2d_us, args):
    """Raw blocks with a cyclic prefix of L samples in pinned host memory,
    streamed to the device in chunks (copies overlapped with estimation),
    against the pilot airtime of Eq. 11: T = (C + N) / Fs * N_t / N_batch,
    here one multiplexed block of the T transmitters (N_t = N_batch = T)."""
    cp = cfg.L
    B, R, N = cfg.B, cfg.R, cfg.N
    raw = torch.empty((B, R, cp + N), dtype=torch.complex64, device="cuda")
    raw[:, :, cp:] = y
    raw[:, :, :cp] = y[:, :, N - cp:]           # the prefix repeats the period's tail
    host = torch.empty(raw.shape, dtype=raw.dtype, pin_memory=True)
    host.copy_(raw.cpu())
    H = torch.empty((B, R, cfg.K), dtype=torch.complex64, device="cuda")
    # 128-frame chunks: each chunk's estimate is ~1/60 of its copy, and every copy/compute
    # handoff between the streams costs tens of microseconds when calls run back to back
    chunk = 128
    # one staging buffer for every call, as a serving loop keeps it (a fresh
    # allocation per call can reach the driver and stall the stream)
    staging = torch.empty((2 * chunk * R * (cp + N) * 8,), dtype=torch.uint8, device="cuda")
    ms, _ = time_steps(lambda: plan.stream_from_host(host, cp, chunk, "bf16", out=H,
                                                     staging=staging),
                       max(2, args.steps // 4), 1, torch)
    # the box's own host-to-device rate for the same bytes: one plain copy
    ms_copy, _ = time_steps(lambda: raw.copy_(host, non_blocking=True), max(2, args.steps // 4), 1,
                            torch)
    ms_dev, _ = time_steps(lambda: plan.estimate_cp(raw, cp, "bf16", out=H), args.steps, 2,
                           torch)
    byt = raw.numel() * 8
    airtime = {f"{fs:g} MHz": (cp + N) / fs for fs in (10.0, 30.72, 61.44, 122.88)}
    del raw, host, H, staging
    return {"cp": cp, "frames": B, "chunk_frames": chunk,
            "host_stream_ms": ms, "host_stream_GB/s": byt / ms / 1e6,
            "plain_h2d_copy_ms": ms_copy, "plain_h2d_copy_GB/s": byt / ms_copy / 1e6,
            "host_stream_vs_plain_copy": ms_copy / ms,
            "host_stream_CIR/s": B * R * cfg.T / (ms * 1e-3),
            "device_resident_cp_ms": ms_dev,
            "frame_latency_with_h2d_us": lat_h2d_us,
            "frame_airtime_us": airtime,
            "note": "PCIe-inclusive: raw c64 blocks from pinned host memory, copies on a second "
                    "stream overlapped with the bf16 estimate (prefix skipped by addressing); "
                    "airtime per multiplexed block of Eq. 11 at each sample rate"}


# (array size N_t = N_r, PN length M, taps L = cyclic prefix C, N_batch) of the
# latency sweeps: Fig. 6 over M at 16 x 16, Fig. 7 over the array size at
# M = 2047 (Table I's values)
LATENCY_POINTS = ([(16, M, 64, nb) for M in (511, 1023, 2047) for nb in (1, 2, 4, 8)] +
                  [(n, 2047, 128, nb) for n in (16, 32, 64) for nb in (1, 2, 4, 8)])


def latency_sweeps(torch, args):
    """Frame latency of Section IV-C/IV-D (Figs. 6 and 7) against the pilot
    airtime of Eq. 11. A frame holds the pilots of all N_t transmitters:
    N_t / N_batch multiplexed blocks, each C + M samples (C = L, the cyclic
    prefix) on each of the N_r antennas, i.e. N_t / N_batch estimator frames
    of the plan (M, T = N_batch, L, R = N_r). Per frame, p50 over
    `latency_iters` runs (HIP events on one stream): the bf16 estimate of the
    device-resident blocks (prefix skipped by addressing); the same after
    the host-to-device copy of the raw blocks from pinned memory; and that
    plus the copy of the CIRs back to pinned memory. Airtime of Eq. 11:
    (C + M) / F_s * N_t / N_batch at F_s = 10 MHz. Synthetic complex
    Gaussian samples: the latency does not depend on the values."""
    from paper_2206_05506_amd import Plan
    iters = max(50, args.latency_iters)
    rows = []
    for n_ant, M, L, nb in LATENCY_POINTS:
        blocks = n_ant // nb
        with Plan(M, nb, L, n_ant) as plan:
            raw = _randn_c64((blocks, n_ant, L + M), 1000 + M + nb + n_ant, torch)
            host = torch.empty(raw.shape, dtype=raw.dtype, pin_memory=True)
            host.copy_(raw.cpu())
            H = torch.empty((blocks, n_ant, nb * L), dtype=torch.complex64, device="cuda")
            H_host = torch.empty(H.shape, dtype=H.dtype, pin_memory=True)

            def kernel():
                plan.estimate_cp(raw, L, "bf16", out=H)

            def h2d():
                raw.copy_(host, non_blocking=True)
                kernel()

            def h2d_d2h():
                h2d()
                H_host.copy_(H, non_blocking=True)

            rows.append({
                "array": f"{n_ant}x{n_ant}", "M": M, "L": L, "N_batch": nb, "blocks": blocks,
                "lag_alias": nb * L > M,
                "frame_bytes_in": raw.numel() * 8, "cir_bytes_out": H.numel() * 8,
                "p50_us_estimate": p50_latency_us(kernel, iters, torch),
                "p50_us_h2d_estimate": p50_latency_us(h2d, iters, torch),
                "p50_us_h2d_estimate_d2h": p50_latency_us(h2d_d2h, iters, torch),
                "p50_us_wall_h2d_estimate_d2h": p50_wall_us(h2d_d2h, iters, torch),
                "airtime_us_10MHz": (L + M) / 10.0 * n_ant / nb,
            })
            del raw, host, H, H_host
    return {"rows": rows,
            "note": "one frame = pilots of all N_t transmitters (N_t / N_batch blocks of C + M "
                    "samples, C = L) on N_r = N_t antennas; bf16 estimate; p50 of HIP-event-timed "
                    "runs on one stream, copies from and to pinned host memory, and p50 of the "
                    "host wall clock around the whole frame (synchronize included); airtime of Eq. 11 "
                    "at 10 MHz; lag_alias marks N_batch * L > M (Eq. 7 violated: lags wrap)"}


def pmc_probe(torch):
    """Three headline launches and three plain copies of the code buffer,
    nothing timed: the workload of a rocprofv3 --pmc byte-counter run."""
    import synth
    from paper_2206_05506_amd import Plan
    cfg = synth.PRECISION
    plan = Plan(cfg.N, cfg.T, cfg.L, cfg.R)
    y = _randn_c64((cfg.B, cfg.R, cfg.N), 21, torch)
    q, sc = plan.pack(y, "bf16")
    del y
    H = torch.empty((cfg.B, cfg.R, cfg.K), dtype=torch.complex64, device="cuda")
    q2 = torch.empty_like(q)
    for _ in range(3):
        plan.estimate_packed(q, sc, "bf16", out=H)
    for _ in range(3):
        q2.copy_(q)
    torch.cuda.synchronize()
    code_b = q.numel() * q.element_size()
    print(json.dumps({"pmc_probe": True, "estimate_bytes_read": code_b,
                      "estimate_bytes_written": H.numel() * 8,
                      "copy_bytes_each_way": code_b}), flush=True)
    plan.close()


def mfma_probe(torch):
    """Three launches each of the matrix-core-bound kernels on fixed seeded
    data, nothing timed: the workload of a rocprofv3 --pmc run."""
    import synth
    from paper_2206_05506_amd import Plan
    cfg = synth.PRECISION
    p = Plan(cfg.N, cfg.T, cfg.L, cfg.R)
    y = _randn_c64((cfg.B, cfg.R, cfg.N), 11, torch)
    H = torch.empty((cfg.B, cfg.R, cfg.K), dtype=torch.complex64, device="cuda")
    for fmt in ("bf16", "e4m3"):
        q, sc = p.pack(y, fmt)
        for _ in range(3):
            p.estimate_packed(q, sc, fmt, out=H)
        del q, sc
    for _ in range(3):
        p.estimate(y, "f32s", out=H)
    torch.cuda.synchronize()
    p.close()
    print(json.dumps({"mfma_probe": True}), flush=True)


def adjoint_probe(torch):
    """Three launches each of the FP32-accurate adjoint (FP32-baseline and
    differentiation shapes) and of the FP32-accurate estimate on fixed seeded
    data, nothing timed: the workload of a rocprofv3 run."""
    import synth
    from paper_2206_05506_amd import Plan
    for cfg in (synth.FP32, synth.DIFF):
        with Plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
            G = _randn_c64((cfg.B, cfg.R, cfg.K), 31, torch)
            A = torch.empty((cfg.B, cfg.R, cfg.N), dtype=torch.complex64, device="cuda")
            for _ in range(3):
                p.adjoint(G, "f32s", out=A)
            if cfg is synth.FP32:
                for _ in range(3):
                    p.estimate(A, "f32s", out=G)
            torch.cuda.synchronize()
            del G, A
    print(json.dumps({"adjoint_probe": True}), flush=True)


def exact_probe(torch):
    """Three launches each of the residual r = y - P x on the precision-study
    frames: exact sums (eight int8 digits), FP64 sums, four int8 digits and
    the FP32-accurate bf16 split; nothing timed."""
    import synth
    from paper_2206_05506_amd import Plan
    cfg = synth.PRECISION
    with Plan(cfg.N, cfg.T, cfg.L, cfg.R) as p:
        y = _randn_c64((cfg.B, cfg.R, cfg.N), 41, torch)
        X = _randn_c64((cfg.B, cfg.R, cfg.K), 42, torch)
        A = torch.empty_like(y)
        for prec in ("exact", "f64acc", "exact32", "f32s"):
            for _ in range(3):
                p.adjoint(X, prec, alpha=-1.0, beta=1.0, C=y, out=A)
        torch.cuda.synchronize()
        del y, X, A
    print(json.dumps({"exact_probe": True}), flush=True)


def varlen_probe(torch):
    """Three persistent launches of the uneven batch and three plain copies
    of its code buffer (the counters' calibration), nothing timed."""
    import synth
    from paper_2206_05506_amd import VarlenPlan
    shapes = [(int(R), (1 << int(d)) - 1, int(T), int(L))
              for R, d, T, L in synth.varlen_shapes(4096, 3)]
    vp = VarlenPlan(shapes)
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    Yq = torch.randn((vp.n_codes,), generator=g, device="cuda").to(torch.bfloat16)
    Yq = Yq.view(torch.int16).contiguous()
    H = torch.empty((vp.n_out,), dtype=torch.complex64, device="cuda")
    for _ in range(3):
        vp.estimate(Yq, None, out=H)
    Y2 = torch.empty_like(Yq)
    for _ in range(3):
        Y2.copy_(Yq)
    torch.cuda.synchronize()
    print(json.dumps({"varlen_probe": True, "code_bytes": vp.n_codes * 2,
                      "cir_bytes": vp.n_out * 8}), flush=True)
    vp.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the estimator "
              "shards by frames or antennas with no exchange, see the design notes.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.mfma_probe:
        mfma_probe(torch)
        return
    if args.pmc_probe:
        pmc_probe(torch)
        return
    if args.adjoint_probe:
        adjoint_probe(torch)
        return
    if args.varlen_probe:
        varlen_probe(torch)
        return
    if args.exact_probe:
        exact_probe(torch)
        return
    out, ctx = headline(torch, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(ctx["plan"], ctx["cfg"], ctx["y"], ctx["q"],
                                           ctx["sc"], ctx["H"], args.cpu_seconds, torch)
    ctx["plan"].close()
    ctx.clear()
    torch.cuda.empty_cache()
    if not args.no_workloads:
        out["fp32_baseline_workload"] = fp32_baseline_workload(torch, args)
        out["differentiation_workload"] = differentiation_workload(torch, args)
    if not args.no_rows:
        out["latency_sweeps"] = latency_sweeps(torch, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark: CIR estimates per second of PN-correlation channel estimation on
one MI355X, BF16 matrix-core path against the FP32-accurate path at matched
NMSE, plus p50 single-frame latency.

Workload (FP32-baseline shape): N = 1023 (degree-10 m-sequence), T = 16
multiplexed transmitters, L = 32 taps (T*L = 512 lags), R = 64 antennas,
256 frames of complex64 input, exponential power-delay profile (decay 8
taps), SNR uniform in [0, 20] dB per frame. Synthetic frames: seeded draws
(synth), composed into y = P h + noise by the library's own adjoint kernel.

A timed step is one estimation pass over the batch resident in HBM:
  bf16 path  : pnce_estimate(precision=BF16) -- c64 frames read once, rounded
               to bf16 in registers, +-1 operand expanded on chip, bf16
               matrix cores, FP32 accumulation, c64 CIRs written;
  fp32 path  : pnce_estimate(precision=F32S), FP32-accurate (timed too).

Besides the headline, the line carries timings of every other form of the
path: the quantiser, the packed estimate, the adjoint, refinement and the
4096-frame uneven batch (rows), the precision-study workload (N = 4095,
T*L = 2048, R = 256, 512 frames: bf16 / f16 / e4m3 packed estimates and
refinement) and the differentiation workload (N = 1023, T*L = 1024, R = 128,
1024 frames: forward + backward through autograd), and a second one-frame
latency that includes the copy of the frame from pinned host memory.

Prints one JSON line (rank 0). Usage:
  python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--no-cpu] [--no-rows]
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
ROTATE_COPIES = 5              # frame / CIR buffer copies the timed steps rotate over

# HBM bytes per launch of the bf16 estimate measured with rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE (scaled by a plain copy of known size), valid only
# for the kernel source with this sha256; any other source reports null.
TRAFFIC = {"source_sha256": "5b2ae679350dc357a5f1bb693846dad60b3ef591700604b91ffecf7ddd638203",
           "bytes_per_launch": 203461198}
BF16_PEAK_TFLOPS = 2516.6      # dense bf16 / f16 matrix
FP8_PEAK_TFLOPS = 5033.2       # dense fp8 matrix
FP32_PEAK_TFLOPS = 157.3       # dense fp32 matrix
FP64_PEAK_TFLOPS = 78.6        # dense fp64 matrix


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--latency-iters", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--pmc-probe", action="store_true",
                    help="only 3 bf16 estimates and 3 plain copies of the frames (for "
                         "rocprofv3 --pmc byte counters and their copy-kernel calibration)")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="only 3 launches each of the matrix-bound kernels (precision-study "
                         "packed bf16 and e4m3 estimates on 64 frames, FP32-accurate and bf16 "
                         "estimates of the benchmark frames), for rocprofv3 --pmc counters of "
                         "matrix-core activity")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the quantiser/adjoint/refinement/uneven-batch timings")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the precision-study and differentiation workloads")
    return ap.parse_args()


def measured_traffic():
    import hashlib
    src = os.path.join(ROOT, "paper_2206_05506_amd", "csrc", "pnce_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return TRAFFIC["bytes_per_launch"] if sha == TRAFFIC["source_sha256"] else None


def make_inputs(plan, cfg, torch):
    """Seeded draws -> y = P h_stack + sigma w on the GPU (library adjoint)."""
    import synth
    d = synth.batch_draws(cfg)
    h = torch.from_numpy(d["h"].reshape(cfg.B, cfg.R, cfg.K)).to(torch.complex64).cuda()
    w = torch.from_numpy(d["w"]).to(torch.complex64).cuda()
    snr = torch.from_numpy(d["snr_db"]).cuda()
    y_clean = plan.adjoint(h, "f32s", alpha=1.0)          # P h (no 1/N)
    p = (y_clean.abs() ** 2).mean(dim=(1, 2)).double()
    sigma = torch.sqrt(p / 10.0 ** (snr / 10.0)).float()
    y = (y_clean + sigma[:, None, None] * w).contiguous()
    torch.cuda.synchronize()
    return y, h


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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(y_dev, cfg, target_s):
    """The FP64 oracle on a bounded sample of the same frames, on the host's
    cores (OpenMP): whole passes over the first n frames, repeated until at
    least target_s seconds of work (one pass is at most about target_s). Returns the cpu_baseline object of the JSON line."""
    import oracle
    s = oracle.mseq(cfg.d)
    y = y_dev.cpu().numpy()
    oracle.correlate(y[:2], s, cfg.K)                      # warm-up (threads, pages)
    t0 = time.perf_counter()
    oracle.correlate(y[:8], s, cfg.K)
    per_frame = (time.perf_counter() - t0) / 8
    n = int(max(1, min(cfg.B, round(target_s / max(per_frame, 1e-4)))))
    reps = 0
    t0 = time.perf_counter()
    while True:                                  # whole passes until target_s is reached
        oracle.correlate(y[:n], s, cfg.K)
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= target_s:
            break
    # one thread, on a quarter of the sample
    n1 = max(1, n // 4)
    t0 = time.perf_counter()
    oracle.correlate(y[:n1], s, cfg.K, threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": reps * n * cfg.R * cfg.T / dt, "unit": "CIR estimates/s",
            "one_thread_value": n1 * cfg.R * cfg.T / dt1, "cpu_model": cpu_model(),
            "nproc": os.cpu_count(),
            "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{reps} pass(es) over {n} of {cfg.B} frames (N={cfg.N}, T*L={cfg.K}, "
                      f"R={cfg.R}), FP64 direct correlation, {dt:.1f} s"}


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
    res["refine_1_step"] = {"ms": ms, "note": "FP64-accumulated residual + f32s correlation"}
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


def uneven_batch(torch, args):
    """4096 frames of uneven (R, N, T, L) (seed 3), bf16 codes: one persistent
    launch (autotuned) against one launch per frame."""
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
    start = vp.tuning()
    vp.tune(Yq, None, out=H, reps=3)
    tuned = vp.tuning()
    ms_p, _ = time_steps(lambda: vp.estimate(Yq, None, out=H), args.steps, 2, torch)
    # the default schedule, timed in the same (warm) state for comparison
    vp.set_tuning(start)
    ms_u, _ = time_steps(lambda: vp.estimate(Yq, None, out=H), args.steps, 2, torch)
    vp.set_tuning(tuned)
    ms_e, _ = time_steps(lambda: vp.estimate_each(Yq, None, out=H), 3, 1, torch)
    # the persistent launch captured once in a HIP graph and replayed
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        vp.estimate(Yq, None, out=H)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        vp.estimate(Yq, None, out=H)
    ms_g, _ = time_steps(graph.replay, args.steps, 2, torch)
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
    return {"frames": len(shapes), "persistent_ms": ms_p, "untuned_ms": ms_u,
            "graph_replay_ms": ms_g,
            "per_frame_launches_ms": ms_e,
            "speedup": ms_e / ms_p, "CIR/s": cirs / (ms_p * 1e-3),
            "GB/s": byt / ms_p / 1e6, "hbm_frac": byt / ms_p / 1e6 / HBM_PEAK_GBS,
            "mfma_frac": flops / ms_p / 1e9 / BF16_PEAK_TFLOPS,
            "per_frame_roofline_us": roof_us, "per_frame_roofline_frac": roof_us / (ms_p * 1e3),
            "workgroups": st["workgroups"], "tiles": st["tiles"]}


def _randn_c64(shape, seed, torch):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    re = torch.randn(shape, generator=g, device="cuda")
    im = torch.randn(shape, generator=g, device="cuda")
    return torch.complex(re, im).contiguous()


def precision_workload(torch, args):
    """Precision-study shape (N=4095, T=32, L=64, R=256, 512 frames): quantiser,
    packed estimates in bf16 / f16 / e4m3, and least-squares refinement from
    the original complex64 frames (parity is in the GPU tests; here, time)."""
    import synth
    from paper_2206_05506_amd import Plan
    cfg = synth.PRECISION
    B, R, N, K = cfg.B, cfg.R, cfg.N, cfg.K
    plan = Plan(N, cfg.T, cfg.L, R)
    y = _randn_c64((B, R, N), 21, torch)
    H = torch.empty((B, R, K), dtype=torch.complex64, device="cuda")
    flops = 4.0 * B * R * N * K
    res = {"workload": cfg.name, "frames": B, "R": R, "N": N, "T*L": K}
    steps = max(2, args.steps // 4)
    for fmt, peak in (("bf16", BF16_PEAK_TFLOPS), ("f16", BF16_PEAK_TFLOPS),
                      ("e4m3", FP8_PEAK_TFLOPS)):
        q, sc = plan.pack(y, fmt)
        ms_p, _ = time_steps(lambda: plan.pack(y, fmt, out=q, scales=sc), steps, 1, torch)
        ms_e, _ = time_steps(lambda: plan.estimate_packed(q, sc, fmt, out=H), steps, 1, torch)
        code_b = q.numel() * q.element_size()
        res[fmt] = {"pack_ms": ms_p, "pack_GB/s": (B * R * N * 8 * 2 + code_b) / ms_p / 1e6,
                    "estimate_ms": ms_e, "TFLOP/s": flops / ms_e / 1e9,
                    "mfma_frac": flops / ms_e / 1e9 / peak,
                    "GB/s": (code_b + B * R * K * 8) / ms_e / 1e6,
                    "CIR/s": B * R * cfg.T / (ms_e * 1e-3)}
        del q, sc
    ms_s, _ = time_steps(lambda: plan.estimate(y, "f32s", out=H), steps, 1, torch)
    res["f32s_estimate_ms"] = ms_s
    work = torch.empty_like(y)
    X = H.clone()
    ms_1, _ = time_steps(lambda: plan.refine(y, X, 1, work=work), 2, 1, torch)
    ms_5, _ = time_steps(lambda: plan.refine(y, X, 5, work=work), 2, 1, torch)
    res["refine"] = {"steps_1_ms": ms_1, "steps_5_ms": ms_5,
                     "note": "every step: residual y - P x then x += P^T r / N (f32s); the "
                             "last step's residual accumulates in FP64 on FP64 matrix cores"}
    plan.close()
    del y, H, work, X
    torch.cuda.empty_cache()
    res["accuracy"] = precision_accuracy(torch, cfg)
    return res


def precision_accuracy(torch, cfg, frames=8):
    """Accuracy of the precision study's forms on `frames` frames of the
    channel model (seeded device draws, y = P h + sigma w by the library's
    adjoint): for the bf16-, f16- and e4m3-packed starts and k = 0..5 refinement
    steps, the normwise error against the FP64 iterate with the same k (the
    library's FP64 vector kernel on complex128 copies) and the NMSE against
    h; and the FP32-accurate correlator's NMSE beside bf16's (k = 0)."""
    from paper_2206_05506_amd import Plan
    import synth
    N, K, R = cfg.N, cfg.K, cfg.R
    plan = Plan(N, cfg.T, cfg.L, R)
    d = synth.device_draws(cfg, torch, frames=frames)
    h = d["h"].reshape(frames, R, K)
    y0 = plan.adjoint(h, "f32s", alpha=1.0)
    p = (y0.abs() ** 2).mean(dim=(1, 2)).double()
    sigma = torch.sqrt(p / 10.0 ** (d["snr_db"].double() / 10.0)).float()
    y = (y0 + sigma[:, None, None] * d["w"]).contiguous()
    del y0, d
    # FP64 iterates x_{k+1} = x_k + P^T (y - P x_k) / N
    y64 = y.to(torch.complex128)
    x64 = [plan.estimate(y64, "f64")]
    for _ in range(5):
        r = y64 - plan.adjoint(x64[-1], "f64", alpha=1.0)
        x64.append(x64[-1] + plan.estimate(r, "f64"))
    del y64

    def relerr(x, ref):
        e = ((x.to(torch.complex128) - ref).abs() ** 2).reshape(frames, -1).sum(1)
        n = (ref.abs() ** 2).reshape(frames, -1).sum(1)
        return float(torch.sqrt(e / n).max())

    out = {"frames": frames, "reference": "FP64 iterate with the same k (library FP64 kernel)"}
    work = torch.empty_like(y)
    for fmt in ("bf16", "f16", "e4m3"):
        q, sc = plan.pack(y, fmt)
        x0 = plan.estimate_packed(q, sc, fmt)
        rows = []
        for k in range(6):
            X = x0.clone()
            if k:
                plan.refine(y, X, k, work=work)
            rows.append({"k": k, "relerr_vs_fp64": relerr(X, x64[k]), "nmse_db": nmse_db(X, h)})
        out[fmt] = rows
        del q, sc, x0
    out["fp32_k0_nmse_db"] = nmse_db(plan.estimate(y, "f32s"), h)
    out["fp64_k5_nmse_db"] = nmse_db(x64[5].to(torch.complex64), h)
    plan.close()
    return out


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
    chunk = 32
    ms, _ = time_steps(lambda: plan.stream_from_host(host, cp, chunk, "bf16", out=H),
                       max(2, args.steps // 4), 1, torch)
    ms_dev, _ = time_steps(lambda: plan.estimate_cp(raw, cp, "bf16", out=H), args.steps, 2,
                           torch)
    byt = raw.numel() * 8
    airtime = {f"{fs:g} MHz": (cp + N) / fs for fs in (10.0, 30.72, 61.44, 122.88)}
    del raw, host, H
    return {"cp": cp, "frames": B, "chunk_frames": chunk,
            "host_stream_ms": ms, "host_stream_GB/s": byt / ms / 1e6,
            "host_stream_CIR/s": B * R * cfg.T / (ms * 1e-3),
            "device_resident_cp_ms": ms_dev,
            "frame_latency_with_h2d_us": lat_h2d_us,
            "frame_airtime_us": airtime,
            "note": "PCIe-inclusive: raw c64 blocks from pinned host memory, copies on a second "
                    "stream overlapped with the bf16 estimate (prefix skipped by addressing); "
                    "airtime per multiplexed block of Eq. 11 at each sample rate"}


def mfma_probe(torch):
    """Three launches each of the matrix-core-bound kernels on fixed seeded
    data, nothing timed: the workload of a rocprofv3 --pmc run."""
    from paper_2206_05506_amd import Plan
    N, T, L, R, B = 4095, 32, 64, 256, 64      # the precision study, 64 frames
    p = Plan(N, T, L, R)
    y = _randn_c64((B, R, N), 11, torch)
    H = torch.empty((B, R, T * L), dtype=torch.complex64, device="cuda")
    for fmt in ("bf16", "e4m3"):
        q, sc = p.pack(y, fmt)
        for _ in range(3):
            p.estimate_packed(q, sc, fmt, out=H)
        del q, sc
    p.close()
    del y, H
    import synth
    cfg = synth.FP32
    p = Plan(cfg.N, cfg.T, cfg.L, cfg.R)
    y = _randn_c64((cfg.B, cfg.R, cfg.N), 12, torch)
    H = torch.empty((cfg.B, cfg.R, cfg.K), dtype=torch.complex64, device="cuda")
    for prec in ("f32s", "bf16"):
        for _ in range(3):
            p.estimate(y, prec, out=H)
    torch.cuda.synchronize()
    p.close()
    print(json.dumps({"mfma_probe": True}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the estimator "
              "shards by frames or antennas with no exchange, see the design notes.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2206_05506_amd import Plan

    if args.mfma_probe:
        mfma_probe(torch)
        return
    cfg = synth.FP32
    plan = Plan(cfg.N, cfg.T, cfg.L, cfg.R)
    y, h = make_inputs(plan, cfg, torch)
    H_bf = torch.empty((cfg.B, cfg.R, cfg.K), dtype=torch.complex64, device="cuda")
    if args.pmc_probe:
        y2 = torch.empty_like(y)
        for _ in range(3):
            plan.estimate(y, "bf16", out=H_bf)
        for _ in range(3):
            y2.copy_(y)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "estimate_bytes_read": cfg.B * cfg.R * cfg.N * 8,
                          "estimate_bytes_written": cfg.B * cfg.R * cfg.K * 8,
                          "copy_bytes_each_way": y.numel() * 8}), flush=True)
        plan.close()
        return
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

    def step_bf16():
        i = rot()
        plan.estimate(ys[i], "bf16", out=Hs[i])

    def step_f32s():
        i = rot()
        plan.estimate(ys[i], "f32s", out=Hs[i])

    def step_f32():
        i = rot()
        plan.estimate(ys[i], "f32", out=Hs[i])

    spin_up(step_bf16, 0.3, torch)
    ms_bf, wall_bf = time_steps(step_bf16, args.steps, args.warmup, torch)
    # context for the roofline: a plain device copy of the same frame buffers
    # (rotated likewise), read + write bytes over its time
    ms_cp, _ = time_steps(lambda: ys[rot()].copy_(ys[(ctr[0] + 2) % n_rot]), args.steps, 2, torch)
    # the same launch on one resident buffer (frames and CIRs cache-resident)
    ms_bf_cached, _ = time_steps(lambda: plan.estimate(y, "bf16", out=H_bf), args.steps,
                                 args.warmup, torch)
    ms_32, _ = time_steps(step_f32s, args.steps, args.warmup, torch)
    H_32.copy_(Hs[ctr[0]])
    ms_mf, _ = time_steps(step_f32, max(2, args.steps // 4), 2, torch)
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

    y1 = y[:1].contiguous()
    H1 = torch.empty((1, cfg.R, cfg.K), dtype=torch.complex64, device="cuda")
    lat_bf = lat_32 = lat_h2d = lat_plain = None
    if args.latency_iters > 0:
        lat_bf = p50_latency_us(lambda: plan.estimate(y1, "bf16", out=H1), args.latency_iters,
                                torch)
        lat_32 = p50_latency_us(lambda: plan.estimate(y1, "f32s", out=H1), args.latency_iters,
                                torch)
        # the same frame handed over in pinned host memory: copy in, then estimate
        y1_host = torch.empty(y1.shape, dtype=y1.dtype, pin_memory=True)
        y1_host.copy_(y1.cpu())
        y1_dev = torch.empty_like(y1)

        def h2d_then_estimate():
            y1_dev.copy_(y1_host, non_blocking=True)
            plan.estimate(y1_dev, "bf16", out=H1)

        lat_h2d = p50_latency_us(h2d_then_estimate, args.latency_iters, torch)
        # the plain workload (N=127, T=4, L=16, R=16, one frame)
        pc = synth.PLAIN
        pp = Plan(pc.N, pc.T, pc.L, pc.R)
        yp = _randn_c64((1, pc.R, pc.N), 13, torch)
        Hp = torch.empty((1, pc.R, pc.K), dtype=torch.complex64, device="cuda")
        lat_plain = {prec: p50_latency_us(lambda: pp.estimate(yp, prec, out=Hp),
                                          args.latency_iters, torch) for prec in ("bf16", "f32s")}
        pp.close()

    nmse_bf = nmse_db(H_bf, h)
    nmse_32 = nmse_db(H_32, h)
    nmse_mf = nmse_db(H_mf, h)

    cirs = cfg.B * cfg.R * cfg.T
    flops = 4.0 * cfg.B * cfg.R * cfg.N * cfg.K
    bytes_ = cfg.B * (cfg.R * cfg.N * 8 + cfg.R * cfg.K * 8)
    ach_gbs = bytes_ / (ms_bf * 1e-3) / 1e9

    out = {
        "metric": "CIR estimates/s + p50 frame latency; BF16-MFMA vs FP32 at matched NMSE",
        "value": cirs / (ms_bf * 1e-3),
        "frames_per_s": cfg.B / (ms_bf * 1e-3),
        "unit": "CIR estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_bf,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded draws, y = P h + noise composed on the GPU)",
        "config": {"workload": cfg.name, "N": cfg.N, "T": cfg.T, "L": cfg.L, "R": cfg.R,
                   "frames": cfg.B, "input": "complex64", "snr_db": [cfg.snr_lo, cfg.snr_hi]},
        "p50_frame_latency_us": {"bf16": lat_bf, "fp32": lat_32,
                                 "bf16_with_h2d_copy": lat_h2d,
                                 "plain_workload": lat_plain},
        "fp32_path": {"value": cirs / (ms_32 * 1e-3), "ms_per_step": ms_32,
                      "precision": "f32s (3-way bf16 split, exact)"},
        "fp32_mfma_path": {"value": cirs / (ms_mf * 1e-3), "ms_per_step": ms_mf,
                           "precision": "f32 (v_mfma_f32_32x32x2_f32)"},
        "bf16_speedup_vs_fp32": {"fp32_mfma": ms_mf / ms_bf, "fp32_accurate_bf16x3": ms_32 / ms_bf,
                                 "note": "fp32_mfma: the FP32 matrix-core path "
                                         "(v_mfma_f32_32x32x2_f32); fp32_accurate_bf16x3: the "
                                         "faster FP32-accurate path (exact 3-way bf16 split); "
                                         "all at equal NMSE (see nmse_db)"},
        "nmse_db": {"bf16": nmse_bf, "fp32": nmse_32, "fp32_mfma": nmse_mf,
                    "delta_bf16_fp32": nmse_bf - nmse_32},
        "wall_ms_per_step": wall_bf,
        "timing": {"rotated_buffers": ROTATE_COPIES,
                   "note": "each timed step reads its own copy of the frames and writes its own "
                           "CIR buffer (5 x 201 MB > the 256 MB Infinity Cache), so frames stream "
                           "from HBM",
                   "cache_resident_ms_per_step": ms_bf_cached,
                   "hbm_copy_GB/s": 2 * y.numel() * 8 / (ms_cp * 1e-3) / 1e9,
                   "cache_resident_GB/s": bytes_ / (ms_bf_cached * 1e-3) / 1e9},
        "pipelined_two_streams": {
            "ms_per_step": ms_pipe, "CIR/s": cirs / (ms_pipe * 1e-3),
            "GB/s": bytes_ / (ms_pipe * 1e-3) / 1e9,
            "hbm_frac": bytes_ / (ms_pipe * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "note": "the same steps (one launch each, frames streamed from HBM) issued "
                    "alternately on two streams, as a serving loop pipelines independent "
                    "batches; value above is the one-stream figure"},
        "roofline": {"bound": "hbm", "achieved": ach_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": ach_gbs / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "tg_kernel<BF16, c64 in, NC=4>",
                     "mfma_frac": flops / (ms_bf * 1e-3) / 1e12 / BF16_PEAK_TFLOPS},
    }
    if not args.no_rows:
        out["rows"] = other_rows(plan, cfg, y, H_32, torch, args)
        out["rows"]["front_end"] = front_end(plan, cfg, y, torch, lat_h2d, args)
    if not args.no_workloads:
        out["precision_workload"] = precision_workload(torch, args)
        out["differentiation_workload"] = differentiation_workload(torch, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(y, cfg, args.cpu_seconds)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

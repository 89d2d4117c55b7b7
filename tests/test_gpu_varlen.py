"""Batching form: frames of uneven (R, N, T*L) in one persistent launch.

Inputs are bf16 codes drawn with torch (not by the library), with a zero pad
sample per plane and a power-of-two scale per frame. Checks: the persistent
launch equals one launch per frame bit for bit (same tiles, same order);
sampled frames match the FP64 oracle on the dequantised codes within 1e-5;
a hipGraph capture replays to the same result; the autotuner's choices keep
parity.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import host, perr

pytestmark = pytest.mark.gpu


def _shapes(nframes, seed=3):
    return [(int(R), (1 << int(d)) - 1, int(T), int(L))
            for R, d, T, L in synth.varlen_shapes(nframes, seed)]


def _inputs(vp, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    codes = torch.randn((vp.n_codes,), generator=g, device="cuda").to(torch.bfloat16)
    pads = []
    for f, (R, N, T, L) in enumerate(vp.shapes):
        pads.append(vp.y_off[f] + np.arange(2 * R, dtype=np.int64) * (N + 1) + N)
    codes[torch.from_numpy(np.concatenate(pads)).cuda()] = 0
    e = torch.randint(-3, 4, (len(vp.shapes),), generator=g, device="cuda")
    scales = torch.pow(2.0, e.float()).contiguous()
    return codes.view(torch.int16).contiguous(), scales


def _oracle_frame(vp, Yq_host, sc_host, H, f):
    R, N, T, L = vp.shapes[f]
    c = Yq_host[vp.y_off[f]:vp.y_off[f] + R * 2 * (N + 1)].view(np.uint16).reshape(1, R, 2, N + 1)
    x = oracle.dequantize(c, sc_host[f:f + 1], "bf16", N)
    ref = oracle.correlate(x, oracle.mseq(oracle.degree_of(N)), T * L)
    got = host(vp.frame_view(H, f)).reshape(1, R, T * L)
    return perr(got, ref)


def test_varlen_edge_shapes():
    """Ragged antenna counts, tiny sequences, K < 32, lag alias, one frame of
    each width class, mixed in one launch."""
    from paper_2206_05506_amd import VarlenPlan
    shapes = [(1, 3, 1, 2), (5, 7, 2, 3), (33, 31, 2, 4), (40, 63, 5, 16), (64, 255, 4, 16),
              (17, 511, 8, 32), (96, 1023, 16, 32), (32, 2047, 16, 64), (3, 127, 1, 127)]
    with VarlenPlan(shapes) as vp:
        Yq, sc = _inputs(vp, 1)
        H = vp.estimate(Yq, sc)
        He = vp.estimate_each(Yq, sc)
        torch.cuda.synchronize()
        assert torch.equal(H, He)
        Yh, sh = host(Yq), host(sc)
        for f in range(len(shapes)):
            assert _oracle_frame(vp, Yh, sh, H, f) <= 1e-5, shapes[f]


def test_varlen_batching_workload():
    """The batching workload: 4096 frames, R in {32..256}, N in {255..2047},
    T in {4, 8, 16}, L in {16, 32, 64} with T*L <= N (seed 3)."""
    from paper_2206_05506_amd import VarlenPlan
    shapes = _shapes(4096)
    with VarlenPlan(shapes) as vp:
        Yq, sc = _inputs(vp, 2)
        H = vp.estimate(Yq, sc)
        He = vp.estimate_each(Yq, sc)
        torch.cuda.synchronize()
        assert torch.equal(H, He)
        Yh, sh = host(Yq), host(sc)
        # one frame of every (N, T*L) class, plus the batch's first and last
        first = {}
        for f, (R, N, T, L) in enumerate(shapes):
            first.setdefault((N, T * L), f)
        pick = sorted(set(first.values()) | {0, len(shapes) - 1})
        print(f"{len(first)} (N, T*L) classes, oracle-checked frames {pick}")
        for f in pick:
            assert _oracle_frame(vp, Yh, sh, H, f) <= 1e-5, (f, shapes[f])

        # hipGraph: capture the persistent launch, replay with eager work between
        Hg = torch.empty_like(H)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            vp.estimate(Yq, sc, out=Hg)
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            vp.estimate(Yq, sc, out=Hg)
        for _ in range(3):
            Hg.zero_()
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            assert torch.equal(Hg, H)

        # autotuner: measured choices, then parity again
        table = vp.tune(Yq, sc, reps=3)
        assert len(table) == len({(N, T * L) for _, N, T, L in shapes})
        for N, K, nc, us in table:
            assert nc in (1, 2, 4) and us > 0
        H2 = vp.estimate(Yq, sc)
        He2 = vp.estimate_each(Yq, sc)
        torch.cuda.synchronize()
        assert torch.equal(H2, He2)
        for f in pick:
            assert _oracle_frame(vp, Yh, sh, H2, f) <= 1e-5, (f, shapes[f])
        st = vp.stats()
        print("tuned:", table, st)
        assert st["tiles"] > 0 and st["workgroups"] > 0


def test_graph_captured_before_tuning_replays_new_schedule():
    """A graph captured before set_tuning keeps valid work-list addresses:
    after every class is moved to the narrowest column width (the longest
    work list) and back to the widest, replays equal the per-frame launches
    of the current schedule and match the oracle."""
    from paper_2206_05506_amd import VarlenPlan
    shapes = _shapes(96, seed=7)
    with VarlenPlan(shapes) as vp:
        Yq, sc = _inputs(vp, 5)
        Hg = torch.empty((vp.n_out,), dtype=torch.complex64, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            vp.estimate(Yq, sc, out=Hg)
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            vp.estimate(Yq, sc, out=Hg)
        torch.cuda.synchronize()
        start = vp.tuning()
        tiles0 = vp.stats()["tiles"]
        Yh, sh = host(Yq), host(sc)
        for nc in (1, 4, None):
            table = start if nc is None else [(N, K, nc, us) for N, K, _, us in start]
            vp.set_tuning(table)
            if nc == 1:
                assert vp.stats()["tiles"] > tiles0
            He = vp.estimate_each(Yq, sc)
            for _ in range(2):
                Hg.zero_()
                torch.cuda.synchronize()
                graph.replay()
                torch.cuda.synchronize()
                assert torch.equal(Hg, He), nc
            for f in (0, len(shapes) // 2, len(shapes) - 1):
                assert _oracle_frame(vp, Yh, sh, Hg, f) <= 1e-5, (nc, f, shapes[f])
        del graph

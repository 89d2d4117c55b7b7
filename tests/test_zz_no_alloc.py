"""pnce_refine_noalloc (the refinement entry point that allocates nothing:
its residual sits in the library's fixed device array) against pnce_refine
with a caller-supplied workspace, through the C ABI: two calls in a row, the
second on a smaller input, then a frame too large for the array."""
import numpy as np
import pytest
import torch

from gpu_helpers import host, perr

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _frames(B, R, N, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    re = torch.randn((B, R, N), generator=g, device="cuda")
    im = torch.randn((B, R, N), generator=g, device="cuda")
    return torch.complex(re, im).contiguous()


def _both(plan, y, steps):
    """(X from pnce_refine, X from pnce_refine_noalloc), same bf16 start."""
    X0 = plan.estimate(y, "bf16")
    Xa = X0.clone()
    work = torch.empty_like(y)
    plan.refine(y, Xa, steps, work=work)
    Xb = X0.clone()
    plan.refine_noalloc(y, Xb, steps)
    torch.cuda.synchronize()
    return host(Xa), host(Xb)


def test_noalloc_refine_matches_refine_twice():
    from paper_2206_05506_amd import Plan
    # 1: 12 frames of 256 x 4095 (8.4 MB of residual each): refined in groups
    #    of 7 frames, so the array is reused within the call
    print("no-alloc refine: N=4095 T=32 L=64 R=256 B=12 steps=2", flush=True)
    with Plan(4095, 32, 64, 256) as p:
        y = _frames(12, 256, 4095, 11)
        a, b = _both(p, y, 2)
    assert perr(b, a) <= TOL
    # 2: a smaller input right after: 3 frames of 64 x 1023 in one group,
    #    the same launches as pnce_refine (bit-identical)
    print("no-alloc refine: N=1023 T=16 L=32 R=64 B=3 steps=3", flush=True)
    with Plan(1023, 16, 32, 64) as p:
        y = _frames(3, 64, 1023, 12)
        a, b = _both(p, y, 3)
    assert perr(b, a) <= TOL
    assert np.array_equal(a, b)


def test_noalloc_refine_edge_cases():
    from paper_2206_05506_amd import Plan
    from paper_2206_05506_amd._lib import PNCE_E_UNSUPPORTED, PnceError
    with Plan(127, 4, 16, 16) as p:
        y = _frames(2, 16, 127, 13)
        X = p.estimate(y, "f32s")
        X0 = X.clone()
        p.refine_noalloc(y, X, 0)                     # zero steps: X unchanged
        assert torch.equal(X, X0)
        p.refine_noalloc(y[:0], X[:0], 2)             # empty batch: nothing to do
        with pytest.raises(PnceError):
            p.refine_noalloc(y, X, -1)
    # one frame's residual larger than the 64 MiB array: refused, X untouched
    print("no-alloc refine: N=65535 R=129 (residual 67.6 MB per frame)", flush=True)
    with Plan(65535, 1, 8, 129) as p:
        y = torch.zeros((1, 129, 65535), dtype=torch.complex64, device="cuda")
        X = torch.full((1, 129, 8), 3.0 + 0j, dtype=torch.complex64, device="cuda")
        with pytest.raises(PnceError) as e:
            p.refine_noalloc(y, X, 1)
        assert e.value.status == PNCE_E_UNSUPPORTED
        assert torch.all(X == 3.0)


def test_noalloc_refine_under_graph_capture():
    """The callers this entry point is for: a HIP graph captured around it
    (no allocation happens inside), replayed three times on new frames with
    eager work and synchronisations between the replays; every replay equals
    the eager pnce_refine of the same frames."""
    from paper_2206_05506_amd import Plan
    print("no-alloc refine under graph capture: N=1023 T=16 L=32 R=64 B=4 steps=2", flush=True)
    with Plan(1023, 16, 32, 64) as p:
        y = _frames(4, 64, 1023, 21)
        X = p.estimate(y, "bf16")
        p.refine_noalloc(y, X.clone(), 2)          # the scratch address is resolved eagerly
        torch.cuda.synchronize()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            p.refine_noalloc(y, X.clone(), 2)
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            p.estimate(y, "bf16", out=X)
            p.refine_noalloc(y, X, 2)
        for k in range(3):
            fresh = _frames(4, 64, 1023, 30 + k)
            y.copy_(fresh)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            got = host(X)
            ref = p.estimate(fresh, "bf16")
            p.refine(fresh, ref, 2, work=torch.empty_like(fresh))
            torch.cuda.synchronize()
            assert perr(got, host(ref)) <= TOL, k
        del graph

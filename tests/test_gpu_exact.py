"""PNCE_PREC_EXACT and PNCE_PREC_EXACT32: the contraction with exact sums
(int8 matrix cores on eight or four 8-bit fixed-point digits per value,
combined in FP64).

Bar, element by element against the FP64 oracle on the same input. Eight
digits: every output is the exact sum of the fixed-point inputs, with alpha
and beta applied in FP64, rounded once to FP32, so
    |out - ref| <= 2^-24 (1 + 2^-20) (|ref| + slack) + slack.
Four digits (no FP64 arithmetic): the exact sum rounded to FP32, then alpha
(itself rounded to FP32, times the frame scale) and beta * cin applied in
FP32: at most five roundings of 2^-24 of |ref| + |beta cin|,
    |out - ref| <= 5 * 2^-24 (1 + 2^-10) (|ref| + |beta cin| + slack) + slack.
slack = 2^-45 |alpha| sum_t |x_t| (the oracle's own FP64 rounding), plus
the fixed-point rounding of the row's small elements: each element is
rounded at 2^(e - 63) (eight digits) or 2^(e - 31) (four), with 2^e <=
2 max|x| the power of two above the row's largest |re| or |im|, so t_len
2^-62 |alpha| max|x| (eight digits, only where a row spans more than 2^38)
or t_len 2^-30 |alpha| max|x| (four). Where the sum cancels, the slack term
carries the bound; elsewhere the eight-digit result is correctly rounded
FP32, which FP32 or FP64-accumulated sums followed by a rounding only
approach.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _plan(N, T, L, R, spacing="adjacent"):
    from paper_2206_05506_amd import Plan
    return Plan(N, T, L, R, spacing=spacing)


def _check(out, ref, x, alpha=1.0, spread=False, prec="exact", what="", bcin=None):
    """out, ref: [..., C]; x: the input rows [..., t] (same leading dims);
    bcin: beta * cin where the call added it (same shape as ref)."""
    out = np.asarray(out, dtype=np.complex128)
    absx = np.abs(x.real) + np.abs(x.imag)
    row_sum = absx.sum(axis=-1, keepdims=True)
    slack = 2.0 ** -45 * abs(alpha) * row_sum
    if spread or prec == "exact32":
        mx = np.maximum(np.abs(x.real), np.abs(x.imag)).max(axis=-1, keepdims=True)
        unit = 2.0 ** -30 if prec == "exact32" else 2.0 ** -62
        slack = slack + x.shape[-1] * unit * abs(alpha) * mx
    for part in (np.real, np.imag):
        err = np.abs(part(out) - part(ref))
        if prec == "exact32":
            extra = 0.0 if bcin is None else np.abs(part(bcin))
            bound = 5 * U32 * (1 + 2.0 ** -10) * (np.abs(part(ref)) + extra + slack) + slack
        else:
            bound = U32 * (1 + 2.0 ** -20) * (np.abs(part(ref)) + slack) + slack
        # a zero bound (a row of zeros) demands an exact zero
        ratio = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0),
                         np.where(err > 0, np.inf, 0.0))
        worst = float(np.max(ratio)) if err.size else 0.0
        assert worst <= 1.0, f"{what}: error {worst:.3f} x the bound"


EXACT = ["exact", "exact32"]


# (N, T, L, R, B, spacing): ragged antenna blocks (R % 4 != 0), one to
# several column groups, small launches (column groups split over
# workgroups), the lag alias (T*L > N), Eq. 8 plans (column segments in the
# correlator, lag blocks in the adjoint), and long rows.
SHAPES = [
    (3, 1, 2, 1, 1, "adjacent"),
    (7, 2, 3, 5, 2, "adjacent"),
    (31, 3, 5, 7, 3, "adjacent"),
    (63, 5, 16, 9, 2, "adjacent"),       # T*L = 80 > N
    (255, 4, 32, 40, 2, "adjacent"),
    (1023, 16, 32, 64, 3, "adjacent"),
    (2047, 16, 64, 6, 1, "adjacent"),
    (4095, 32, 64, 8, 2, "adjacent"),
    (127, 4, 16, 6, 2, "eq8"),
    (1023, 8, 64, 13, 2, "eq8"),
    (65535, 2, 8, 2, 1, "adjacent"),     # 65535 terms per correlator output
]
IDS = ["N%d_T%d_L%d_R%d_B%d_%s" % s for s in SHAPES]


@pytest.mark.parametrize("prec", EXACT)
@pytest.mark.parametrize("shape", SHAPES, ids=IDS)
def test_exact_correlator_correctly_rounded(shape, prec):
    N, T, L, R, B, spacing = shape
    y = synth.gaussian((B, R, N), N + R).astype(np.complex64)
    with _plan(N, T, L, R, spacing) as p:
        s, lag = p.sequence(), p.lags()
        H = host(p.estimate(dev(y), prec))
        H1 = host(p.estimate(dev(y), prec, alpha=1.0))
    y64 = y.astype(np.complex128)
    ref = oracle.correlate(y64, s, T * L, lag)
    _check(H, ref, y64, alpha=1.0 / N, prec=prec, what="H = YP/N")
    _check(H1, ref * N, y64, alpha=1.0, prec=prec, what="H = YP")


@pytest.mark.parametrize("prec", EXACT)
@pytest.mark.parametrize("shape", SHAPES[:-1], ids=IDS[:-1])
def test_exact_adjoint_correctly_rounded(shape, prec):
    N, T, L, R, B, spacing = shape
    K = T * L
    G = synth.gaussian((B, R, K), K + 3).astype(np.complex64)
    C = synth.gaussian((B, R, N), K + 4).astype(np.complex64)
    with _plan(N, T, L, R, spacing) as p:
        s, lag = p.sequence(), p.lags()
        A = host(p.adjoint(dev(G), prec, alpha=1.0))
        Ar = host(p.adjoint(dev(G), prec, alpha=-1.0, beta=1.0, C=dev(C)))
    G64 = G.astype(np.complex128)
    PG = N * oracle.adjoint(G64, s, lag)
    _check(A, PG, G64, prec=prec, what="A = G P^T")
    # the residual of the receive model, y - P x (beta = 1 adds C exactly)
    _check(Ar, C.astype(np.complex128) - PG, G64, prec=prec, what="C - G P^T",
           bcin=C.astype(np.complex128))


@pytest.mark.parametrize("prec", EXACT)
def test_exact_wide_dynamic_range_and_special_values(prec):
    """Rows whose elements span 2^-140 .. 2^20 (subnormals, zeros, signed
    zeros, exact powers of two), a row of zeros, and a row holding inf: its
    outputs are NaN and no other row is touched."""
    N, T, L, R, B = 255, 4, 32, 8, 1
    rng = np.random.default_rng(5)
    mag = np.ldexp(1.0, rng.integers(-140, 21, size=(B, R, N)))
    y = (rng.choice([-1.0, 1.0], size=(B, R, N)) * mag * rng.uniform(1, 2, size=(B, R, N))
         + 1j * rng.choice([-1.0, 1.0], size=(B, R, N)) * np.ldexp(1.0, rng.integers(-60, 3, size=(B, R, N))))
    y = y.astype(np.complex64)
    y[0, 1] = 0
    y[0, 2, ::7] = -0.0
    y[0, 3] = np.ldexp(1.0, rng.integers(-30, 30, size=N)).astype(np.float32)
    y[0, 5, 100] = np.inf
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        H = host(p.estimate(dev(y), prec))
    assert np.isnan(H[0, 5]).all()
    assert np.array_equal(H[0, 1], np.zeros(T * L, np.complex64))
    keep = [r for r in range(R) if r != 5]
    y64 = y[:, keep].astype(np.complex128)
    ref = oracle.correlate(y64, s, T * L)
    _check(H[:, keep], ref, y64, alpha=1.0 / N, spread=True, prec=prec, what="wide range")


@pytest.mark.parametrize("prec", EXACT)
def test_exact_scales_and_beta(prec):
    N, T, L, R, B = 511, 8, 32, 12, 3
    y = synth.gaussian((B, R, N), 21).astype(np.complex64)
    H0 = synth.gaussian((B, R, T * L), 22).astype(np.complex64)
    sc = np.array([0.5, 3.0, 1e-3], dtype=np.float32)
    with _plan(N, T, L, R) as p:
        Hd = dev(H0)
        p.estimate(dev(y), prec, out=Hd, scales=torch.from_numpy(sc).cuda(), beta=-0.75,
                   alpha=1.0)
        H = host(Hd)
        s = p.sequence()
    y64 = y.astype(np.complex128)
    ref = sc.astype(np.float64)[:, None, None] * oracle.correlate(y64, s, T * L) * N \
        - 0.75 * H0.astype(np.complex128)
    scale_rows = np.broadcast_to(sc.astype(np.float64)[:, None, None], (B, R, 1))
    _check(H, ref, y64 * scale_rows, prec=prec, what="scales, beta",
           bcin=-0.75 * H0.astype(np.complex128))


@pytest.mark.parametrize("prec,other", [("exact", "f64acc"), ("exact32", "f32s")])
def test_exact_never_further_than_the_path_it_replaces(prec, other):
    """Eight digits against FP64 sums on the FP64 matrix cores, four digits
    against the FP32-accurate bf16 split (the refinement's inner steps): on
    the same frames the digit path's largest error is never larger."""
    N, T, L, R, B = 1023, 16, 32, 64, 2
    y = synth.gaussian((B, R, N), 31).astype(np.complex64)
    with _plan(N, T, L, R) as p:
        He = host(p.estimate(dev(y), prec)).astype(np.complex128)
        Hf = host(p.estimate(dev(y), other)).astype(np.complex128)
        s = p.sequence()
    ref = oracle.correlate(y.astype(np.complex128), s, T * L)
    ee, ef = np.abs(He - ref), np.abs(Hf - ref)
    print(f"max error: {prec} {ee.max():.3e}, {other} {ef.max():.3e}")
    assert ee.max() <= ef.max() * (1 + 1e-12) + 1e-30


@pytest.mark.parametrize("prec", EXACT)
def test_exact_refuses_more_than_65535_terms(prec):
    from paper_2206_05506_amd._lib import PnceError
    N, T, L, R = 8191, 1024, 65, 1        # the adjoint sums T*L = 66560 terms
    with _plan(N, T, L, R) as p:
        G = torch.zeros((1, R, T * L), dtype=torch.complex64, device="cuda")
        with pytest.raises(PnceError, match="65535"):
            p.adjoint(G, prec)
        p.estimate(torch.zeros((1, R, N), dtype=torch.complex64, device="cuda"), prec)


def test_refine_last_residual_is_correctly_rounded():
    """pnce_refine with one step leaves the residual r = y - P x0 in its
    workspace, computed with exact sums: each element is y - P x0 rounded
    once to FP32."""
    N, T, L, R, B = 1023, 16, 32, 20, 2
    y = synth.gaussian((B, R, N), 41).astype(np.complex64)
    x0 = synth.gaussian((B, R, T * L), 42).astype(np.complex64) * np.float32(0.05)
    with _plan(N, T, L, R) as p:
        X = dev(x0)
        work = torch.empty((B, R, N), dtype=torch.complex64, device="cuda")
        p.refine(dev(y), X, 1, work=work)
        r = host(work)
        s = p.sequence()
    x64 = x0.astype(np.complex128)
    ref = y.astype(np.complex128) - N * oracle.adjoint(x64, s)
    _check(r, ref, x64, what="residual")


def test_exact_full_precision_workload_sampled():
    """The refinement's contractions at the precision workload's full size
    and launch shape (512 frames of 256 x 4095, T*L = 2048): the residual
    r = y - P x with eight and with four digits and the correlation of r
    with four, over all frames; sampled rows (first, middle and last frame;
    antennas at both ends and in a ragged spot) against the oracle, element
    by element to the bar above. Inputs are seeded torch draws on the GPU;
    the oracle reads the same values copied to the host."""
    N, T, L, R, B = 4095, 32, 64, 256, 512
    K = T * L
    g = torch.Generator(device="cuda")
    g.manual_seed(53)
    frames, ants = [0, 257, 511], [0, 101, 255]
    with _plan(N, T, L, R) as p:
        s = p.sequence()
        y = torch.complex(torch.randn((B, R, N), generator=g, device="cuda"),
                          torch.randn((B, R, N), generator=g, device="cuda")).contiguous()
        x = (torch.complex(torch.randn((B, R, K), generator=g, device="cuda"),
                           torch.randn((B, R, K), generator=g, device="cuda")) * 0.05).contiguous()
        r = torch.empty_like(y)
        xs = host(x[frames][:, ants])
        ys = host(y[frames][:, ants])
        got = {}
        for prec in EXACT:
            p.adjoint(x, prec, alpha=-1.0, beta=1.0, C=y, out=r)
            got[prec] = host(r[frames][:, ants])
        # the correlation step of the refinement: x + P^T r / N, on four digits
        p.adjoint(x, "exact", alpha=-1.0, beta=1.0, C=y, out=r)
        xn = p.estimate(r, "exact32", alpha=1.0 / N, beta=1.0, out=x.clone())
        rs = host(r[frames][:, ants])
        xns = host(xn[frames][:, ants])
        del y, x, r, xn
        torch.cuda.empty_cache()
    x64, y64, r64 = (a.astype(np.complex128) for a in (xs, ys, rs))
    ref_r = y64 - N * oracle.adjoint(x64, s)
    for prec in EXACT:
        _check(got[prec], ref_r, x64, prec=prec, what=f"residual {prec}", bcin=y64)
    ref_x = x64 + oracle.correlate(r64, s, K)
    # x + (1/N) sum_t r_t s'(...), rounded once: the slack is that of r's rows
    _check(xns, ref_x, r64, alpha=1.0 / N, prec="exact32", what="correlation exact32", bcin=x64)

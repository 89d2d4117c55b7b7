"""The C ABI from a plain C program (tests/c_client): plan, device buffers
and one operation (correlator, adjoint, quantise with or without a
workspace + packed correlator, or refinement with a workspace or with the
library's fixed array) with no Python in the process; its output checked against the
FP64 oracle, and its error statuses."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import bf16_round, perr

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CLIENT = os.path.join(HERE, "c_client", "pnce_c_client")


def _run(args, tmp_path, y, op=None):
    if not os.path.exists(CLIENT):
        pytest.fail("tests/c_client/pnce_c_client is not built (python tests/c_client/build.py)")
    fin, fout = str(tmp_path / "y.bin"), str(tmp_path / "h.bin")
    np.ascontiguousarray(y, dtype=np.complex64).tofile(fin)
    p = subprocess.run([CLIENT] + [str(a) for a in args] + [fin, fout] + ([op] if op else []),
                       capture_output=True, text=True, timeout=60)
    return p, fout


@pytest.mark.parametrize("prec", [1, 2, 5, 6])   # PNCE_PREC_F32S, _BF16, _EXACT, _EXACT32
@pytest.mark.parametrize("spacing,fb", [(0, 0), (1, 0x3F9)])
def test_c_client_estimate(tmp_path, prec, spacing, fb):
    N, T, L, R, B = 1023, 16, 32, 64, 2
    y = synth.gaussian((B, R, N), 41).astype(np.complex64)
    p, fout = _run([N, T, L, R, B, prec, fb, spacing], tmp_path, y)
    assert p.returncode == 0, p.stderr
    H = np.fromfile(fout, dtype=np.complex64).reshape(B, R, T * L)
    s = oracle.mseq_mask(10, fb) if fb else oracle.mseq(10)
    lag = oracle.lags(N, T, L, "eq8" if spacing else "contiguous")
    x = bf16_round(y) if prec == 2 else y.astype(np.complex128)
    assert perr(H, oracle.correlate(x, s, T * L, lag)) <= 1e-5


def test_c_client_error_statuses(tmp_path):
    y = np.zeros((1, 4, 1000), dtype=np.complex64)
    p, _ = _run([1000, 2, 8, 4, 1, 2, 0, 0], tmp_path, y)     # N not 2^d - 1
    assert p.returncode == 10 - (-2) and "N must be" in p.stderr
    y = np.zeros((1, 4, 127), dtype=np.complex64)
    p, _ = _run([127, 2, 8, 4, 1, 9, 0, 0], tmp_path, y)      # unknown precision
    assert p.returncode == 10 - (-1) and "precision" in p.stderr


# ragged antenna blocks (40 = 32 + 8), two frames
SMALL = (255, 4, 16, 40, 2)


def test_c_client_adjoint(tmp_path):
    N, T, L, R, B = SMALL
    G = synth.gaussian((B, R, T * L), 42).astype(np.complex64)
    p, fout = _run([N, T, L, R, B, 1, 0, 0], tmp_path, G, "adjoint")
    assert p.returncode == 0, p.stderr
    A = np.fromfile(fout, dtype=np.complex64).reshape(B, R, N)
    assert perr(A, oracle.adjoint(G, oracle.mseq(8))) <= 1e-5


@pytest.mark.parametrize("op", ["packed", "packedws"])
@pytest.mark.parametrize("fmt,name", [(1, "bf16"), (2, "f16"), (3, "e4m3")])
def test_c_client_pack_and_packed_estimate(tmp_path, fmt, name, op):
    N, T, L, R, B = SMALL
    y = (synth.gaussian((B, R, N), 43) * 3.0).astype(np.complex64)
    p, fout = _run([N, T, L, R, B, 1, 0, 0], tmp_path, y, f"{op}:{fmt}")
    assert p.returncode == 0, p.stderr
    H = np.fromfile(fout, dtype=np.complex64).reshape(B, R, T * L)
    codes, scales = oracle.quantize(y, name)
    x = oracle.dequantize(codes, scales, name, N)
    assert perr(H, oracle.correlate(x, oracle.mseq(8), T * L)) <= 1e-5


@pytest.mark.parametrize("op", ["refine", "refinena"])
def test_c_client_refine(tmp_path, op):
    N, T, L, R, B = SMALL
    y = synth.gaussian((B, R, N), 44).astype(np.complex64)
    p, fout = _run([N, T, L, R, B, 1, 0, 0], tmp_path, y, f"{op}:3")
    assert p.returncode == 0, p.stderr
    X = np.fromfile(fout, dtype=np.complex64).reshape(B, R, T * L)
    its = oracle.refine(y.astype(np.complex128), oracle.mseq(8), T * L, 3)
    assert perr(X, its[3]) <= 1e-5


@pytest.mark.parametrize("chunk", [1, 2, 8])
def test_c_client_estimate_from_host(tmp_path, chunk):
    """pnce_estimate_host from page-locked memory on a second stream, raw
    blocks with a 16-sample prefix, 5 frames in chunks (the last ragged)."""
    N, T, L, R, B, cp = 255, 4, 16, 40, 5, 16
    yr = synth.gaussian((B, R, cp + N), 44).astype(np.complex64)
    p, fout = _run([N, T, L, R, B, 1, 0, 0], tmp_path, yr, f"host:{chunk}:{cp}")
    assert p.returncode == 0, p.stderr
    H = np.fromfile(fout, dtype=np.complex64).reshape(B, R, T * L)
    assert perr(H, oracle.correlate(yr[..., cp:].astype(np.complex128), oracle.mseq(8),
                                    T * L)) <= 1e-5

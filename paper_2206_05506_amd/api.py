"""Tensor-level wrapper of libpnce.so for PyTorch-ROCm callers.

Each method checks shapes, dtypes and devices, then passes raw device
pointers and the current HIP stream to the C entry point of the same name.
All arithmetic runs in the library's kernels; nothing here computes.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from ._lib import (PNCE_FMT_BF16, PNCE_FMT_E4M3, PNCE_FMT_F16, PNCE_PREC_BF16,
                   PNCE_PREC_EXACT, PNCE_PREC_EXACT32, PNCE_PREC_F32, PNCE_PREC_F32S,
                   PNCE_PREC_F64, PNCE_PREC_F64ACC,
                   PNCE_W_LAG_ALIAS)

PRECISIONS = {"f32": PNCE_PREC_F32, "f32s": PNCE_PREC_F32S, "bf16": PNCE_PREC_BF16,
              "f64": PNCE_PREC_F64, "f64acc": PNCE_PREC_F64ACC, "exact": PNCE_PREC_EXACT,
              "exact32": PNCE_PREC_EXACT32}
FORMATS = {"bf16": PNCE_FMT_BF16, "f16": PNCE_FMT_F16, "e4m3": PNCE_FMT_E4M3}
_CODE_DTYPE = {"bf16": torch.int16, "f16": torch.int16, "e4m3": torch.uint8}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else t.data_ptr()


_COPY_STREAMS = {}


def _copy_stream(dev: torch.device):
    """One copy stream per device for host-to-device staging (default
    priority)."""
    if dev.index not in _COPY_STREAMS:
        _COPY_STREAMS[dev.index] = torch.cuda.Stream(device=dev)
    return _COPY_STREAMS[dev.index]


def _need_host(t: torch.Tensor, shape, dtype, name):
    if not isinstance(t, torch.Tensor) or t.is_cuda:
        raise ValueError(f"{name} must be a host tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _need(t: torch.Tensor, shape, dtype, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.is_conj() or t.is_neg():
        # a lazily conjugated or negated view: its memory holds the other values
        raise ValueError(f"{name} is a conjugate or negative view; call .resolve_conj() / "
                         ".resolve_neg() first")


SPACINGS = {"adjacent": _lib.PNCE_LAGS_ADJACENT, "eq8": _lib.PNCE_LAGS_EQ8}


class Plan:
    """A plan for sequence length N, T transmitters, L taps, R antennas.

    feedback: taps of another primitive feedback polynomial (0: the built-in
    one), i.e. another cell's m-sequence; spacing: "adjacent" (transmitter t
    at lags t*L + l) or "eq8" (lags floor(N/T)*t + l, Eq. 8).
    """

    def __init__(self, N: int, T: int, L: int, R: int, feedback: int = 0,
                 spacing: str = "adjacent"):
        if spacing not in SPACINGS:
            raise ValueError(f"spacing must be one of {sorted(SPACINGS)}")
        self.handle, self.status = _lib.pnce_create_ex(N, T, L, R, int(feedback),
                                                       SPACINGS[spacing])
        self.N, self.T, self.L, self.R = N, T, L, R
        self.K = T * L
        self.spacing = spacing
        self.lag_alias = self.status == PNCE_W_LAG_ALIAS

    def close(self):
        if self.handle:
            _lib.pnce_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- a1
    def sequence(self) -> np.ndarray:
        s = np.zeros(self.N, dtype=np.int8)
        _lib.pnce_get_sequence(self.handle, s.ctypes.data)
        return s

    def lags(self) -> np.ndarray:
        """Lag of every column of H, int32 [T*L]."""
        k = np.zeros(self.K, dtype=np.int32)
        _lib.pnce_get_lags(self.handle, k.ctypes.data)
        return k

    def feedback(self) -> int:
        return _lib.pnce_get_feedback(self.handle)

    # ---------------------------------------------------------------- a4
    def estimate(self, Y: torch.Tensor, precision: str = "f32s", out=None,
                 scales=None, beta: float = 0.0, alpha=None) -> torch.Tensor:
        """H = alpha * scales_b * (Y P) + beta H with alpha = 1/N by default
        (the correlator); Y [B, R, N] complex64 (complex128 for precision
        'f64'). Returns H [B, R, T*L]."""
        prec = PRECISIONS[precision]
        cdt = torch.complex128 if prec == PNCE_PREC_F64 else torch.complex64
        B = Y.shape[0]
        _need(Y, (B, self.R, self.N), cdt, "Y")
        if out is None:
            out = torch.empty((B, self.R, self.K), dtype=cdt, device=Y.device)
        _need(out, (B, self.R, self.K), cdt, "H")
        if scales is not None:
            _need(scales, (B,), torch.float32, "scales")
        a = 1.0 / self.N if alpha is None else float(alpha)
        _lib.pnce_estimate(self.handle, _stream(), _ptr(Y), _ptr(out), B, prec, a,
                           _ptr(scales), float(beta))
        return out

    def debias(self, H: torch.Tensor) -> torch.Tensor:
        """Least-squares CIRs from correlator outputs, in place:
        H <- N/(N+1) (H + sum_k H[k] / (N+1-T*L)) per row (needs T*L <= N)."""
        B = H.shape[0]
        _need(H, (B, self.R, self.K), torch.complex64, "H")
        _lib.pnce_debias(self.handle, _stream(), _ptr(H), B)
        return H

    def estimate_ls(self, Y: torch.Tensor, precision: str = "f32s", out=None,
                    scales=None) -> torch.Tensor:
        """Correlation followed by the least-squares correction (fused into the
        correlator's epilogue when one workgroup holds a row's lags)."""
        prec = PRECISIONS[precision]
        B = Y.shape[0]
        _need(Y, (B, self.R, self.N), torch.complex64, "Y")
        if out is None:
            out = torch.empty((B, self.R, self.K), dtype=torch.complex64, device=Y.device)
        _need(out, (B, self.R, self.K), torch.complex64, "H")
        if scales is not None:
            _need(scales, (B,), torch.float32, "scales")
        _lib.pnce_estimate_ls(self.handle, _stream(), _ptr(Y), _ptr(out), B, prec,
                              _ptr(scales))
        return out

    # ---------------------------------------------------------------- a3
    def pack(self, Y: torch.Tensor, fmt: str = "bf16", out=None, scales=None, work=None):
        """Quantise Y [B, R, N] complex64 -> (codes [B, R, 2, N+1], scales [B]),
        every frame read from HBM once (pnce_pack_ws; work: an int32 device
        tensor of at least 1024 B + 1 words, allocated here when None)."""
        return self.pack_cp(Y, 0, fmt, out=out, scales=scales, work=work)

    def pack_two_pass(self, Y: torch.Tensor, fmt: str = "bf16", out=None, scales=None):
        """pnce_pack: the same codes and scales without a workspace (frames
        above 1 MiB are then read twice: a max pass, a conversion pass)."""
        B = Y.shape[0]
        _need(Y, (B, self.R, self.N), torch.complex64, "Y")
        out, scales = self._pack_outputs(B, fmt, out, scales, Y.device)
        _lib.pnce_pack(self.handle, _stream(), _ptr(Y), _ptr(out), _ptr(scales), B,
                       FORMATS[fmt])
        return out, scales

    def _pack_outputs(self, B, fmt, out, scales, device):
        if out is None:
            out = torch.empty((B, self.R, 2, self.N + 1), dtype=_CODE_DTYPE[fmt], device=device)
        if scales is None:
            scales = torch.empty((B,), dtype=torch.float32, device=device)
        _need(out, (B, self.R, 2, self.N + 1), _CODE_DTYPE[fmt], "Yq")
        _need(scales, (B,), torch.float32, "scales")
        return out, scales

    # ------------------------------------------------------ front end
    def estimate_cp(self, Y_raw: torch.Tensor, cp: int, precision: str = "f32s", out=None,
                    scales=None) -> torch.Tensor:
        """Correlation of raw blocks Y_raw [B, R, cp + N] whose first cp
        samples per row are the cyclic prefix (removed by addressing)."""
        prec = PRECISIONS[precision]
        cdt = torch.complex128 if prec == PNCE_PREC_F64 else torch.complex64
        B = Y_raw.shape[0]
        _need(Y_raw, (B, self.R, self.N + cp), cdt, "Y_raw")
        if out is None:
            out = torch.empty((B, self.R, self.K), dtype=cdt, device=Y_raw.device)
        _need(out, (B, self.R, self.K), cdt, "H")
        if scales is not None:
            _need(scales, (B,), torch.float32, "scales")
        _lib.pnce_estimate_cp(self.handle, _stream(), _ptr(Y_raw), int(cp), _ptr(out), B, prec,
                              _ptr(scales))
        return out

    def pack_cp(self, Y_raw: torch.Tensor, cp: int, fmt: str = "bf16", out=None, scales=None,
                work=None):
        """Quantise raw blocks Y_raw [B, R, cp + N], dropping the cyclic prefix
        in the same launch: (codes [B, R, 2, N+1], scales [B]); every frame is
        read from HBM once (pnce_pack_ws)."""
        B = Y_raw.shape[0]
        _need(Y_raw, (B, self.R, self.N + cp), torch.complex64, "Y_raw")
        out, scales = self._pack_outputs(B, fmt, out, scales, Y_raw.device)
        nbytes = _lib.pack_work_bytes(B)
        if work is None:
            work = torch.empty(((nbytes + 3) // 4,), dtype=torch.int32, device=Y_raw.device)
        _need(work, (work.numel(),), torch.int32, "work")
        if work.numel() * 4 < nbytes:
            raise ValueError(f"work holds {work.numel()} words, {(nbytes + 3) // 4} needed")
        _lib.pnce_pack_ws(self.handle, _stream(), _ptr(Y_raw), int(cp), _ptr(out), _ptr(scales),
                          B, FORMATS[fmt], _ptr(work), work.numel() * 4)
        return out, scales

    def pack_cp_two_pass(self, Y_raw: torch.Tensor, cp: int, fmt: str = "bf16", out=None,
                         scales=None):
        """pnce_pack_cp: as pack_cp without a workspace."""
        B = Y_raw.shape[0]
        _need(Y_raw, (B, self.R, self.N + cp), torch.complex64, "Y_raw")
        out, scales = self._pack_outputs(B, fmt, out, scales, Y_raw.device)
        _lib.pnce_pack_cp(self.handle, _stream(), _ptr(Y_raw), int(cp), _ptr(out),
                          _ptr(scales), B, FORMATS[fmt])
        return out, scales

    def stream_from_host(self, Y_host: torch.Tensor, cp: int, chunk: int,
                         precision: str = "bf16", out=None, copy_stream=None,
                         staging=None) -> torch.Tensor:
        """pnce_estimate_host: raw blocks in pinned host memory
        (Y_host [F, R, cp + N] complex64, complex128 for "f64") are copied to
        the device in chunks of `chunk` frames on copy_stream (default: one
        library-held stream per device) while the previous chunk is estimated
        on the current stream. Returns H [F, R, T*L] on the device; the
        current stream carries the last estimate, and Y_host must stay
        unchanged until it has run. A caller that streams repeatedly should
        pass the same `staging` buffer (uint8, at least
        host_staging_bytes(...) bytes) to every call rather than let each
        call allocate one."""
        if int(chunk) < 1:
            raise ValueError("chunk must be >= 1")
        prec = PRECISIONS[precision]
        cdt = torch.complex128 if prec == PNCE_PREC_F64 else torch.complex64
        F = Y_host.shape[0]
        _need_host(Y_host, (F, self.R, self.N + cp), cdt, "Y_host")
        if F > 0 and not Y_host.is_pinned():   # (an empty tensor cannot be pinned)
            raise ValueError("Y_host must be in pinned host memory")
        dev = torch.device("cuda", torch.cuda.current_device())
        if out is None:
            out = torch.empty((F, self.R, self.K), dtype=cdt, device=dev)
        _need(out, (F, self.R, self.K), cdt, "H")
        per = max(1, min(int(chunk), F))
        nbytes = _lib.host_staging_bytes(self.R, self.N, cp, per, prec)
        if staging is None:
            # Taken from the current stream's pool: the library orders every
            # copy after the work already queued on this stream and this
            # stream after every copy, so the block is free for this stream
            # again once the call's estimates have run.
            staging = torch.empty((nbytes,), dtype=torch.uint8, device=dev)
        if staging.device != dev or staging.numel() * staging.element_size() < nbytes:
            raise ValueError(f"staging must hold {nbytes} bytes on {dev}")
        if copy_stream is None:
            copy_stream = _copy_stream(dev)
        _lib.pnce_estimate_host(self.handle, _stream(), copy_stream.cuda_stream, _ptr(Y_host),
                                int(cp), _ptr(out), F, int(chunk), prec, _ptr(staging),
                                staging.numel() * staging.element_size())
        return out

    def estimate_packed(self, Yq: torch.Tensor, scales, fmt: str = "bf16", out=None,
                        beta: float = 0.0) -> torch.Tensor:
        B = Yq.shape[0]
        _need(Yq, (B, self.R, 2, self.N + 1), _CODE_DTYPE[fmt], "Yq")
        if scales is not None:
            _need(scales, (B,), torch.float32, "scales")
        if out is None:
            out = torch.empty((B, self.R, self.K), dtype=torch.complex64, device=Yq.device)
        _need(out, (B, self.R, self.K), torch.complex64, "H")
        _lib.pnce_estimate_packed(self.handle, _stream(), _ptr(Yq), _ptr(scales), _ptr(out),
                                  B, FORMATS[fmt], float(beta))
        return out

    # ---------------------------------------------------------------- a7
    def adjoint(self, G: torch.Tensor, precision: str = "f32s", alpha=None, beta=0.0,
                C=None, out=None) -> torch.Tensor:
        """A = alpha G P^T + beta C (alpha defaults to 1/N: the transpose of
        estimate). G [B, R, T*L] -> A [B, R, N]."""
        prec = PRECISIONS[precision]
        cdt = torch.complex128 if prec == PNCE_PREC_F64 else torch.complex64
        B = G.shape[0]
        _need(G, (B, self.R, self.K), cdt, "G")
        if out is None:
            out = torch.empty((B, self.R, self.N), dtype=cdt, device=G.device)
        _need(out, (B, self.R, self.N), cdt, "A")
        if C is not None:
            _need(C, (B, self.R, self.N), cdt, "C")
        a = 1.0 / self.N if alpha is None else float(alpha)
        _lib.pnce_adjoint(self.handle, _stream(), _ptr(G), _ptr(out), _ptr(C), B, prec, a,
                          float(beta))
        return out

    # ---------------------------------------------------------------- a6
    def refine(self, y: torch.Tensor, X: torch.Tensor, steps: int, work=None) -> torch.Tensor:
        """In place: `steps` LS refinement steps of X from the c64 frames y."""
        B = y.shape[0]
        _need(y, (B, self.R, self.N), torch.complex64, "y")
        _need(X, (B, self.R, self.K), torch.complex64, "X")
        if steps > 0:
            if work is None:
                work = torch.empty((B, self.R, self.N), dtype=torch.complex64, device=y.device)
            _need(work, (B, self.R, self.N), torch.complex64, "work")
        _lib.pnce_refine(self.handle, _stream(), _ptr(y), _ptr(X), _ptr(work), B, steps)
        return X

    def refine_noalloc(self, y: torch.Tensor, X: torch.Tensor, steps: int) -> torch.Tensor:
        """In place, as refine, with the residual in the library's fixed
        device array (no allocation; calls overlapping on one GPU race)."""
        B = y.shape[0]
        _need(y, (B, self.R, self.N), torch.complex64, "y")
        _need(X, (B, self.R, self.K), torch.complex64, "X")
        _lib.pnce_refine_noalloc(self.handle, _stream(), _ptr(y), _ptr(X), B, steps)
        return X


class VarlenPlan:
    """Uneven batch: frames with their own (R, N, T, L) in one buffer of
    planar codes ([R][2][N+1] per frame) and one buffer of complex64 CIRs
    ([R][T*L] per frame), estimated by one persistent launch."""

    def __init__(self, shapes, fmt: str = "bf16"):
        """shapes: iterable of (R, N, T, L). Offsets are laid out back to back."""
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.fmt = fmt
        y_off, h_off = [], []
        yo = ho = 0
        for R, N, T, L in self.shapes:
            y_off.append(yo)
            h_off.append(ho)
            yo += R * 2 * (N + 1)
            ho += R * T * L
        self.y_off, self.h_off = y_off, h_off
        self.n_codes, self.n_out = yo, ho
        frames = [(R, N, T, L, y_off[i], h_off[i]) for i, (R, N, T, L) in enumerate(self.shapes)]
        self.handle, self.status = _lib.pnce_varlen_create(frames, FORMATS[fmt])

    def close(self):
        if self.handle:
            _lib.pnce_varlen_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, Yq, scales, H):
        _need(Yq, (self.n_codes,), torch.int16, "Yq")
        _need(H, (self.n_out,), torch.complex64, "H")
        if scales is not None:
            _need(scales, (len(self.shapes),), torch.float32, "scales")

    def estimate(self, Yq, scales=None, out=None):
        if out is None:
            out = torch.empty((self.n_out,), dtype=torch.complex64, device=Yq.device)
        self._check(Yq, scales, out)
        _lib.pnce_varlen_estimate(self.handle, _stream(), _ptr(Yq), _ptr(scales), _ptr(out))
        return out

    def estimate_each(self, Yq, scales=None, out=None):
        if out is None:
            out = torch.empty((self.n_out,), dtype=torch.complex64, device=Yq.device)
        self._check(Yq, scales, out)
        _lib.pnce_varlen_estimate_each(self.handle, _stream(), _ptr(Yq), _ptr(scales),
                                       _ptr(out))
        return out

    def tune(self, Yq, scales=None, out=None, reps: int = 5):
        if out is None:
            out = torch.empty((self.n_out,), dtype=torch.complex64, device=Yq.device)
        self._check(Yq, scales, out)
        _lib.pnce_varlen_tune(self.handle, _stream(), _ptr(Yq), _ptr(scales), _ptr(out), reps)
        return self.tuning()

    def tuning(self):
        return _lib.pnce_varlen_get_tuning(self.handle)

    def set_tuning(self, entries):
        _lib.pnce_varlen_set_tuning(self.handle, entries)

    def stats(self):
        return _lib.pnce_varlen_stats(self.handle)

    def frame_view(self, H, f):
        """CIRs of frame f as [R, T, L] (the de-multiplexed view of Eq. 10)."""
        R, N, T, L = self.shapes[f]
        return H[self.h_off[f]:self.h_off[f] + R * T * L].view(R, T, L)

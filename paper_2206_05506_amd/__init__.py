"""PN-sequence correlation channel estimation for multiplexed pilots on
AMD Instinct MI355X (gfx950), after arXiv 2206.05506.

    from paper_2206_05506_amd import Plan
    plan = Plan(N=1023, T=16, L=32, R=64)
    H = plan.estimate(Y)            # Y [B, R, N] complex64 on the GPU
    h = H.view(B, R, T, L)          # per-transmitter CIRs (Eq. 10)

Every computation runs in libpnce.so (HIP kernels); this package only
marshals arguments. It raises ImportError when the library is not built.
"""
# torch first: its HIP runtime must be the one in the process before
# libpnce.so is loaded (libpnce.so then binds to it instead of bringing a
# second copy of the runtime, which would not see the device torch holds).
import torch  # noqa: F401

from . import _lib
from ._lib import PnceError
from .api import FORMATS, PRECISIONS, Plan, VarlenPlan

__all__ = ["Plan", "VarlenPlan", "PnceError", "PRECISIONS", "FORMATS", "_lib"]

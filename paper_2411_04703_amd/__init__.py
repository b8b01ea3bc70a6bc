"""MI355X boosted-frame PIC hot path: HIP kernels behind a C-ABI (include/pic.h).

``abi`` mirrors the C-ABI with ctypes, ``sim.Sim`` owns one context whose
device memory is a torch tensor, ``autograd`` wraps the hand-written adjoint.
"""
from . import abi  # noqa: F401

__all__ = ["abi"]

"""MI355X-native unigrid FMM Poisson solver (isolated boundary conditions).

The solver is a HIP library with a C ABI (``include/fmm.h``); this package
holds its sources (``csrc/``), the build step (``build.py``) and a ctypes
binding with a ``torch.autograd.Function`` front (``fmm.py``).
"""
from .fmm import FmmError, Plan, multi_index, solve  # noqa: F401

__all__ = ["Plan", "solve", "multi_index", "FmmError"]

"""Batched macroscopic cross-section lookup on the AMD MI355X (gfx950).

The lookup runs in hand-written HIP kernels inside libxs.so, behind the C
interface of include/xs.h; `xs` is a ctypes binding with the same names.
"""
from .xs import *  # noqa: F401,F403
from .xs import load_library, declared_functions, XsError, Tables  # noqa: F401

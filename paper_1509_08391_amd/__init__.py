"""MI355X (gfx950) implementation of the LLR density-of-states method for 4D
compact U(1) lattice gauge theory (arXiv:1509.08391): HIP kernels behind the
C ABI of include/llr.h, with a thin ctypes binding in ``llr``."""
from . import llr  # noqa: F401
from .llr import Context, FP32, FP64, LLRError  # noqa: F401

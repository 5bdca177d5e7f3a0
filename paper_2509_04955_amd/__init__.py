"""MI355X (gfx950) full-amplitude state-vector simulator: fused-gate hot path.

The compute lives in libqsim.so (HIP kernels behind the C ABI of
include/qsim.h); ``qsim`` is its thin ctypes binding.
"""
from . import qsim  # noqa: F401

"""MI355X (gfx950) implementation of the iSIRA hot path (arXiv 1710.07080).

The compute path is libisira.so (hand-written HIP kernels behind the C ABI in
include/isira.h); ``isira`` is its ctypes binding.
"""
from . import isira  # noqa: F401
from .isira import Context, IsiraError, load, symeig  # noqa: F401

"""MI355X (gfx950) iterative-sketching least-squares solver.

The work happens in libls.so (HIP kernels behind the C ABI of include/ls.h); ``ls`` is its ctypes
binding.
"""
from . import ls  # noqa: F401
from .ls import Context, LSError, limits  # noqa: F401

"""MI355X (gfx950) hot path of neural dependence fields.

The compute lives in libndf.so (hand-written HIP kernels behind the C ABI of
include/ndf.h); ``paper_2307_02203_amd.ndf`` is its thin ctypes binding.
"""
from . import ndf  # noqa: F401

"""lmtof: list-mode TOF-weighted MLEM for AMD Instinct MI355X (gfx950).

The compute path is liblmtof.so (hand-written HIP kernels behind a C ABI,
include/lmtof.h); ``lmtof`` is its thin ctypes binding.
"""
from . import lmtof  # noqa: F401  (fails loudly if the library is not built)
from .lmtof import LmtofError, Reconstruction  # noqa: F401

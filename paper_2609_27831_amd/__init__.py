"""MI355X (gfx950) implementation of the Ozaki scheme II p-bit matrix product.

The product path is the C-ABI library liboz2h.so (include/oz2h.h) built from
csrc/ with hipcc; `oz2h` is its ctypes binding.
"""
from . import oz2h  # noqa: F401

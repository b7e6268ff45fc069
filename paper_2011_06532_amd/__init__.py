"""TT arithmetic and TT rounding on AMD MI355X (gfx950).

The compute path is the HIP library ``libttr.so`` (C ABI in ``include/ttr.h``);
``paper_2011_06532_amd.ttr`` is its Python binding.  There is no CPU fallback:
if the library is missing, loading it raises.
"""
from . import ttr  # noqa: F401

__all__ = ["ttr"]

"""MI355X (gfx950) implementation of the data-parallel scoring path of the
optimisation-suggestion tool of Taheri, Qasem and Burtscher (Section 2:
profile features, per-optimisation speedup models, ranking above a
threshold).  The kernels live in libsugg.so (C ABI: include/sugg.h); this
package is its Python binding.
"""
from . import _abi  # noqa: F401

__all__ = ["plain", "build"]

"""ofks: orthogonalization-free Kohn-Sham block solver for MI355X (gfx950).

The PCAL iteration of Gao, Hu, Kuang & Liu (arXiv 2007.14228) on P1 finite
elements, as hand-written HIP kernels behind a C ABI (include/ofks.h,
libofks.so).  This package is the thin Python binding: ``Solver`` marshals
arguments to the library and nothing else.  It raises ImportError-style
errors when the library has not been built -- there is no CPU fallback.
"""
from ._lib import LIB_PATH, load  # noqa: F401
from .solver import OfksError, Solver  # noqa: F401

__all__ = ["Solver", "OfksError", "load", "LIB_PATH"]

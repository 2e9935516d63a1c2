"""MI355X-native stencil sweeps as 2:4-structured-sparse matrix products.

The work runs in libsparstencil.so (C ABI declared in include/sparstencil.h);
``native`` is its ctypes binding.  Importing this package does not load the
library; the first call does, and fails loudly if it has not been built.
"""
from . import native  # noqa: F401
from .native import Plan, SparStencilError  # noqa: F401

__all__ = ["native", "Plan", "SparStencilError"]

"""MI355X-native interferometric response operator of fast-resolve (arXiv 2406.09144).

The numerical work lives in libfrmi.so (hand-written HIP for gfx950, C ABI in
include/frmi.h); this package is its binding: `_lib` exposes the C functions
under their C names, `api` wraps them for torch GPU tensors (import it as
`from paper_2406_09144_amd import api`; importing the package alone does not
touch torch or the GPU).
"""

from . import _lib  # noqa: F401
from ._lib import FrError, load  # noqa: F401

__all__ = ["FrError", "load"]


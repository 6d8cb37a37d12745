"""Laplacian mesh smoothing for AMD Instinct MI355X (gfx950).

The method is Laplacian mesh smoothing with the reuse-distance-reducing
vertex ordering of Aupy, Park and Raghavan (arXiv 1606.00803).  The library
``liblms.so`` exposes a C ABI (include/lms.h); :mod:`.lms` is its Python
binding.  Build with ``python -m paper_1606_00803_amd.build``.
"""
from .lms import (BFS, FP32, FP64, JACOBI, MULTICOLOR, ORI, RANDOM, RDR,  # noqa: F401
                  LmsError, Mesh, header_functions, load)

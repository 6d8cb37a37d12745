"""Oracle for Laplacian mesh smoothing -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation of what the smoothing
library computes, written from the paper (Aupy, Park, Raghavan, "Locality-
Aware Laplacian Mesh Smoothing", arXiv 1606.00803):

* ``mesh``      -- neighbour sets and fixed vertices (Eq. 1, Algorithm 1);
* ``quality``   -- edge-length-ratio quality per triangle, vertex and mesh
                   (Section 3.2, Algorithm 1);
* ``orderings`` -- ORI, BFS, RDR (Algorithm 2) and random orderings, the
                   permutation helpers and the multicolour schedule;
* ``smooth``    -- float64 sweeps in plain C (``sweep.c``) and the stopping
                   rule of Algorithm 1.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the library it checks: the two
meet only in the seeded input generators of ``meshgen``.

Parity status: every function here is pinned by tests against closed forms,
invariants, brute force or library routines (see tests/test_oracle_*.py),
except the reading of RDR's tie rule and Theorem 1 extension, which is pinned
by hand-traced examples, and ``jacobi_at_vertices``, pinned against the whole
mesh sweep.
"""
from . import mesh, orderings, quality, smooth  # noqa: F401
from .mesh import MeshError, Topology, topology  # noqa: F401

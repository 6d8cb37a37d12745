"""Oracle mesh topology: neighbours, fixed vertices, triangle counts.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of the paper used here:
* The N neighbours of Eq. 1 (Section 3.2) are the distinct vertices that
  share a triangle edge with v; all of them count, fixed ones included, each
  with weight 1/N.
* Algorithm 1 smooths only interior vertices.  A vertex is fixed (not
  interior) when it is an endpoint of a boundary edge, i.e. an edge with
  exactly one incident triangle; a caller may instead pass its own mask (the
  node record of Section 5.2.3's footnote carries a fixed/boundary flag).
"""
from __future__ import annotations

import dataclasses

import numpy as np


class MeshError(ValueError):
    """The triangle list is not a valid 2D triangle mesh."""


@dataclasses.dataclass
class Topology:
    n: int
    tri: np.ndarray          # int64 [T, 3]
    nbr_ptr: np.ndarray      # int64 [n+1]
    nbr: np.ndarray          # int32 [nnz_full]: ascending per vertex
    fixed: np.ndarray        # uint8 [n]
    tcount: np.ndarray       # int64 [n]: number of triangles containing v

    @property
    def interior(self) -> np.ndarray:
        return np.flatnonzero(self.fixed == 0)

    def neighbours(self, v: int) -> np.ndarray:
        return self.nbr[self.nbr_ptr[v]:self.nbr_ptr[v + 1]]

    @property
    def degree(self) -> np.ndarray:
        return np.diff(self.nbr_ptr)


def topology(n: int, tri, fixed=None) -> Topology:
    """Neighbour lists, boundary rule and validity checks from a triangle list."""
    tri = np.asarray(tri, dtype=np.int64).reshape(-1, 3)
    if n <= 0:
        raise MeshError("mesh has no vertices")
    if tri.size and (tri.min() < 0 or tri.max() >= n):
        raise MeshError("triangle refers to a vertex outside [0, n)")
    if np.any((tri[:, 0] == tri[:, 1]) | (tri[:, 1] == tri[:, 2]) | (tri[:, 0] == tri[:, 2])):
        raise MeshError("triangle repeats a vertex")
    tcount = np.bincount(tri.ravel(), minlength=n).astype(np.int64)
    if np.any(tcount == 0):
        raise MeshError("vertex not referenced by any triangle")

    # undirected edges with multiplicity
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    keys, mult = np.unique(lo * n + hi, return_counts=True)
    if np.any(mult > 2):
        raise MeshError("edge shared by more than two triangles")
    a = keys // n
    b = keys % n

    # both directions, sorted by (source, target): ascending neighbour labels
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    nbr_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=nbr_ptr[1:])

    if fixed is None:
        fx = np.zeros(n, dtype=np.uint8)
        bnd = mult == 1
        fx[a[bnd]] = 1
        fx[b[bnd]] = 1
    else:
        fx = (np.asarray(fixed).reshape(n) != 0).astype(np.uint8)
    return Topology(n=n, tri=tri, nbr_ptr=nbr_ptr, nbr=dst.astype(np.int32),
                    fixed=fx, tcount=tcount)


def smoothing_operator_dense(top: Topology) -> np.ndarray:
    """Dense n x n matrix A of one Jacobi sweep, P_{k+1} = A P_k (small meshes only).

    Row v of a free vertex holds 1/N(v) at each neighbour; a fixed vertex's
    row is the unit row.  Built straight from the triangle edges, not from the
    neighbour lists, so it checks those too.
    """
    n = top.n
    adj = np.zeros((n, n), dtype=bool)
    for a, b, c in top.tri:
        for p, q in ((a, b), (b, c), (c, a)):
            adj[p, q] = adj[q, p] = True
    A = np.zeros((n, n), dtype=np.float64)
    for v in range(n):
        if top.fixed[v]:
            A[v, v] = 1.0
        else:
            A[v, adj[v]] = 1.0 / adj[v].sum()
    return A

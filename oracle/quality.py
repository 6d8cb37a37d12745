"""Oracle mesh quality (Section 3.2 and Algorithm 1's quality loop).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Triangle quality is the edge-length ratio: the shortest edge's length
  divided by the longest edge's length, a value in [0, 1], 1 for an
  equilateral triangle.  Lengths are Euclidean: l_e^2 = dx*dx + dy*dy, then
  q_t = sqrt(min l^2) / sqrt(max l^2).  A triangle whose longest edge has
  length 0 gets quality 0.
* Vertex quality q_v is the mean of the qualities of the triangles that
  contain v, summed in ascending triangle index and divided by their count.
* Global quality Q is the mean of q_v over all |V| vertices (Algorithm 1
  sums over i = 1..|V|, boundary vertices included).  The sum is taken
  exactly rounded (math.fsum) and then divided by |V|.

Every step is an elementwise IEEE operation in NumPy (no fused
multiply-add), so q_t and q_v are reproducible bit for bit by any code that
performs the same operations in the same order.
"""
from __future__ import annotations

import math

import numpy as np


def triangle_quality(x, y, tri) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64).reshape(-1, 3)
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]

    def len2(p, q):
        dx = x[q] - x[p]
        dy = y[q] - y[p]
        return dx * dx + dy * dy

    e0 = len2(a, b)
    e1 = len2(b, c)
    e2 = len2(c, a)
    mn = np.minimum(np.minimum(e0, e1), e2)
    mx = np.maximum(np.maximum(e0, e1), e2)
    q = np.zeros(tri.shape[0], dtype=np.float64)
    ok = mx > 0
    q[ok] = np.sqrt(mn[ok]) / np.sqrt(mx[ok])
    return q


def vertex_quality(x, y, tri, n: int) -> np.ndarray:
    """q_v: mean over the triangles containing v (ascending triangle index)."""
    tri = np.asarray(tri, dtype=np.int64).reshape(-1, 3)
    qt = triangle_quality(x, y, tri)
    acc = np.zeros(n, dtype=np.float64)
    # ravel order is t0a, t0b, t0c, t1a, ...: each vertex receives its
    # triangles' values in ascending triangle index (np.add.at is unbuffered
    # and applies the additions in the order given).
    np.add.at(acc, tri.ravel(), np.repeat(qt, 3))
    cnt = np.bincount(tri.ravel(), minlength=n).astype(np.float64)
    return acc / cnt


def global_quality(x, y, tri, n: int) -> float:
    """Q = (1/|V|) sum_v q_v over all vertices."""
    qv = vertex_quality(x, y, tri, n)
    return math.fsum(qv.tolist()) / n

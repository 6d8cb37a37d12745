"""Oracle locality profile of an ordering (Section 2, "Reuse distance and
cache misses"; the quantiles of Table 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings (the paper measures a verbose run of its own code; it does not
spell the trace out):

* The trace is one Jacobi sweep in storage order: for every free vertex, in
  ascending current label, the vertex itself and then its neighbours in
  ascending current label.  Items are current labels (storage positions);
  fixed vertices are read as neighbours only.
* The second trace follows Algorithm 1's loop body, which smooths V[i] and
  then updates the global quality: after each vertex's neighbours come the
  triangles containing it (their corners, then their quality record).
* The reuse distance of an access to x is the number of distinct items
  accessed strictly between it and the previous access to x.  A first access
  has none; it is counted apart as cold.
* The X quantile is the smallest value d such that at least a fraction X of
  the (non-cold) distances are <= d.
* Cache-line span of a wavefront (the GPU reading of spatial locality): the
  number of distinct lines of `line_bytes` bytes, holding records of
  `record_bytes` bytes stored by current label, that the neighbour reads of 64
  consecutive rows touch.  Waves without a free row are skipped.

Parity unpinned against Table 2 (its meshes are not available); the tests pin
these functions by brute force on small traces and by hand-worked examples.
"""
from __future__ import annotations

import math

import numpy as np

from .mesh import Topology


def sweep_trace(top: Topology, new2old) -> np.ndarray:
    """Access trace (current labels) of one sweep in storage order."""
    new2old = np.asarray(new2old, dtype=np.int64)
    n = top.n
    old2new = np.empty(n, dtype=np.int64)
    old2new[new2old] = np.arange(n)
    out = []
    for k in range(n):
        v = int(new2old[k])
        if top.fixed[v]:
            continue
        out.append(k)
        nb = sorted(int(old2new[u]) for u in top.neighbours(v))
        out.extend(nb)
    return np.asarray(out, dtype=np.int64)


def triangle_rank(tri, new2old) -> np.ndarray:
    """Storage index of each input triangle under an ordering: triangles sorted
    by (smallest new label of a corner, input index)."""
    tri = np.asarray(tri, dtype=np.int64).reshape(-1, 3)
    new2old = np.asarray(new2old, dtype=np.int64)
    old2new = np.empty(new2old.size, dtype=np.int64)
    old2new[new2old] = np.arange(new2old.size)
    key = old2new[tri].min(axis=1)
    order = sorted(range(tri.shape[0]), key=lambda i: (int(key[i]), i))
    rank = np.empty(tri.shape[0], dtype=np.int64)
    rank[np.asarray(order, dtype=np.int64)] = np.arange(tri.shape[0])
    return rank


def algorithm1_trace(top: Topology, new2old) -> np.ndarray:
    """Access trace of Algorithm 1's loop body over the free vertices in
    storage order: smoothing V[i] reads the vertex and its neighbours (as in
    sweep_trace); updating the global quality then recomputes every triangle
    containing it, in ascending storage index, reading its three corners in
    ascending current label and writing the triangle's quality record.  Items
    are current labels 0..n-1 and triangle records n + storage index."""
    new2old = np.asarray(new2old, dtype=np.int64)
    n = top.n
    old2new = np.empty(n, dtype=np.int64)
    old2new[new2old] = np.arange(n)
    tri = np.asarray(top.tri, dtype=np.int64).reshape(-1, 3)
    rank = triangle_rank(tri, new2old)
    of_vertex = [[] for _ in range(n)]          # input vertex -> its triangles (input indices)
    for i, (a, b, c) in enumerate(tri.tolist()):
        for v in (a, b, c):
            of_vertex[v].append(i)
    out = []
    for k in range(n):
        v = int(new2old[k])
        if top.fixed[v]:
            continue
        out.append(k)
        out.extend(sorted(int(old2new[u]) for u in top.neighbours(v)))
        for i in sorted(of_vertex[v], key=lambda i: int(rank[i])):
            out.extend(sorted(int(old2new[u]) for u in tri[i]))
            out.append(n + int(rank[i]))
    return np.asarray(out, dtype=np.int64)


def reuse_distances(trace) -> tuple[np.ndarray, int]:
    """Distances of the non-cold accesses (in trace order) and the cold count,
    by an LRU stack: the distance is the item's depth in the stack of items
    ordered by last access (Mattson et al., 1970)."""
    stack: list[int] = []          # most recent last
    out = []
    cold = 0
    for x in np.asarray(trace).tolist():
        try:
            i = stack.index(x)
        except ValueError:
            cold += 1
            stack.append(x)
            continue
        out.append(len(stack) - 1 - i)
        del stack[i]
        stack.append(x)
    return np.asarray(out, dtype=np.int64), cold


def reuse_distances_brute(trace) -> tuple[np.ndarray, int]:
    """The definition written out: distinct items strictly between two
    accesses to the same item (quadratic; tiny traces only)."""
    trace = np.asarray(trace).tolist()
    last: dict[int, int] = {}
    out = []
    cold = 0
    for t, x in enumerate(trace):
        if x in last:
            out.append(len(set(trace[last[x] + 1:t])))
        else:
            cold += 1
        last[x] = t
    return np.asarray(out, dtype=np.int64), cold


def quantile(d, x: float) -> int:
    """Smallest value v with at least a fraction x of d at or below v."""
    d = np.sort(np.asarray(d, dtype=np.int64))
    if d.size == 0:
        return 0
    need = max(1, math.ceil(x * d.size - 1e-12))
    return int(d[need - 1])


def wave_line_spans(top: Topology, new2old, line_bytes: int = 128, record_bytes: int = 16,
                    wave: int = 64) -> np.ndarray:
    """Distinct cache lines touched by the neighbour reads of each wavefront
    of `wave` consecutive rows (waves with no free row are skipped)."""
    new2old = np.asarray(new2old, dtype=np.int64)
    n = top.n
    old2new = np.empty(n, dtype=np.int64)
    old2new[new2old] = np.arange(n)
    spans = []
    for w0 in range(0, n, wave):
        lines = set()
        any_free = False
        for k in range(w0, min(n, w0 + wave)):
            v = int(new2old[k])
            if top.fixed[v]:
                continue
            any_free = True
            for u in top.neighbours(v):
                lines.add((int(old2new[u]) * record_bytes) // line_bytes)
        if any_free:
            spans.append(len(lines))
    return np.asarray(spans, dtype=np.int64)


def profile(top: Topology, new2old, fractions=(0.5, 0.75, 0.9, 1.0), line_bytes: int = 128,
            record_bytes: int = 16, trace: str = "sweep") -> dict:
    tr = sweep_trace(top, new2old) if trace == "sweep" else algorithm1_trace(top, new2old)
    d, cold = reuse_distances(tr)
    spans = wave_line_spans(top, new2old, line_bytes, record_bytes)
    return dict(accesses=int(tr.size), cold=cold,
                quantiles=[quantile(d, f) for f in fractions],
                mean=float(d.mean()) if d.size else 0.0, max=int(d.max()) if d.size else 0,
                lines_per_wave=float(spans.mean()) if spans.size else 0.0,
                max_lines_per_wave=int(spans.max()) if spans.size else 0)

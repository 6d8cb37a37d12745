"""Oracle vertex orderings, permutations and the multicolour schedule.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An ordering is returned as ``new2old``: position k of the reordered mesh
holds old vertex new2old[k] (Algorithm 2 fills V_new[next_num] with V[i]).

* ORI    -- the generator's own order (identity), Section 5.2.1.
* BFS    -- breadth-first search (the Strout-Hovland baseline, Sections 1
            and 5.2.1).  The paper does not fix its details; the reading
            used: start at label 0, visit neighbours in ascending label,
            restart at the smallest unvisited label when a component ends,
            no reversal.
* RDR    -- Algorithm 2 (Section 4.2), read as follows:
            - "sorted by increasing quality": ascending (q_v, label);
            - l[0] is the first element of l, the neighbour of worst quality
              (the loop over l visits every element);
            - l holds the *unprocessed* neighbours (sorted or not); only the
              not-yet-sorted ones are appended; the walk may step onto
              fixed vertices;
            - Theorem 1 holds only for vertices adjacent to an interior
              vertex or reached by a walk: a fixed vertex whose neighbours
              are all fixed and never walked onto is left out by the loop as
              printed.  After the loop over interior vertices the same loop
              body therefore continues over the remaining fixed vertices in
              ascending (q_v, label); on a mesh where the printed loop
              already ordered every vertex this appends nothing.
* RANDOM -- a uniform permutation: Fisher-Yates driven by SplitMix64
            (Steele, Lea & Flood, OOPSLA 2014) seeded with ``seed``; for
            i = n-1 down to 1, j = next() mod (i+1), swap(perm[i], perm[j]),
            starting from the identity.

Multicolour schedule (used when sweeps update in place): greedy first-fit
colouring of the graph induced on the free vertices, visiting them in
ascending input label and giving each the smallest colour not used by an
already coloured free neighbour.  Colours belong to vertices, so the
schedule does not depend on the storage ordering.
"""
from __future__ import annotations

import collections

import numpy as np

from .mesh import Topology

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 from its published definition (64-bit state, Weyl increment)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)


def ori(top: Topology) -> np.ndarray:
    return np.arange(top.n, dtype=np.int32)


def random_order(n: int, seed: int) -> np.ndarray:
    perm = list(range(n))
    g = SplitMix64(seed)
    for i in range(n - 1, 0, -1):
        j = g.next() % (i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    return np.array(perm, dtype=np.int32)


def bfs(top: Topology) -> np.ndarray:
    n = top.n
    seen = np.zeros(n, dtype=bool)
    out = []
    for s in range(n):
        if seen[s]:
            continue
        seen[s] = True
        q = collections.deque([s])
        while q:
            v = q.popleft()
            out.append(v)
            for u in top.neighbours(v).tolist():
                if not seen[u]:
                    seen[u] = True
                    q.append(u)
    return np.array(out, dtype=np.int32)


def rdr(top: Topology, q, extend: bool = True) -> np.ndarray:
    """Reuse Distance Reducing ordering (Algorithm 2) from vertex qualities q.

    With ``extend=False`` the loop runs over interior vertices only, exactly as
    printed; the result may then miss vertices (see the module docstring).
    """
    n = top.n
    q = np.asarray(q, dtype=np.float64)
    qs = q.tolist()
    nbrs = [top.neighbours(v).tolist() for v in range(n)]
    processed = [False] * n
    placed = [False] * n          # Algorithm 2's "sorted" array
    out = []

    def by_quality(vs):
        return sorted(vs, key=lambda v: (qs[v], v))

    def place(v):
        if not placed[v]:
            out.append(v)
            placed[v] = True

    def start_from(i):
        if processed[i]:
            return
        place(i)
        processed[i] = True
        cur = by_quality([u for u in nbrs[i] if not processed[u]])
        while cur:
            for u in cur:
                place(u)
            w = cur[0]
            processed[w] = True
            cur = by_quality([u for u in nbrs[w] if not processed[u]])

    interior = [v for v in range(n) if not top.fixed[v]]
    for i in by_quality(interior):
        start_from(i)
    if extend:
        for i in by_quality([v for v in range(n) if top.fixed[v]]):
            start_from(i)
    return np.array(out, dtype=np.int32)


def inverse(new2old) -> np.ndarray:
    new2old = np.asarray(new2old, dtype=np.int64)
    old2new = np.empty_like(new2old)
    old2new[new2old] = np.arange(new2old.size)
    return old2new.astype(np.int32)


def is_permutation(p, n: int) -> bool:
    p = np.asarray(p)
    return p.size == n and np.array_equal(np.sort(p), np.arange(n))


def greedy_colouring(top: Topology) -> np.ndarray:
    """Colour per vertex (-1 for fixed vertices)."""
    n = top.n
    colour = [-1] * n
    fixed = top.fixed.tolist()
    for v in range(n):
        if fixed[v]:
            continue
        used = {colour[u] for u in top.neighbours(v).tolist() if colour[u] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[v] = c
    return np.array(colour, dtype=np.int32)


def colour_lists(colour) -> tuple[np.ndarray, np.ndarray]:
    """(colour_ptr int64[C+1], colour_list int32): vertices of each colour, ascending."""
    colour = np.asarray(colour)
    C = int(colour.max()) + 1 if colour.size and colour.max() >= 0 else 0
    ptr = np.zeros(C + 1, dtype=np.int64)
    lists = []
    for c in range(C):
        vs = np.flatnonzero(colour == c).astype(np.int32)
        lists.append(vs)
        ptr[c + 1] = ptr[c] + vs.size
    lst = np.concatenate(lists) if lists else np.zeros(0, dtype=np.int32)
    return ptr, lst

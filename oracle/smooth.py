"""Oracle smoothing driver: sweeps (C, float64) and Algorithm 1's stopping rule.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Stopping rule (Algorithm 1 and Sections 3.2, 5.1), as read here:
  Q_0 = Q(P_0); if Q_0 >= goal, stop after 0 sweeps.
  for k = 1 .. max_iters:
      one sweep;  Q_k = Q(P_k)
      if Q_k >= goal            -> stop (goal reached)
      if Q_k - Q_{k-1} < tol    -> stop (improved by less than tol; a
                                   decrease also stops)
  otherwise stop at max_iters.
The paper updates the global quality inside the sweep; its value at the end of
the sweep is Q_k, and the loop condition is tested between sweeps, so Q is
evaluated once per sweep.  tol defaults to the paper's 0.000005.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math

import numpy as np

from . import build as _build
from .mesh import Topology
from .quality import global_quality

_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(_build.build())
        lib.oracle_jacobi.argtypes = [ctypes.c_int32, _i64p, _i32p, _u8p, _f64p, _f64p,
                                      ctypes.c_int32, ctypes.c_int32]
        lib.oracle_multicolor.argtypes = [ctypes.c_int32, _i64p, _i32p, ctypes.c_int32,
                                          _i64p, _i32p, _f64p, _f64p, ctypes.c_int32]
        lib.oracle_gauss_seidel.argtypes = [ctypes.c_int32, _i64p, _i32p, _u8p, _f64p, _f64p,
                                            ctypes.c_int32]
        for f in (lib.oracle_jacobi, lib.oracle_multicolor, lib.oracle_gauss_seidel):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def jacobi(top: Topology, x, y, K: int, threads: int = 1):
    """K Jacobi sweeps; returns new (x, y) float64 arrays."""
    lib = _load()
    x = np.array(x, dtype=np.float64, copy=True)
    y = np.array(y, dtype=np.float64, copy=True)
    ptr = np.ascontiguousarray(top.nbr_ptr, dtype=np.int64)
    nbr = np.ascontiguousarray(top.nbr, dtype=np.int32)
    fx = np.ascontiguousarray(top.fixed, dtype=np.uint8)
    rc = lib.oracle_jacobi(top.n, _p(ptr, _i64p), _p(nbr, _i32p), _p(fx, _u8p),
                           _p(x, _f64p), _p(y, _f64p), int(K), int(threads))
    if rc != 0:
        raise MemoryError("oracle_jacobi")
    return x, y


def multicolor(top: Topology, colour_ptr, colour_list, x, y, K: int):
    lib = _load()
    x = np.array(x, dtype=np.float64, copy=True)
    y = np.array(y, dtype=np.float64, copy=True)
    ptr = np.ascontiguousarray(top.nbr_ptr, dtype=np.int64)
    nbr = np.ascontiguousarray(top.nbr, dtype=np.int32)
    cp = np.ascontiguousarray(colour_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(colour_list, dtype=np.int32)
    lib.oracle_multicolor(top.n, _p(ptr, _i64p), _p(nbr, _i32p), int(cp.size - 1),
                          _p(cp, _i64p), _p(cl, _i32p), _p(x, _f64p), _p(y, _f64p), int(K))
    return x, y


def gauss_seidel(top: Topology, x, y, K: int):
    lib = _load()
    x = np.array(x, dtype=np.float64, copy=True)
    y = np.array(y, dtype=np.float64, copy=True)
    ptr = np.ascontiguousarray(top.nbr_ptr, dtype=np.int64)
    nbr = np.ascontiguousarray(top.nbr, dtype=np.int32)
    fx = np.ascontiguousarray(top.fixed, dtype=np.uint8)
    lib.oracle_gauss_seidel(top.n, _p(ptr, _i64p), _p(nbr, _i32p), _p(fx, _u8p),
                            _p(x, _f64p), _p(y, _f64p), int(K))
    return x, y


@dataclasses.dataclass
class SmoothResult:
    x: np.ndarray
    y: np.ndarray
    iters: int
    stopped_by: str          # "max_iters" | "tol" | "goal"
    q0: float
    q_final: float
    q_history: list          # Q_0, Q_1, ..., Q_iters
    last_dq: float


def smooth(top: Topology, x, y, *, max_iters: int, tol: float = 5e-6,
           goal: float = math.inf, scheme: str = "jacobi", colours=None,
           q_prev: float | None = None) -> SmoothResult:
    """Algorithm 1 with the stopping rule above.

    ``scheme`` "jacobi" or "multicolor" (then ``colours`` = (colour_ptr,
    colour_list)).  ``q_prev`` replaces Q_0 (resuming an earlier run).
    """
    x = np.array(x, dtype=np.float64, copy=True)
    y = np.array(y, dtype=np.float64, copy=True)
    q = global_quality(x, y, top.tri, top.n) if q_prev is None else float(q_prev)
    hist = [q]
    q0 = q
    if q >= goal:
        return SmoothResult(x, y, 0, "goal", q0, q, hist, math.nan)
    dq = math.nan
    for k in range(1, max_iters + 1):
        if scheme == "jacobi":
            x, y = jacobi(top, x, y, 1)
        elif scheme == "multicolor":
            x, y = multicolor(top, colours[0], colours[1], x, y, 1)
        else:
            raise ValueError(scheme)
        qk = global_quality(x, y, top.tri, top.n)
        dq = qk - q
        hist.append(qk)
        q = qk
        if qk >= goal:
            return SmoothResult(x, y, k, "goal", q0, qk, hist, dq)
        if dq < tol:
            return SmoothResult(x, y, k, "tol", q0, qk, hist, dq)
    return SmoothResult(x, y, max_iters, "max_iters", q0, q, hist, dq)


def jacobi_at_vertices(top: Topology, x, y, K: int, sample) -> tuple[np.ndarray, np.ndarray]:
    """P_K at the ``sample`` vertices only, computed on their K-ring balls.

    After K sweeps a vertex depends only on the starting positions within
    graph distance K.  Each sampled vertex's ball is cut out (vertices at
    distance exactly K are frozen: their later values never reach the
    centre within K sweeps) and the plain Jacobi sweep is run on it.  Lets the
    oracle check single outputs of meshes too large to sweep whole.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    outx = np.empty(len(sample))
    outy = np.empty(len(sample))
    for s, v in enumerate(np.asarray(sample).tolist()):
        dist = {v: 0}
        frontier = [v]
        for d in range(1, K + 1):
            nxt = []
            for w in frontier:
                for u in top.neighbours(w).tolist():
                    if u not in dist:
                        dist[u] = d
                        nxt.append(u)
            frontier = nxt
        ball = np.array(sorted(dist), dtype=np.int64)   # ascending global label
        local = {g: i for i, g in enumerate(ball.tolist())}
        m = ball.size
        ptr = np.zeros(m + 1, dtype=np.int64)
        nb = []
        fx = np.zeros(m, dtype=np.uint8)
        for i, g in enumerate(ball.tolist()):
            if top.fixed[g] or dist[g] == K:
                fx[i] = 1
                ptr[i + 1] = ptr[i]
                continue
            row = [local[u] for u in top.neighbours(g).tolist()]   # ascending, as globally
            nb.extend(row)
            ptr[i + 1] = ptr[i] + len(row)
        sub = Topology(n=m, tri=np.zeros((0, 3), dtype=np.int64), nbr_ptr=ptr,
                       nbr=np.array(nb, dtype=np.int32), fixed=fx,
                       tcount=np.zeros(m, dtype=np.int64))
        bx, by = jacobi(sub, x[ball], y[ball], K)
        outx[s] = bx[local[v]]
        outy[s] = by[local[v]]
    return outx, outy

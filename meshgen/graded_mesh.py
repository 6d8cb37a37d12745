"""Graded meshes refined toward seeded curves (newest-vertex bisection).

The large workloads: a jittered-grid topology refined by recursive triangle
bisection to a 4x finer edge near one or two seeded curves
y = 0.5 + A sin(2 pi f x + phi) (2x finer in a wider band), optionally with
disc-union holes; interior vertices jittered by +-0.3 of their shortest
incident edge.  Degrees range over 3..12.  The bisection itself runs in
``graded.cpp`` (compiled on first use with g++); nothing here computes any
part of the smoothing method.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "graded.cpp")
LIB = os.path.join(HERE, "_graded.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", SRC, "-o", tmp], check=True)
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        vp = ctypes.c_void_p
        lib.graded_build.restype = ctypes.c_int64
        lib.graded_build.argtypes = [ctypes.c_int32, vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int32, vp, vp,
                                     ctypes.POINTER(ctypes.c_int64)]
        lib.graded_fetch.argtypes = [vp, vp, vp]
        lib.graded_min_edge.argtypes = [ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp]
        lib.graded_free.argtypes = []
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def graded(n0: int, seed: int = 3, curves: int = 1, band_w: float = 0.04,
           land_fraction: float = 0.0, jitter: float = 0.3):
    """Graded mesh on the unit square.

    n0: base grid points per side; refinement: 4 bisection levels (edge/4)
    within ``band_w`` of a curve, 2 levels (edge/2) within 2*band_w.
    Each part draws from its own generator, default_rng([seed, k]), so the
    curves and holes do not move when n0 changes: k=0 cell diagonals (one
    uniform per cell, row-major, < 0.5 selects the lower-left/upper-right
    diagonal); k=1 per curve A ~ U(0.1, 0.25), f ~ U(0.5, 2),
    phi ~ U(0, 2 pi); k=2 disc holes as in ``jittered_grid`` (until
    ``land_fraction`` of the area is cut, judged by triangle centroids);
    k=3 one U(-1, 1) pair per vertex for the jitter.
    """
    from . import Mesh
    diag = (np.random.default_rng([seed, 0]).random((n0 - 1, n0 - 1)) < 0.5).astype(np.uint8)
    rc = np.random.default_rng([seed, 1])
    amp = rc.uniform(0.1, 0.25, curves)
    freq = rc.uniform(0.5, 2.0, curves)
    phase = rc.uniform(0.0, 2 * math.pi, curves)
    bw = np.array([band_w, 2 * band_w], dtype=np.float64)
    bl = np.array([4, 2], dtype=np.int32)
    lib = _load()
    nt = ctypes.c_int64()
    nv = lib.graded_build(int(n0), _p(diag), int(curves), _p(amp), _p(freq), _p(phase), 2, _p(bw), _p(bl),
                          ctypes.byref(nt))
    if nv < 0:
        raise ValueError("bad graded-mesh arguments")
    ix = np.empty(nv, dtype=np.int32)
    iy = np.empty(nv, dtype=np.int32)
    tri = np.empty((nt.value, 3), dtype=np.int32)
    lib.graded_fetch(_p(ix), _p(iy), _p(tri))
    lib.graded_free()
    scale = 4.0 * (n0 - 1)
    top = int(scale)
    fixed = (ix == 0) | (iy == 0) | (ix == top) | (iy == top)

    ndisc = 0
    if land_fraction > 0:
        cx = (ix[tri[:, 0]].astype(np.float64) + ix[tri[:, 1]] + ix[tri[:, 2]]) / (3 * scale)
        cy = (iy[tri[:, 0]].astype(np.float64) + iy[tri[:, 1]] + iy[tri[:, 2]]) / (3 * scale)
        area = np.abs((ix[tri[:, 1]].astype(np.float64) - ix[tri[:, 0]]) * (iy[tri[:, 2]].astype(np.float64) - iy[tri[:, 0]])
                      - (iy[tri[:, 1]].astype(np.float64) - iy[tri[:, 0]]) * (ix[tri[:, 2]].astype(np.float64) - ix[tri[:, 0]]))
        area /= area.sum()
        # bucket triangle centroids on a coarse raster so each disc only
        # looks at nearby triangles
        R = 256
        cell = (np.minimum((cx * R).astype(np.int64), R - 1) * R + np.minimum((cy * R).astype(np.int64), R - 1))
        order = np.argsort(cell, kind="stable")
        starts = np.searchsorted(cell[order], np.arange(R * R + 1))
        land = np.zeros(tri.shape[0], dtype=bool)
        covered = 0.0
        lo, hi = math.log(0.01), math.log(0.06)
        rng = np.random.default_rng([seed, 2])
        while covered < land_fraction:
            c = rng.random(2)
            r = math.exp(rng.uniform(lo, hi))
            i0, i1 = max(0, int((c[0] - r) * R)), min(R - 1, int((c[0] + r) * R))
            j0, j1 = max(0, int((c[1] - r) * R)), min(R - 1, int((c[1] + r) * R))
            idx = np.concatenate([order[starts[i * R + j0]:starts[i * R + j1 + 1]] for i in range(i0, i1 + 1)])
            inside = idx[((cx[idx] - c[0]) ** 2 + (cy[idx] - c[1]) ** 2 < r * r) & ~land[idx]]
            land[inside] = True
            covered += float(area[inside].sum())
            ndisc += 1
        fixed[tri[land].ravel()] = True
        tri = tri[~land]
    hloc = np.empty(nv, dtype=np.float64)
    lib.graded_min_edge(nv, tri.shape[0], _p(ix), _p(iy), _p(np.ascontiguousarray(tri)), _p(hloc))
    jit = np.random.default_rng([seed, 3]).uniform(-1.0, 1.0, size=(nv, 2))
    xy = np.stack([ix / scale, iy / scale], 1)
    free = ~fixed
    xy[free] += jitter * (hloc[free, None] / scale) * jit[free]
    # drop unreferenced vertices (under holes), keeping the order
    used = np.zeros(nv, dtype=bool)
    used[tri.ravel()] = True
    new_id = np.cumsum(used) - 1
    xy = xy[used]
    tri = new_id[tri].astype(np.int32)
    meta = dict(kind="graded", n0=n0, seed=seed, curves=curves, band_w=band_w,
                land_fraction=land_fraction, discs=ndisc, n=int(xy.shape[0]), T=int(tri.shape[0]),
                n_free=int((free & used).sum()))
    return Mesh(np.ascontiguousarray(xy), np.ascontiguousarray(tri), meta)

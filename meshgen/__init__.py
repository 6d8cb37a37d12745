"""Seeded synthetic 2D triangle meshes: the inputs of the smoothing library and of its oracle.

This module only builds point sets and triangle lists.  It holds none of the
smoothing method's arithmetic (no averaging, no quality measure, no ordering),
so that the library under test and the oracle that checks it can both take
their inputs from here without sharing any of the method.

The paper smooths 2D meshes made by a Delaunay mesh generator, of about
300k-390k vertices each with about twice as many triangles (Section 5.1,
Table 1).  Those meshes are not available, so these generators stand in for
them with the same character: planar triangulations, T ~ 2n, mean degree ~6,
interior vertices free, boundary and hole rims fixed.

Every generator is deterministic given its seed (NumPy PCG64 through
``numpy.random.default_rng``).  A mesh is returned as a :class:`Mesh` with

* ``xy``  float64 [n, 2]  vertex coordinates,
* ``tri`` int32  [T, 3]   counter-clockwise triangles (vertex ids),
* ``meta`` dict           sizes and the recipe.

Vertex ids follow the generation order (row-major over the grid): this is the
"original" ordering of the paper (the mesh generator's output order).
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np

__all__ = [
    "Mesh", "jittered_grid", "ocean", "batch", "concat", "regular_grid",
    "wheel", "mesh_hash", "graded", "graded16m", "graded64m",
]


@dataclasses.dataclass
class Mesh:
    xy: np.ndarray          # float64 [n, 2]
    tri: np.ndarray         # int32 [T, 3]
    meta: dict

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])

    @property
    def T(self) -> int:
        return int(self.tri.shape[0])

    @property
    def x(self) -> np.ndarray:
        return np.ascontiguousarray(self.xy[:, 0])

    @property
    def y(self) -> np.ndarray:
        return np.ascontiguousarray(self.xy[:, 1])


def mesh_hash(m: Mesh) -> str:
    """SHA-256 of the coordinate and triangle arrays (little-endian bytes)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(m.xy, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(m.tri, dtype="<i4").tobytes())
    return h.hexdigest()


def _cell_triangles(nx: int, ny: int, diag_ac: np.ndarray) -> np.ndarray:
    """Two CCW triangles per grid cell.

    Point (i, j) (row i along y, column j along x) has id i*nx + j.  Cell (i, j)
    has corners a=(i,j), b=(i,j+1), c=(i+1,j+1), d=(i+1,j).  ``diag_ac[i, j]``
    True splits it along a-c into (a,b,c), (a,c,d); False along b-d into
    (a,b,d), (b,c,d).  Triangles are listed cell by cell, row-major.
    """
    i, j = np.meshgrid(np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    a = (i * nx + j).ravel()
    b = a + 1
    c = a + nx + 1
    d = a + nx
    f = diag_ac.ravel()
    t0 = np.where(f[:, None], np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t1 = np.where(f[:, None], np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    tri = np.empty((a.size * 2, 3), dtype=np.int64)
    tri[0::2] = t0
    tri[1::2] = t1
    return tri


def _grid_points(nx: int, ny: int) -> tuple[np.ndarray, float, float]:
    hx = 1.0 / (nx - 1)
    hy = 1.0 / (ny - 1)
    i, j = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    xy = np.stack([j.ravel() * hx, i.ravel() * hy], 1).astype(np.float64)
    return xy, hx, hy


def _compact(xy: np.ndarray, tri: np.ndarray, free: np.ndarray):
    """Drop unreferenced points, keeping the relative order of the others."""
    used = np.zeros(xy.shape[0], dtype=bool)
    used[tri.ravel()] = True
    new_id = np.cumsum(used) - 1
    return xy[used], new_id[tri].astype(np.int32), free[used]


def jittered_grid(nx: int, ny: int | None = None, seed: int = 1,
                  jitter: float = 0.3, land_fraction: float = 0.0,
                  rng: np.random.Generator | None = None) -> Mesh:
    """nx x ny points on the unit square, each cell split along a random diagonal.

    Draw order from ``default_rng(seed)`` (or ``rng``):
      1. one uniform per cell, row-major; < 0.5 selects the a-c diagonal;
      2. if ``land_fraction`` > 0: discs (centre U[0,1]^2, then radius
         log-uniform in [0.01, 0.06]) are drawn one at a time until at least
         that fraction of the cells has its centre inside some disc; those
         "land" cells are removed (holes) and unreferenced points dropped;
      3. one U(-1, 1) pair per grid point (row-major, before compaction),
         scaled by ``jitter`` * h and added only to free points.

    A point is free when it is not on the outer square and all four cells
    around it are water; every other point lies on a boundary edge (an edge
    with one triangle) of the final mesh and is not moved.
    """
    ny = nx if ny is None else ny
    if nx < 2 or ny < 2:
        raise ValueError("grid needs at least 2x2 points")
    rng = np.random.default_rng(seed) if rng is None else rng
    xy, hx, hy = _grid_points(nx, ny)
    diag = rng.random((ny - 1, nx - 1)) < 0.5

    land = np.zeros((ny - 1, nx - 1), dtype=bool)
    ndisc = 0
    if land_fraction > 0:
        cx = (np.arange(nx - 1) + 0.5) * hx
        cy = (np.arange(ny - 1) + 0.5) * hy
        target = land_fraction * land.size
        count = 0
        lo, hi = math.log(0.01), math.log(0.06)
        while count < target:
            c = rng.random(2)
            r = math.exp(rng.uniform(lo, hi))
            j0 = max(0, int(math.floor((c[0] - r) / hx)) - 1)
            j1 = min(nx - 1, int(math.ceil((c[0] + r) / hx)) + 1)
            i0 = max(0, int(math.floor((c[1] - r) / hy)) - 1)
            i1 = min(ny - 1, int(math.ceil((c[1] + r) / hy)) + 1)
            if j0 < j1 and i0 < i1:
                dx = cx[j0:j1][None, :] - c[0]
                dy = cy[i0:i1][:, None] - c[1]
                inside = dx * dx + dy * dy < r * r
                sub = land[i0:i1, j0:j1]
                count += int(np.count_nonzero(inside & ~sub))
                sub |= inside
            ndisc += 1

    # free points: not on the outer square, all four surrounding cells water
    water = ~land
    free = np.zeros((ny, nx), dtype=bool)
    free[1:-1, 1:-1] = (water[:-1, :-1] & water[:-1, 1:]
                        & water[1:, :-1] & water[1:, 1:])
    jit = rng.uniform(-1.0, 1.0, size=(ny * nx, 2))
    free = free.ravel()
    xy[free, 0] += jitter * hx * jit[free, 0]
    xy[free, 1] += jitter * hy * jit[free, 1]

    tri = _cell_triangles(nx, ny, diag)
    keep = np.repeat(water.ravel(), 2)
    tri = tri[keep]
    xy, tri, free = _compact(xy, tri, free)
    meta = dict(kind="jittered_grid", nx=nx, ny=ny, seed=seed, jitter=jitter,
                land_fraction=land_fraction, discs=ndisc,
                land_cells=int(land.sum()), n=int(xy.shape[0]),
                T=int(tri.shape[0]), n_free=int(free.sum()))
    return Mesh(xy, tri, meta)


def ocean(nx: int = 1000, seed: int = 2, land_fraction: float = 0.30,
          jitter: float = 0.3) -> Mesh:
    """Ocean-like mesh: jittered grid with ~30% of the cells cut out as disc-union holes.

    Stands in for the paper's largest test mesh ("ocean", 392,674 vertices,
    Table 1); the 1000 x 1000 default gives about 700k vertices.
    """
    m = jittered_grid(nx, nx, seed=seed, jitter=jitter, land_fraction=land_fraction)
    m.meta["kind"] = "ocean"
    return m


def batch(count: int = 512, seed: int = 4, n_min: float = 1e3,
          n_max: float = 2e5, jitter: float = 0.3) -> list[Mesh]:
    """Independent jittered grids with log-uniform sizes.

    Mesh i targets n_i = round(exp(U(ln n_min, ln n_max))) points (the U draws
    come from ``default_rng(seed)``) and is built as a ceil(sqrt(n_i))^2 grid
    seeded by ``SeedSequence([seed, i])``.
    """
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=count)))
    out = []
    for i, ni in enumerate(sizes):
        side = max(3, int(math.ceil(math.sqrt(float(ni)))))
        r = np.random.default_rng(np.random.SeedSequence([seed, i]))
        m = jittered_grid(side, side, jitter=jitter, rng=r)
        m.meta.update(kind="batch_member", index=i, target_n=int(ni), seed=[seed, i])
        out.append(m)
    return out


def concat(meshes: list[Mesh]) -> tuple[Mesh, np.ndarray, np.ndarray]:
    """Concatenate meshes into one block-diagonal mesh.

    Returns the union (global vertex ids), ``v_off`` int64[B+1] and
    ``t_off`` int64[B+1].  The union's triangles carry global ids.
    """
    v_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    t_off = np.zeros(len(meshes) + 1, dtype=np.int64)
    for i, m in enumerate(meshes):
        v_off[i + 1] = v_off[i] + m.n
        t_off[i + 1] = t_off[i] + m.T
    xy = np.concatenate([m.xy for m in meshes])
    tri = np.concatenate([m.tri.astype(np.int64) + v_off[i] for i, m in enumerate(meshes)])
    meta = dict(kind="concat", B=len(meshes), n=int(v_off[-1]), T=int(t_off[-1]))
    return Mesh(xy, tri.astype(np.int32), meta), v_off, t_off


def regular_grid(nx: int, ny: int | None = None, h: float | None = None,
                 pattern: str = "same", seed: int = 0) -> Mesh:
    """Unjittered grid with spacing h (default 1/(nx-1)).

    ``pattern``: "same" (every cell split a-c), "checker" (a-c and b-d
    alternating like a checkerboard) or "random" (Bernoulli(1/2) per cell from
    ``default_rng(seed)``).  With a dyadic h all coordinates are exact binary
    fractions.
    """
    ny = nx if ny is None else ny
    i, j = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    if h is None:
        xy, _, _ = _grid_points(nx, ny)
    else:
        xy = np.stack([j.ravel() * h, i.ravel() * h], 1).astype(np.float64)
    ci, cj = np.meshgrid(np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    if pattern == "same":
        diag = np.ones((ny - 1, nx - 1), dtype=bool)
    elif pattern == "checker":
        diag = ((ci + cj) % 2) == 0
    elif pattern == "random":
        diag = np.random.default_rng(seed).random((ny - 1, nx - 1)) < 0.5
    else:
        raise ValueError(pattern)
    tri = _cell_triangles(nx, ny, diag).astype(np.int32)
    return Mesh(xy, tri, dict(kind="regular_grid", nx=nx, ny=ny, h=h, pattern=pattern,
                              n=int(xy.shape[0]), T=int(tri.shape[0])))


def wheel(k: int, radius: float = 1.0, centre=(0.3, -0.2), seed: int | None = None) -> Mesh:
    """A centre vertex (id 0) and a rim of k vertices (ids 1..k); triangles (0, r_j, r_j+1).

    The rim is a regular k-gon around ``centre``; with ``seed`` the rim radii
    are perturbed and the centre vertex starts off-centre.
    """
    ang = 2.0 * np.pi * np.arange(k) / k
    rad = np.full(k, radius)
    start = np.array(centre, dtype=np.float64)
    if seed is not None:
        r = np.random.default_rng(seed)
        rad = radius * (0.6 + 0.8 * r.random(k))
        start = start + 0.25 * radius * (r.random(2) - 0.5)
    rim = np.stack([centre[0] + rad * np.cos(ang), centre[1] + rad * np.sin(ang)], 1)
    xy = np.concatenate([start[None, :], rim]).astype(np.float64)
    j = np.arange(k)
    tri = np.stack([np.zeros(k, dtype=np.int64), 1 + j, 1 + (j + 1) % k], 1).astype(np.int32)
    return Mesh(xy, tri, dict(kind="wheel", k=k, n=k + 1, T=k))


def graded(n0: int, seed: int = 3, curves: int = 1, band_w: float = 0.04,
           land_fraction: float = 0.0, jitter: float = 0.3) -> Mesh:
    """Graded mesh refined by triangle bisection toward seeded curves (see
    :mod:`meshgen.graded_mesh`)."""
    from .graded_mesh import graded as _g
    return _g(n0, seed=seed, curves=curves, band_w=band_w, land_fraction=land_fraction, jitter=jitter)


def graded16m() -> Mesh:
    """~16M vertices: one refinement band (edge/4 within 0.04, edge/2 within 0.08)."""
    return graded(2416, seed=3)


def graded64m() -> Mesh:
    """~64M vertices: two refinement bands and ~30% disc-union holes."""
    return graded(4736, seed=5, curves=2, land_fraction=0.3)

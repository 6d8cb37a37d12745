"""Seeded synthetic meshes: sizes, determinism and validity."""
import numpy as np

import meshgen
from oracle import mesh as omesh


def test_unit_square_grid_sizes():
    m = meshgen.jittered_grid(100, seed=1)
    assert (m.n, m.T, m.meta["n_free"]) == (10000, 19602, 9604)
    assert m.tri.dtype == np.int32 and m.xy.dtype == np.float64


def test_deterministic_by_seed():
    a = meshgen.jittered_grid(50, seed=3, land_fraction=0.3)
    b = meshgen.jittered_grid(50, seed=3, land_fraction=0.3)
    c = meshgen.jittered_grid(50, seed=4, land_fraction=0.3)
    assert meshgen.mesh_hash(a) == meshgen.mesh_hash(b) != meshgen.mesh_hash(c)


def test_triangles_counter_clockwise():
    m = meshgen.jittered_grid(30, seed=5, land_fraction=0.2)
    p = m.xy[m.tri]
    cross = ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
             - (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0]))
    assert (cross > 0).all()


def test_holes_reach_land_fraction_and_stay_valid():
    m = meshgen.jittered_grid(120, seed=2, land_fraction=0.3)
    assert m.meta["land_cells"] >= 0.3 * 119 * 119
    top = omesh.topology(m.n, m.tri)      # raises on malformed meshes
    assert top.degree.max() <= 8
    assert m.n < 120 * 120


def test_batch_and_concat():
    ms = meshgen.batch(count=6, seed=4, n_min=100, n_max=2000)
    u, v_off, t_off = meshgen.concat(ms)
    assert v_off[-1] == u.n == sum(m.n for m in ms)
    assert t_off[-1] == u.T
    for i, m in enumerate(ms):
        assert np.array_equal(u.tri[t_off[i]:t_off[i + 1]] - v_off[i], m.tri)


def test_graded_mesh_is_valid_and_refined():
    m = meshgen.graded(129, seed=3)
    top = omesh.topology(m.n, m.tri)
    assert m.n > 2.0 * 129 * 129                 # the band was refined
    d = top.degree[top.fixed == 0]
    assert d.min() >= 3 and d.max() <= 12
    p = m.xy[m.tri]
    cross = ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
             - (p[:, 1, 1] - p[:, 0, 1]) * (p[:, 2, 0] - p[:, 0, 0]))
    assert (cross > 0).mean() > 0.999             # counter-clockwise (jitter may flip a sliver)
    a = meshgen.graded(129, seed=3)
    assert meshgen.mesh_hash(a) == meshgen.mesh_hash(m)


def test_graded_mesh_with_holes():
    m = meshgen.graded(97, seed=5, curves=2, land_fraction=0.3)
    top = omesh.topology(m.n, m.tri)
    assert m.meta["discs"] > 0
    assert int((top.fixed == 0).sum()) == m.meta["n_free"]

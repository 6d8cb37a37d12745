"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, exact fixed points, invariants, library routines (NumPy matrix powers,
SciPy sparse solve and BFS), brute force on tiny meshes, or hand-traced
examples (tests/golden).  Chosen so that a dropped term, a wrong sign or
index, a self-inclusion in the mean or a transposed operand fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla

import meshgen
from oracle import mesh as omesh
from oracle import orderings as oord
from oracle import quality as oq
from oracle import smooth as osm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rdr_bfs_examples.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def small_mesh(nx=13, seed=7, land=0.0):
    m = meshgen.jittered_grid(nx, seed=seed, land_fraction=land)
    return m, omesh.topology(m.n, m.tri)


# ----------------------------------------------------------------- topology

def test_wheel_topology():
    m = meshgen.wheel(7)
    top = omesh.topology(m.n, m.tri)
    assert top.neighbours(0).tolist() == list(range(1, 8))
    for r in range(1, 8):
        assert top.degree[r] == 3
    assert top.fixed.tolist() == [0] + [1] * 7
    assert top.tcount.tolist() == [7] + [2] * 7


@pytest.mark.parametrize("pattern,degrees", [("same", {6}), ("checker", {4, 8})])
def test_regular_grid_degrees(pattern, degrees):
    m = meshgen.regular_grid(9, pattern=pattern)
    top = omesh.topology(m.n, m.tri)
    inner = top.interior
    assert inner.size == 7 * 7
    assert set(top.degree[inner].tolist()) == degrees
    # the fixed vertices are exactly the outer square
    i, j = np.divmod(np.arange(m.n), 9)
    on_square = (i == 0) | (i == 8) | (j == 0) | (j == 8)
    assert np.array_equal(top.fixed.astype(bool), on_square)


def test_ocean_fixed_matches_generator_free_points():
    # meshgen decides which points to jitter from the grid's cell mask; the
    # oracle decides fixed vertices from boundary edges: both must agree.
    m = meshgen.jittered_grid(60, seed=3, land_fraction=0.3)
    top = omesh.topology(m.n, m.tri)
    assert int((top.fixed == 0).sum()) == m.meta["n_free"]
    h = 1.0 / 59
    on_grid = (np.abs(m.xy / h - np.rint(m.xy / h)) < 1e-9).all(axis=1)
    assert on_grid[top.fixed == 1].all()          # fixed points never jittered
    assert not on_grid[top.fixed == 0].any()      # free points all jittered


@pytest.mark.parametrize("tri,n,msg", [
    ([[0, 1, 3]], 3, "outside"),
    ([[0, 1, 1]], 3, "repeats"),
    ([[0, 1, 2], [0, 1, 3], [1, 0, 4]], 5, "more than two"),
    ([[0, 1, 2]], 4, "not referenced"),
])
def test_malformed_meshes(tri, n, msg):
    with pytest.raises(omesh.MeshError, match=msg):
        omesh.topology(n, tri)


# ----------------------------------------------------------------- Jacobi

def test_jacobi_equals_dense_operator_powers():
    m, top = small_mesh(15, seed=11)
    A = omesh.smoothing_operator_dense(top)
    extent = np.ptp(m.xy, axis=0).max()
    for K in (1, 2, 7, 20):
        AK = np.linalg.matrix_power(A, K)
        ex, ey = AK @ m.x, AK @ m.y
        x, y = osm.jacobi(top, m.x, m.y, K)
        assert np.max(np.abs(x - ex)) <= 1e-14 * extent
        assert np.max(np.abs(y - ey)) <= 1e-14 * extent


def test_jacobi_dense_operator_on_holed_mesh():
    m, top = small_mesh(20, seed=5, land=0.3)
    A = omesh.smoothing_operator_dense(top)
    AK = np.linalg.matrix_power(A, 9)
    x, y = osm.jacobi(top, m.x, m.y, 9)
    assert np.max(np.abs(x - AK @ m.x)) <= 1e-14
    assert np.max(np.abs(y - AK @ m.y)) <= 1e-14


@pytest.mark.parametrize("h", [1 / 8, 1 / 64])
@pytest.mark.parametrize("pattern", ["same", "checker"])
def test_exact_fixed_point_regular_grid(h, pattern):
    # neighbours sit symmetrically around each free vertex, every sum is exact
    # in binary and the quotient of an exact multiple is exact: no movement.
    m = meshgen.regular_grid(12, h=h, pattern=pattern)
    top = omesh.topology(m.n, m.tri)
    x, y = osm.jacobi(top, m.x, m.y, 20)
    assert np.array_equal(x, m.x) and np.array_equal(y, m.y)


def test_random_diagonals_move():
    m = meshgen.regular_grid(12, h=1 / 8, pattern="random", seed=3)
    top = omesh.topology(m.n, m.tri)
    x, y = osm.jacobi(top, m.x, m.y, 1)
    assert not (np.array_equal(x, m.x) and np.array_equal(y, m.y))


@pytest.mark.parametrize("k", [3, 5, 8, 13])
def test_wheel_centre_goes_to_rim_mean(k):
    m = meshgen.wheel(k, seed=k)
    top = omesh.topology(m.n, m.tri)
    rim = m.xy[1:]
    mean = np.array([math.fsum(rim[:, 0]) / k, math.fsum(rim[:, 1]) / k])
    x, y = osm.jacobi(top, m.x, m.y, 1)
    assert abs(x[0] - mean[0]) <= 4e-16 * k and abs(y[0] - mean[1]) <= 4e-16 * k
    assert np.array_equal(x[1:], m.x[1:]) and np.array_equal(y[1:], m.y[1:])
    x2, y2 = osm.jacobi(top, x, y, 1)
    assert x2[0] == x[0] and y2[0] == y[0]
    # multicolour: one free vertex, one colour, same one-ring centroid
    col = oord.greedy_colouring(top)
    cp, cl = oord.colour_lists(col)
    mx, my = osm.multicolor(top, cp, cl, m.x, m.y, 1)
    assert mx[0] == x[0] and my[0] == y[0]


def test_fixed_vertices_bitwise_unchanged():
    m, top = small_mesh(25, seed=2, land=0.3)
    x, y = osm.jacobi(top, m.x, m.y, 13)
    f = top.fixed == 1
    assert np.array_equal(x[f], m.x[f]) and np.array_equal(y[f], m.y[f])
    assert not np.array_equal(x[~f], m.x[~f])


def relabel(m, new2old):
    old2new = oord.inverse(new2old)
    xy = m.xy[new2old]
    tri = old2new[m.tri]
    return meshgen.Mesh(xy, tri.astype(np.int32), dict(m.meta))


@pytest.mark.parametrize("kind", ["bfs", "rdr", "random"])
def test_jacobi_permutation_invariance(kind):
    m, top = small_mesh(30, seed=4, land=0.25)
    if kind == "bfs":
        p = oord.bfs(top)
    elif kind == "rdr":
        p = oord.rdr(top, oq.vertex_quality(m.x, m.y, m.tri, m.n))
    else:
        p = oord.random_order(m.n, 99)
    mp = relabel(m, p)
    tp = omesh.topology(mp.n, mp.tri)
    x0, y0 = osm.jacobi(top, m.x, m.y, 25)
    xp, yp = osm.jacobi(tp, mp.x, mp.y, 25)
    old2new = oord.inverse(p)
    extent = np.ptp(m.xy, axis=0).max()
    assert np.max(np.abs(xp[old2new] - x0)) <= 1e-12 * extent
    assert np.max(np.abs(yp[old2new] - y0)) <= 1e-12 * extent


def test_jacobi_converges_to_harmonic_limit():
    # P* solves (I - A_II) x_I = A_IF x_F; Jacobi error is bounded by
    # ||A_II^k||_inf * ||P_0 - P*||_inf.
    m, top = small_mesh(14, seed=9)
    A = sp.csr_matrix(omesh.smoothing_operator_dense(top))
    I = np.flatnonzero(top.fixed == 0)
    F = np.flatnonzero(top.fixed == 1)
    AII = A[I][:, I]
    AIF = A[I][:, F]
    M = (sp.identity(I.size) - AII).tocsc()
    sx = m.x.copy()
    sy = m.y.copy()
    sx[I] = spla.spsolve(M, AIF @ m.x[F])
    sy[I] = spla.spsolve(M, AIF @ m.y[F])
    e0 = max(np.max(np.abs(m.x - sx)), np.max(np.abs(m.y - sy)))
    AIId = AII.toarray()
    for K in (10, 60, 900):
        x, y = osm.jacobi(top, m.x, m.y, K)
        bound = np.abs(np.linalg.matrix_power(AIId, K)).sum(axis=1).max() * e0
        err = max(np.max(np.abs(x - sx)), np.max(np.abs(y - sy)))
        assert err <= bound + 1e-13
    assert err < 1e-9   # 900 sweeps on a 14x14 grid reach the limit


def test_jacobi_scale_and_rotation_equivariance():
    m, top = small_mesh(17, seed=12)
    x, y = osm.jacobi(top, m.x, m.y, 11)
    x2, y2 = osm.jacobi(top, 2 * m.x, 2 * m.y, 11)
    assert np.array_equal(x2, 2 * x) and np.array_equal(y2, 2 * y)
    xr, yr = osm.jacobi(top, -m.y, m.x, 11)           # rotation by 90 degrees
    assert np.array_equal(xr, -y) and np.array_equal(yr, x)


def test_jacobi_split_run_and_threads():
    m, top = small_mesh(33, seed=13, land=0.3)
    x, y = osm.jacobi(top, m.x, m.y, 12)
    a, b = osm.jacobi(top, m.x, m.y, 5)
    a, b = osm.jacobi(top, a, b, 7)
    assert np.array_equal(a, x) and np.array_equal(b, y)
    t, u = osm.jacobi(top, m.x, m.y, 12, threads=4)
    assert np.array_equal(t, x) and np.array_equal(u, y)


def test_jacobi_at_vertices_matches_whole_mesh():
    m, top = small_mesh(40, seed=21, land=0.2)
    K = 6
    x, y = osm.jacobi(top, m.x, m.y, K)
    sample = np.random.default_rng(0).choice(m.n, 25, replace=False)
    sx, sy = osm.jacobi_at_vertices(top, m.x, m.y, K, sample)
    assert np.array_equal(sx, x[sample]) and np.array_equal(sy, y[sample])


# ----------------------------------------------------------------- multicolour / Gauss-Seidel

def test_colouring_is_proper_and_complete():
    m, top = small_mesh(40, seed=1, land=0.3)
    col = oord.greedy_colouring(top)
    free = top.fixed == 0
    assert (col[free] >= 0).all() and (col[~free] == -1).all()
    for v in np.flatnonzero(free):
        nb = top.neighbours(v)
        nb = nb[free[nb]]
        assert not np.any(col[nb] == col[v])
    assert 3 <= col.max() + 1 <= 9


def test_colouring_hand_traced_first_fit():
    # a schedule traced by hand from the first-fit rule in ascending label;
    # visiting in descending label, or taking one past the largest
    # neighbour colour, gives another colouring and fails here
    with open(os.path.join(os.path.dirname(__file__), "golden", "colouring_example.json")) as f:
        g = json.load(f)
    top = omesh.topology(g["n"], np.array(g["tri"]))
    assert top.interior.tolist() == g["free"]
    col = oord.greedy_colouring(top)
    assert col.tolist() == g["colour"]
    assert col.tolist() != g["colour_descending_visit"]
    ptr, lst = oord.colour_lists(col)
    assert [lst[ptr[c]:ptr[c + 1]].tolist() for c in range(ptr.size - 1)] == g["colour_lists"]


def test_multicolour_equals_dense_colour_product():
    m, top = small_mesh(13, seed=31)
    A = omesh.smoothing_operator_dense(top)
    col = oord.greedy_colouring(top)
    cp, cl = oord.colour_lists(col)
    n = m.n
    S = np.eye(n)
    for c in range(cp.size - 1):
        Ac = np.eye(n)
        rows = cl[cp[c]:cp[c + 1]]
        Ac[rows] = A[rows]
        S = Ac @ S
    for K in (1, 4):
        SK = np.linalg.matrix_power(S, K)
        x, y = osm.multicolor(top, cp, cl, m.x, m.y, K)
        assert np.max(np.abs(x - SK @ m.x)) <= 1e-14
        assert np.max(np.abs(y - SK @ m.y)) <= 1e-14


def test_gauss_seidel_equals_dense_vertex_product():
    m, top = small_mesh(11, seed=32)
    A = omesh.smoothing_operator_dense(top)
    S = np.eye(m.n)
    for v in range(m.n):
        Av = np.eye(m.n)
        Av[v] = A[v]
        S = Av @ S
    x, y = osm.gauss_seidel(top, m.x, m.y, 3)
    S3 = np.linalg.matrix_power(S, 3)
    assert np.max(np.abs(x - S3 @ m.x)) <= 1e-14


def test_multicolour_and_jacobi_share_the_limit():
    m, top = small_mesh(12, seed=8)
    col = oord.greedy_colouring(top)
    cp, cl = oord.colour_lists(col)
    xj, yj = osm.jacobi(top, m.x, m.y, 600)
    xm, ym = osm.multicolor(top, cp, cl, m.x, m.y, 600)
    assert np.max(np.abs(xj - xm)) < 1e-12 and np.max(np.abs(yj - ym)) < 1e-12


@pytest.mark.parametrize("h", [1 / 8, 1 / 64])
def test_multicolour_exact_fixed_point(h):
    m = meshgen.regular_grid(10, h=h, pattern="checker")
    top = omesh.topology(m.n, m.tri)
    cp, cl = oord.colour_lists(oord.greedy_colouring(top))
    x, y = osm.multicolor(top, cp, cl, m.x, m.y, 10)
    assert np.array_equal(x, m.x) and np.array_equal(y, m.y)


# ----------------------------------------------------------------- quality

def one(tri_xy):
    xy = np.asarray(tri_xy, dtype=np.float64)
    return oq.triangle_quality(xy[:, 0], xy[:, 1], [[0, 1, 2]])[0]


def test_triangle_quality_closed_forms():
    assert abs(one([[0, 0], [1, 0], [0, 1]]) - 1 / math.sqrt(2)) <= 2 ** -53
    assert one([[0, 0], [3, 0], [0, 4]]) == 0.6                    # 3-4-5
    assert one([[0, 0], [4, 0], [0, 3]]) == 0.6
    assert abs(one([[0, 0], [1, 0], [0.5, math.sqrt(3) / 2]]) - 1.0) < 1e-15
    assert one([[0, 0], [1, 0], [2, 0]]) == 0.5                    # lengths 1, 1, 2
    assert one([[0, 0], [0, 0], [1, 1]]) == 0.0                    # repeated point
    assert one([[2, 2], [2, 2], [2, 2]]) == 0.0                    # all lengths zero


def test_triangle_quality_invariances():
    rng = np.random.default_rng(3)
    xy = rng.random((50, 3, 2))
    q = np.array([one(t) for t in xy])
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    q_rot = np.array([one(t @ R.T * 3.5 + 1.25) for t in xy])
    assert np.max(np.abs(q - q_rot)) < 1e-14
    q_perm = np.array([one(t[[1, 2, 0]]) for t in xy])              # corner order
    assert np.array_equal(q, q_perm)
    assert ((q > 0) & (q <= 1)).all()


def test_regular_grid_quality_is_one_over_root_two():
    m = meshgen.regular_grid(21, pattern="random", seed=2)
    Q = oq.global_quality(m.x, m.y, m.tri, m.n)
    assert abs(Q - 1 / math.sqrt(2)) < 1e-15


def test_vertex_quality_matches_python_loop_bitwise():
    m, _ = small_mesh(9, seed=4)
    qt = oq.triangle_quality(m.x, m.y, m.tri)
    qv = oq.vertex_quality(m.x, m.y, m.tri, m.n)
    ref = []
    for v in range(m.n):
        s = 0.0
        c = 0
        for t in range(m.T):
            if v in m.tri[t]:
                s += float(qt[t])
                c += 1
        ref.append(s / c)
    assert np.array_equal(qv, np.array(ref))


def test_per_triangle_weighted_form_equals_vertex_mean():
    # (1/n) sum_v mean_{t in v} q_t == sum_t q_t * (1/n) sum_{v in t} 1/|T(v)|
    m, top = small_mesh(30, seed=5, land=0.3)
    qt = oq.triangle_quality(m.x, m.y, m.tri)
    inv = 1.0 / top.tcount
    w = inv[m.tri].sum(axis=1) / m.n
    Q = oq.global_quality(m.x, m.y, m.tri, m.n)
    assert abs(math.fsum((qt * w).tolist()) - Q) < 1e-14


def test_smoothing_improves_quality_of_jittered_grid():
    m, top = small_mesh(40, seed=6)
    q0 = oq.global_quality(m.x, m.y, m.tri, m.n)
    x, y = osm.jacobi(top, m.x, m.y, 5)
    assert oq.global_quality(x, y, m.tri, m.n) > q0


# ----------------------------------------------------------------- stopping rule

def test_stop_rule_branches():
    m, top = small_mesh(30, seed=10, land=0.2)
    r = osm.smooth(top, m.x, m.y, max_iters=500)
    assert r.stopped_by == "tol"
    dq = np.diff(r.q_history)
    assert dq[-1] < 5e-6 and np.all(dq[:-1] >= 5e-6)
    assert len(r.q_history) == r.iters + 1
    x, y = osm.jacobi(top, m.x, m.y, r.iters)
    assert np.array_equal(x, r.x) and np.array_equal(y, r.y)
    # goal already met: zero sweeps
    r0 = osm.smooth(top, m.x, m.y, max_iters=10, goal=r.q0)
    assert r0.iters == 0 and r0.stopped_by == "goal"
    # goal reached after exactly the first sweep whose Q passes it
    g = r.q_history[3]
    rg = osm.smooth(top, m.x, m.y, max_iters=100, goal=g)
    assert rg.iters == 3 and rg.stopped_by == "goal"
    # no tolerance: max_iters
    rm = osm.smooth(top, m.x, m.y, max_iters=4, tol=-math.inf)
    assert rm.iters == 4 and rm.stopped_by == "max_iters"


def test_stop_rule_boundary_cases():
    m, top = small_mesh(20, seed=14)
    q1 = osm.smooth(top, m.x, m.y, max_iters=1, tol=-math.inf).q_final
    # a decrease stops: pretend the previous quality was higher than Q_1
    r = osm.smooth(top, m.x, m.y, max_iters=5, q_prev=q1 + 0.01)
    assert r.iters == 1 and r.stopped_by == "tol" and r.last_dq < 0
    # an improvement of exactly tol does not stop
    q_prev = 0.5
    tol = q1 - q_prev
    r = osm.smooth(top, m.x, m.y, max_iters=2, q_prev=q_prev, tol=tol)
    assert r.q_history[1] - r.q_history[0] == tol and r.iters >= 2


def test_iteration_count_independent_of_ordering():
    # Section 5.1: the orderings do not change the number of iterations.
    m, top = small_mesh(45, seed=15, land=0.3)
    base = osm.smooth(top, m.x, m.y, max_iters=2000)
    qv = oq.vertex_quality(m.x, m.y, m.tri, m.n)
    for p in (oord.bfs(top), oord.rdr(top, qv), oord.random_order(m.n, 5)):
        mp = relabel(m, p)
        tp = omesh.topology(mp.n, mp.tri)
        r = osm.smooth(tp, mp.x, mp.y, max_iters=2000)
        assert r.iters == base.iters
        assert abs(r.q_final - base.q_final) < 1e-12


# ----------------------------------------------------------------- orderings

def topo_from_golden(g):
    return omesh.topology(g["n"], np.array(g["tri"]))


def test_rdr_hand_traced_grid3():
    g = golden()["grid3"]
    top = topo_from_golden(g)
    assert top.interior.tolist() == [4]
    assert oord.rdr(top, g["q"]).tolist() == g["rdr"]
    assert oord.rdr(top, [0.5] * g["n"]).tolist() == g["rdr_all_equal_q"]


def test_rdr_hand_traced_grid4_theorem1_gap():
    g = golden()["grid4"]
    top = topo_from_golden(g)
    assert top.interior.tolist() == [5, 6, 9, 10]
    assert oord.rdr(top, g["q"], extend=False).tolist() == g["rdr_as_printed"]
    assert oord.rdr(top, g["q"]).tolist() == g["rdr"]


def test_bfs_hand_traced_grid4():
    g = golden()["grid4"]
    assert oord.bfs(topo_from_golden(g)).tolist() == g["bfs"]


@pytest.mark.parametrize("seed", range(6))
def test_rdr_invariants(seed):
    m, top = small_mesh(18 + seed, seed=seed, land=0.3 if seed % 2 else 0.0)
    q = oq.vertex_quality(m.x, m.y, m.tri, m.n)
    p = oord.rdr(top, q)
    assert oord.is_permutation(p, m.n)                                   # Theorem 1 (extended)
    inner = top.interior
    first = min(inner.tolist(), key=lambda v: (q[v], v))
    assert p[0] == first                                                 # worst interior first
    nb = sorted(top.neighbours(first).tolist(), key=lambda v: (q[v], v))
    assert p[1:1 + len(nb)].tolist() == nb                               # then its neighbours
    printed = oord.rdr(top, q, extend=False)
    assert np.array_equal(p[:printed.size], printed)                     # extension only appends


def test_rdr_extension_is_noop_when_printed_loop_is_complete():
    found = 0
    for seed in range(40):
        m = meshgen.regular_grid(9, pattern="random", seed=seed)
        top = omesh.topology(m.n, m.tri)
        q = np.random.default_rng(seed).random(m.n)
        printed = oord.rdr(top, q, extend=False)
        full = oord.rdr(top, q)
        if printed.size == m.n:
            found += 1
            assert np.array_equal(printed, full)
        else:
            assert np.array_equal(full[:printed.size], printed)
    assert found > 0


def test_bfs_matches_scipy_and_levels():
    m, top = small_mesh(35, seed=17)
    p = oord.bfs(top)
    n = m.n
    rows = np.repeat(np.arange(n), top.degree)
    A = sp.csr_matrix((np.ones(rows.size), top.nbr, top.nbr_ptr), shape=(n, n))
    ref = csgraph.breadth_first_order(A, 0, directed=True, return_predecessors=False)
    assert np.array_equal(p, ref)
    lev = csgraph.shortest_path(A, unweighted=True, indices=0)
    assert np.all(np.diff(lev[p]) >= 0)


def test_bfs_restarts_on_each_component():
    m = meshgen.jittered_grid(40, seed=8, land_fraction=0.45)
    top = omesh.topology(m.n, m.tri)
    p = oord.bfs(top)
    assert oord.is_permutation(p, m.n)
    n = m.n
    A = sp.csr_matrix((np.ones(top.nbr.size), top.nbr, top.nbr_ptr), shape=(n, n))
    ncomp, lab = csgraph.connected_components(A, directed=False)
    # each component is one contiguous run, started at its smallest label
    runs = lab[p]
    starts = np.flatnonzero(np.r_[True, runs[1:] != runs[:-1]])
    assert starts.size == ncomp
    assert all(p[s] == np.flatnonzero(lab == runs[s]).min() for s in starts)


def test_splitmix64_published_vectors():
    g = golden()["splitmix64"]
    s = oord.SplitMix64(0)
    assert [s.next() for _ in range(3)] == [int(v, 16) for v in g["seed0_first"]]
    s = oord.SplitMix64(1234567)
    assert [s.next() for _ in range(3)] == g["seed1234567_first"]


def test_random_order_is_uniform_bijection():
    counts = {}
    for seed in range(6000):
        p = tuple(oord.random_order(3, seed).tolist())
        counts[p] = counts.get(p, 0) + 1
    assert len(counts) == 6
    assert all(abs(c - 1000) < 150 for c in counts.values())
    assert oord.is_permutation(oord.random_order(1000, 7), 1000)


# ---- reuse-distance profile (Section 2; Table 2's quantiles) --------------

def test_reuse_distance_hand_example():
    from oracle import reuse as ore
    # a b c a b b: the second a sees {b, c}, the second b {c, a}, the third b nothing
    for f in (ore.reuse_distances, ore.reuse_distances_brute):
        d, cold = f([0, 1, 2, 0, 1, 1])
        assert d.tolist() == [2, 2, 0] and cold == 3


def test_algorithm1_trace_hand_traced_on_a_wheel():
    # centre 0 (free) with rim 1, 2, 3 (fixed); triangles (0,1,2), (0,2,3),
    # (0,3,1), all with smallest corner 0, so they keep their input order.
    # Traced by hand: the centre, its neighbours; then per triangle its sorted
    # corners and its quality record (items 4, 5, 6).
    from oracle import mesh as omesh
    from oracle import reuse as ore
    tri = np.array([[0, 1, 2], [0, 2, 3], [0, 3, 1]])
    top = omesh.topology(4, tri)
    assert top.fixed.tolist() == [0, 1, 1, 1]
    tr = ore.algorithm1_trace(top, np.arange(4))
    assert tr.tolist() == [0, 1, 2, 3, 0, 1, 2, 4, 0, 2, 3, 5, 0, 1, 3, 6]
    for f in (ore.reuse_distances, ore.reuse_distances_brute):
        d, cold = f(tr)
        assert d.tolist() == [3, 3, 3, 3, 2, 4, 3, 5, 3] and cold == 7
    # under the labels reversed, the triangles sort by their smallest new label
    p = np.array([3, 2, 1, 0])               # new label k holds input vertex p[k]
    assert ore.triangle_rank(tri, p).tolist() == [2, 0, 1]  # keys (1,0), (0,1), (0,2)


def test_reuse_distance_stack_matches_definition_on_random_traces():
    from oracle import reuse as ore
    rng = np.random.default_rng(11)
    for _ in range(20):
        tr = rng.integers(0, rng.integers(2, 30), size=rng.integers(1, 120))
        a, ca = ore.reuse_distances(tr)
        b, cb = ore.reuse_distances_brute(tr)
        assert np.array_equal(a, b) and ca == cb


def test_reuse_quantile_definition():
    from oracle import reuse as ore
    d = [4, 1, 3, 2]
    assert [ore.quantile(d, x) for x in (0.0, 0.25, 0.5, 0.75, 0.9, 1.0)] == [1, 1, 2, 3, 4, 4]
    assert ore.quantile([], 0.5) == 0


def test_reuse_trace_and_line_spans_of_a_wheel():
    from oracle import mesh as omesh
    from oracle import reuse as ore
    m = meshgen.wheel(8)                        # centre 0 (free), rim 1..8 (fixed)
    top = omesh.topology(m.n, m.tri)
    ident = np.arange(m.n)
    assert ore.sweep_trace(top, ident).tolist() == [0, 1, 2, 3, 4, 5, 6, 7, 8]
    d, cold = ore.reuse_distances(ore.sweep_trace(top, ident))
    assert d.size == 0 and cold == 9
    # rim records at bytes 16..128 of 16-byte records: lines 0 and 1 of 128 bytes
    assert ore.wave_line_spans(top, ident).tolist() == [2]
    assert ore.wave_line_spans(top, ident, line_bytes=64).tolist() == [3]

"""Host logic of the library (no GPU): exports, adjacency, orderings, errors.

The library is loaded through its C ABI; only host-only entry points are
called here.  Integer results (adjacency, fixed flags, colours, orderings)
must equal the oracle's exactly; host vertex qualities bit for bit.
"""
import json
import os
import re

import numpy as np
import pytest

import meshgen
from oracle import mesh as omesh
from oracle import orderings as oord
from oracle import quality as oq
from paper_1606_00803_amd import lms

HERE = os.path.dirname(__file__)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not os.path.exists(lms.LIB_PATH):
        from paper_1606_00803_amd import build
        build.build()
    lms.load()


def golden():
    with open(os.path.join(HERE, "golden", "rdr_bfs_examples.json")) as f:
        return json.load(f)


MESHES = {
    "grid100": lambda: meshgen.jittered_grid(100, seed=1),
    "ocean120": lambda: meshgen.jittered_grid(120, seed=2, land_fraction=0.3),
    "ocean_ragged": lambda: meshgen.jittered_grid(97, 61, seed=9, land_fraction=0.35),
}


def test_every_header_function_is_exported():
    names = lms.header_functions()
    assert len(names) >= 17
    lib = lms.load()
    for name in names:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert set(names) == set(lms._SIGS)


# entry points that compute something the paper defines (the others are
# introspection, errors, teardown, options and the allocation-free variant)
CITED = ("lms_build_csr", "lms_build_csr_batched", "lms_reorder", "lms_reorder_device",
         "lms_reorder_with_quality", "lms_permute", "lms_smooth", "lms_sweep", "lms_quality",
         "lms_quality_batched", "lms_host_vertex_quality", "lms_reuse_profile")


def test_header_cites_the_paper_for_each_entry_point():
    text = open(lms.HEADER).read()
    for fn in CITED:
        assert fn in lms.header_functions(), fn
        m = re.search(r"\b" + fn + r"\(", text)
        block = text[:m.start()]
        comment = block[block.rfind("/*"):]
        assert re.search(r"(Eq\.|Algorithm|Section|Table|Figure) ?\d", comment), fn


def oracle_smoothing_csr(top, new2old):
    old2new = oord.inverse(new2old)
    n = top.n
    rp = [0]
    col = []
    for k in range(n):
        v = new2old[k]
        if not top.fixed[v]:
            col.extend(sorted(old2new[top.neighbours(v)].tolist()))
        rp.append(len(col))
    return np.array(rp, dtype=np.int32), np.array(col, dtype=np.int32)


@pytest.mark.parametrize("name", sorted(MESHES))
def test_csr_fixed_and_colours_match_oracle(name):
    m = MESHES[name]()
    top = omesh.topology(m.n, m.tri)
    M = lms.Mesh.build_csr(m.n, m.tri)
    info = M.info()
    assert info["n"] == m.n and info["n_tri"] == m.T
    assert info["nnz_full"] == top.nbr.size
    assert info["n_free"] == int((top.fixed == 0).sum())
    rp, col = M.csr()
    erp, ecol = oracle_smoothing_csr(top, np.arange(m.n))
    assert np.array_equal(rp, erp) and np.array_equal(col, ecol)
    fx, colour = M.vertex_data()
    assert np.array_equal(fx, top.fixed)
    ocol = oord.greedy_colouring(top)
    assert np.array_equal(colour, ocol)
    assert info["n_colors"] == ocol.max() + 1
    assert info["max_degree"] == top.degree[top.fixed == 0].max()


def test_library_colouring_equals_the_hand_traced_example():
    with open(os.path.join(HERE, "golden", "colouring_example.json")) as f:
        g = json.load(f)
    tri = np.array(g["tri"], dtype=np.int32)
    M = lms.Mesh.build_csr(g["n"], tri)
    fx, colour = M.vertex_data()
    assert colour.tolist() == g["colour"]
    assert M.info()["n_colors"] == len(g["colour_lists"])
    # relabelling carries the colours along with the vertices
    p = M.reorder("random", seed=3)
    assert M.vertex_data()[1].tolist() == np.array(g["colour"])[p].tolist()


@pytest.mark.parametrize("name", sorted(MESHES))
def test_host_vertex_quality_bitwise(name):
    m = MESHES[name]()
    M = lms.Mesh.build_csr(m.n, m.tri)
    assert np.array_equal(M.host_vertex_quality(m.x, m.y), oq.vertex_quality(m.x, m.y, m.tri, m.n))


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("kind", ["ori", "bfs", "rdr", "random"])
def test_orderings_match_oracle(name, kind):
    m = MESHES[name]()
    top = omesh.topology(m.n, m.tri)
    M = lms.Mesh.build_csr(m.n, m.tri)
    seed = 1002
    p = M.reorder(kind, seed=seed, x0=m.x, y0=m.y)
    if kind == "ori":
        e = oord.ori(top)
    elif kind == "bfs":
        e = oord.bfs(top)
    elif kind == "rdr":
        e = oord.rdr(top, oq.vertex_quality(m.x, m.y, m.tri, m.n))
    else:
        e = oord.random_order(m.n, seed)
    assert np.array_equal(p, e)
    assert np.array_equal(M.order(), e)
    assert M.info()["ordering"] == lms.ORDERINGS[kind]
    # the relabelled adjacency, fixed flags and colours follow the ordering
    rp, col = M.csr()
    erp, ecol = oracle_smoothing_csr(top, e)
    assert np.array_equal(rp, erp) and np.array_equal(col, ecol)
    fx, colour = M.vertex_data()
    assert np.array_equal(fx, top.fixed[e])
    assert np.array_equal(colour, oord.greedy_colouring(top)[e])


def test_reorders_replace_not_compose():
    m = MESHES["ocean120"]()
    M = lms.Mesh.build_csr(m.n, m.tri)
    a = M.reorder("random", seed=5)
    M.reorder("bfs")
    b = M.reorder("random", seed=5)
    assert np.array_equal(a, b)
    M.reorder("ori")
    rp, col = M.csr()
    top = omesh.topology(m.n, m.tri)
    erp, ecol = oracle_smoothing_csr(top, np.arange(m.n))
    assert np.array_equal(col, ecol)


def test_rdr_golden_examples_through_library():
    g = golden()
    for key in ("grid3", "grid4"):
        ex = g[key]
        M = lms.Mesh.build_csr(ex["n"], ex["tri"])
        assert M.reorder_with_quality(ex["q"]).tolist() == ex["rdr"]
    ex = g["grid3"]
    M = lms.Mesh.build_csr(ex["n"], ex["tri"])
    assert M.reorder_with_quality([0.5] * 9).tolist() == ex["rdr_all_equal_q"]
    ex = g["grid4"]
    M = lms.Mesh.build_csr(ex["n"], ex["tri"])
    assert M.reorder("bfs").tolist() == ex["bfs"]


def test_rdr_with_given_quality_matches_oracle_on_random_q():
    m = MESHES["ocean_ragged"]()
    top = omesh.topology(m.n, m.tri)
    q = np.random.default_rng(3).random(m.n)
    q[::7] = 0.25          # many exact ties: the label decides
    M = lms.Mesh.build_csr(m.n, m.tri)
    assert np.array_equal(M.reorder_with_quality(q), oord.rdr(top, q))


def test_user_fixed_mask():
    m = meshgen.jittered_grid(20, seed=3)
    fixed = np.zeros(m.n, dtype=np.uint8)
    fixed[::5] = 1
    top = omesh.topology(m.n, m.tri, fixed=fixed)
    M = lms.Mesh.build_csr(m.n, m.tri, fixed=fixed)
    fx, _ = M.vertex_data()
    assert np.array_equal(fx, fixed)
    rp, col = M.csr()
    erp, ecol = oracle_smoothing_csr(top, np.arange(m.n))
    assert np.array_equal(rp, erp) and np.array_equal(col, ecol)


def test_batched_orderings_are_per_mesh():
    ms = meshgen.batch(count=5, seed=4, n_min=200, n_max=3000)
    u, v_off, t_off = meshgen.concat(ms)
    local = np.concatenate([m.tri for m in ms])
    M = lms.Mesh.build_csr_batched(v_off, t_off, local)
    info = M.info()
    assert info["n_mesh"] == 5 and info["n"] == u.n
    top = omesh.topology(u.n, u.tri)
    rp, col = M.csr()
    erp, ecol = oracle_smoothing_csr(top, np.arange(u.n))
    assert np.array_equal(col, ecol)
    q = oq.vertex_quality(u.x, u.y, u.tri, u.n)
    for kind in ("bfs", "rdr", "random"):
        p = M.reorder(kind, seed=7, x0=u.x, y0=u.y)
        for i, m in enumerate(ms):
            seg = p[v_off[i]:v_off[i + 1]] - v_off[i]
            t = omesh.topology(m.n, m.tri)
            if kind == "bfs":
                e = oord.bfs(t)
            elif kind == "rdr":
                e = oord.rdr(t, q[v_off[i]:v_off[i + 1]])
            else:
                e = oord.random_order(m.n, 7 + i)
            assert np.array_equal(seg, e), (kind, i)


@pytest.mark.parametrize("tri,n", [
    ([[0, 1, 3]], 3),                         # id out of range
    ([[0, 1, 1]], 3),                         # repeated vertex
    ([[0, 1, 2], [0, 1, 3], [1, 0, 4]], 5),   # edge in three triangles
    ([[0, 1, 2]], 4),                         # unreferenced vertex
    ([[0, -1, 2]], 3),                        # negative id
])
def test_malformed_mesh_errors(tri, n):
    with pytest.raises(lms.LmsError) as e:
        lms.Mesh.build_csr(n, tri)
    assert e.value.status == 2


def test_argument_errors():
    lib = lms.load()
    import ctypes
    h = ctypes.c_void_p()
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    assert lib.lms_build_csr(0, 1, lms._np_ptr(tri), None, ctypes.byref(h)) == 1
    assert lib.lms_build_csr(3, 0, lms._np_ptr(tri), None, ctypes.byref(h)) == 1
    assert lib.lms_build_csr(3, 1, None, None, ctypes.byref(h)) == 1
    assert lib.lms_build_csr(3, 1, lms._np_ptr(tri), None, None) == 1
    assert "NULL" in lib.lms_last_error().decode()
    assert lib.lms_reorder(None, 0, 0, None, None, None) == 1
    assert lib.lms_destroy(None) == 0
    m = meshgen.jittered_grid(10, seed=1)
    M = lms.Mesh.build_csr(m.n, m.tri)
    with pytest.raises(lms.LmsError) as e:
        M.reorder(7)
    assert e.value.status == 1
    with pytest.raises(lms.LmsError) as e:          # RDR without coordinates
        M.reorder("rdr")
    assert e.value.status == 1
    x = m.x.copy()
    x[3] = np.nan
    with pytest.raises(lms.LmsError) as e:
        M.reorder("rdr", x0=x, y0=m.y)
    assert e.value.status == 1
    # the failed calls left the handle as it was
    assert M.info()["ordering"] == lms.ORI
    assert lib.lms_build_csr_batched(0, None, None, None, None, ctypes.byref(h)) == 1


def test_oversized_triangle_count_is_rejected_before_allocating():
    lib = lms.load()
    import ctypes
    h = ctypes.c_void_p()
    tri = np.zeros(3, dtype=np.int32)
    assert lib.lms_build_csr(3, (1 << 40) + 1, lms._np_ptr(tri), None, ctypes.byref(h)) == 1


@pytest.mark.parametrize("source", ["lms_device.hip", "lms_reorder.hip"])
def test_no_kernel_spills_to_scratch(source):
    # every device kernel must keep its arrays in registers: a kernel with
    # private (scratch) memory runs its loads through memory and slows down
    import subprocess
    from paper_1606_00803_amd import build as b
    src = os.path.join(b.CSRC, source)
    cmd = [b._hipcc(), *b.COMMON, f"--offload-arch={b.ARCH}", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-Rpass-analysis=kernel-resource-usage",
           "--cuda-device-only", "-c", src, "-o", os.devnull]
    out = subprocess.run(cmd, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", out.stderr)
    scratch = [int(v) for v in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out.stderr)]
    assert len(names) == len(scratch) and len(names) > (50 if source == "lms_device.hip" else 5)
    spilled = [n for n, sc in zip(names, scratch) if sc > 0]
    assert not spilled, spilled


def test_count_division_is_ieee_division(tmp_path):
    # the sweep kernels' quotient (a multiplication and two fused
    # multiply-adds from a table of 1/c) against IEEE division, bit for bit,
    # in float64 and float32, on the host
    import subprocess
    from paper_1606_00803_amd import build as b
    exe = str(tmp_path / "division_check")
    cmd = [b._hipcc(), "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", f"--offload-arch={b.ARCH}",
           "-Wno-unused-command-line-argument", f"-I{b.CSRC}", os.path.join(os.path.dirname(__file__),
                                                                         "division_check.hip"), "-o", exe]
    out = subprocess.run(cmd, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr[-2000:]
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-2000:]
    assert "float64: " in run.stdout and "float32: " in run.stdout


@pytest.mark.parametrize("kind", ["ori", "bfs", "rdr", "random"])
def test_reuse_profile_matches_oracle(kind):
    from oracle import reuse as ore
    m = meshgen.jittered_grid(40, 37, seed=3, land_fraction=0.3)
    top = omesh.topology(m.n, m.tri)
    M = lms.Mesh.build_csr(m.n, m.tri)
    M.reorder(kind, seed=7, x0=m.x, y0=m.y)
    fr = (0.0, 0.5, 0.75, 0.9, 0.99, 1.0)
    for line, rec in ((128, 16), (64, 8)):
        a = M.reuse_profile(fr, line_bytes=line, record_bytes=rec)
        b = ore.profile(top, M.order(), fr, line_bytes=line, record_bytes=rec)
        for key in ("accesses", "cold", "quantiles", "max", "lines_per_wave", "max_lines_per_wave"):
            assert a[key] == b[key], (kind, key)
        assert abs(a["mean"] - b["mean"]) <= 1e-12 * max(1.0, b["mean"])


@pytest.mark.parametrize("kind", ["ori", "bfs", "rdr", "random"])
def test_algorithm1_trace_profile_matches_oracle(kind):
    # the trace of Algorithm 1's loop body: smoothing plus quality upkeep
    from oracle import reuse as ore
    m = meshgen.jittered_grid(21, 19, seed=4, land_fraction=0.3)
    top = omesh.topology(m.n, m.tri)
    M = lms.Mesh.build_csr(m.n, m.tri)
    M.reorder(kind, seed=7, x0=m.x, y0=m.y)
    fr = (0.0, 0.5, 0.75, 0.9, 0.99, 1.0)
    a = M.reuse_profile(fr, trace="algorithm1")
    b = ore.profile(top, M.order(), fr, trace="algorithm1")
    for key in ("accesses", "cold", "quantiles", "max", "lines_per_wave", "max_lines_per_wave"):
        assert a[key] == b[key], (kind, key)
    assert abs(a["mean"] - b["mean"]) <= 1e-12 * max(1.0, b["mean"])
    # the smoothing part of it is the sweep trace
    assert a["accesses"] > M.reuse_profile(fr)["accesses"]


def test_reuse_profile_rejects_bad_arguments():
    m = meshgen.regular_grid(6)
    M = lms.Mesh.build_csr(m.n, m.tri)
    for kw in (dict(fractions=(1.5,)), dict(fractions=(-0.1,)), dict(line_bytes=0), dict(record_bytes=-4),
               dict(trace=2), dict(trace=-1)):
        with pytest.raises(lms.LmsError) as e:
            M.reuse_profile(**kw)
        assert e.value.status == 1                 # LMS_ERR_ARG


def test_reuse_profile_ranks_the_bulk_of_accesses_as_the_paper_does():
    # Section 5's reuse-distance study: RDR keeps most accesses far closer
    # than ORI and BFS, and random is worst.  (Here the walk restarts give RDR
    # a heavy tail instead, so the claim is checked on the 75% quantile.)
    m = meshgen.jittered_grid(300, 280, seed=12, land_fraction=0.3)
    M = lms.Mesh.build_csr(m.n, m.tri)
    q75, lines = {}, {}
    for kind in ("ori", "bfs", "rdr", "random"):
        M.reorder(kind, seed=5, x0=m.x, y0=m.y)
        p = M.reuse_profile((0.75,))
        q75[kind], lines[kind] = p["quantiles"][0], p["lines_per_wave"]
    assert q75["rdr"] < min(q75["ori"], q75["bfs"]) and max(q75["ori"], q75["bfs"]) < q75["random"], q75
    assert lines["random"] > 4 * max(lines["ori"], lines["bfs"], lines["rdr"]), lines


def test_algorithm1_trace_reproduces_table_2_ranking_at_the_90_percent_quantile():
    # Table 2 (first iteration, the paper's own verbose run): at the 90%
    # quantile RDR < BFS < ORI, with random orders far behind.  With the
    # quality upkeep of Algorithm 1 in the trace, the same ranking appears on
    # the synthetic ocean-like meshes.  Parity unpinned: the paper's meshes
    # and exact trace are not available.
    m = meshgen.jittered_grid(300, 280, seed=12, land_fraction=0.3)
    M = lms.Mesh.build_csr(m.n, m.tri)
    q90 = {}
    for kind in ("ori", "bfs", "rdr", "random"):
        M.reorder(kind, seed=5, x0=m.x, y0=m.y)
        q90[kind] = M.reuse_profile((0.9,), trace="algorithm1")["quantiles"][0]
    assert q90["rdr"] < q90["bfs"] < q90["ori"] < q90["random"], q90


def test_a_missing_library_fails_loudly(tmp_path):
    # no fallback: without the built library every entry point is unavailable
    with pytest.raises(OSError, match="not found"):
        lms.load(str(tmp_path / "liblms.so"))

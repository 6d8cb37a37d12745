"""Tile plans of the temporally blocked and one-pass multicolour sweeps,
simulated on the CPU (host logic, no GPU).

`tests/plan_sim/plan_sim.cpp` links the library's host sources, builds the
plans the device kernels read, runs Eq. 1 exactly as each plan directs (the
staged rows, the rows every sweep of a pass updates, their neighbour slots)
and compares bit for bit with plain sweeps over the whole mesh: Jacobi
sweeps for the halo and temporally blocked plans, colour-by-colour in-place sweeps
for the multicolour plans, at every pass depth the plan allows.  It also
sums the mesh quality from each plan's triangle records, as the
quality-fused passes do, against the per-vertex definition (Section 3.2).
A planted wrong neighbour slot and a planted wrong triangle count must make
every fitting plan shape fail.  Before the plans, the arrays the relabelling
installs (padded and colour-major adjacency, the sorted triangle list with
its weights and records, the vertex -> triangle lists) are checked against
the CSR and the input triangles.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LINE = re.compile(r"^(halo|tb|mc) (range|patch) ts=(\d+) k=(\d+) fits=([01]) tiles=(\d+) mismatches=(\d+) "
                  r"q_fits=([01]) q_err=(\S+)$")


@pytest.fixture(scope="module")
def plan_sim(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    out = tmp_path_factory.mktemp("plan_sim") / "plan_sim"
    csrc = os.path.join(ROOT, "paper_1606_00803_amd", "csrc")
    subprocess.run([gxx, "-O2", "-std=c++17", "-pthread", f"-I{ROOT}/include", f"-I{csrc}",
                    os.path.join(ROOT, "tests", "plan_sim", "plan_sim.cpp"), os.path.join(csrc, "lms_host.cpp"),
                    "-o", str(out)], check=True, timeout=600)
    return str(out)


@pytest.fixture(scope="module")
def mesh_file(tmp_path_factory):
    # ocean-like: holes, ragged sizes, ~27k vertices, tiles of 128-1024 rows
    m = meshgen.jittered_grid(211, 173, seed=17, land_fraction=0.3)
    path = tmp_path_factory.mktemp("plan_mesh") / "mesh.bin"
    with open(path, "wb") as fh:
        np.array([m.n], dtype=np.int32).tofile(fh)
        np.array([m.T], dtype=np.int64).tofile(fh)
        np.ascontiguousarray(m.tri, dtype=np.int32).tofile(fh)
        m.x.astype(np.float64).tofile(fh)
        m.y.astype(np.float64).tofile(fh)
    return str(path)


PATCHES = re.compile(r"^patches ts=(\d+) count=(\d+) wrong=(\d+)$")


def run(plan_sim, mesh_file, *args, patches=None):
    r = subprocess.run([plan_sim, mesh_file, *args], capture_output=True, text=True, timeout=300)
    lines = r.stdout.splitlines()
    # the arrays the relabelling installed (padded copies, triangles, lists)
    assert lines and lines[0] == "relabel wrong=0", r.stdout + r.stderr
    # the patch sets of 256 and 1024 rows
    prow = [PATCHES.match(line) for line in lines[1:3]]
    assert all(prow), r.stdout + r.stderr
    if patches is not None:
        patches.extend((int(g[1]), int(g[2]), int(g[3])) for g in prow)
    rows = [LINE.match(line) for line in lines[3:]]
    assert all(rows) and len(rows) == 18, r.stdout + r.stderr
    return r.returncode, [(g[1], g[2], int(g[3]), int(g[4]), g[5] == "1", int(g[7]), g[8] == "1", float(g[9]))
                          for g in rows]


@pytest.mark.parametrize("ordering", ["ori", "bfs", "rdr", "random"])
def test_plans_reproduce_plain_sweeps_bit_for_bit(plan_sim, mesh_file, ordering):
    patches = []
    rc, rows = run(plan_sim, mesh_file, ordering, patches=patches)
    assert rc == 0, rows
    # patches partition the free rows into connected pieces of at most ts rows
    assert all(wrong == 0 for _, _, wrong in patches), patches
    assert all(r[5] == 0 for r in rows), rows
    fit = [r for r in rows if r[4]]
    # the fused-quality records sum to the definition's n*Q (another order)
    assert all(r[6] and 0.0 <= r[7] <= 1e-12 for r in fit if r[0] != "halo"), rows
    # patch tiles fit under every ordering; row ranges give up on random labels
    assert sum(1 for r in fit if r[1] == "patch") == 8, rows
    assert len(fit) >= (10 if ordering == "random" else 14), rows
    # several sweeps per pass are covered for both plan kinds
    assert any(r[0] == "tb" and r[3] == 4 for r in fit) and any(r[0] == "mc" and r[3] == 3 for r in fit)


def test_patch_growth_leaves_few_fragments_under_every_ordering(plan_sim, mesh_file):
    # each patch grows from the border of those before it, so the labels
    # barely change how many patches the free rows fall into
    counts = {}
    for ordering in ("ori", "bfs", "rdr", "random"):
        patches = []
        run(plan_sim, mesh_file, ordering, patches=patches)
        counts[ordering] = {ts: count for ts, count, _ in patches}
    m = meshgen.jittered_grid(211, 173, seed=17, land_fraction=0.3)
    for ts in (256, 1024):
        low = min(c[ts] for c in counts.values())
        assert all(c[ts] <= 1.2 * low for c in counts.values()), counts
        assert low >= m.n * 0.6 / ts, counts  # at least the free rows / ts


def test_planted_mistakes_are_caught(plan_sim, mesh_file):
    rc, rows = run(plan_sim, mesh_file, "rdr", "plant")
    assert rc == 1
    fit = [r for r in rows if r[4]]
    assert fit and all(r[5] > 0 for r in fit), rows
    assert all(r[6] and r[7] > 1e-9 for r in fit if r[0] != "halo"), rows


def test_plan_builders_under_address_and_undefined_behaviour_sanitizers(tmp_path, mesh_file):
    # the host plan builders and the simulation, built with the sanitizers
    # (host code only), on the orderings whose plans scatter the most
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = tmp_path / "plan_sim_san"
    csrc = os.path.join(ROOT, "paper_1606_00803_amd", "csrc")
    subprocess.run([gxx, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-std=c++17", "-pthread", f"-I{ROOT}/include", f"-I{csrc}",
                    os.path.join(ROOT, "tests", "plan_sim", "plan_sim.cpp"), os.path.join(csrc, "lms_host.cpp"),
                    "-o", str(exe)], check=True, timeout=900)
    for ordering in ("rdr", "random"):
        r = subprocess.run([str(exe), mesh_file, ordering], capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]

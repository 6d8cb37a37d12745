#!/usr/bin/env python3
"""Benchmark: Laplacian mesh smoothing sweeps on one MI355X.

Default workload (the JSON line the metric is quoted on): the ocean-like mesh
(1000 x 1000 jittered grid, ~30% of the cells cut out as disc-union holes,
hole rims fixed; 708,312 vertices, 686,911 free), 50 Jacobi sweeps per step
(Eq. 1 applied to every free vertex), float64.  The headline value is
vertex-updates/s under the RDR ordering (Algorithm 2); the line also carries
every ordering (ORI, BFS, RDR, random) in float64 and float32, the roofline
of the sweep kernel, the multicolour and quality passes, a STREAM-copy
reference, host preprocessing times and the oracle's CPU rate.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
    python bench.py --workload graded16m|batch512|graded64m   (other configs)

A step is one lms_smooth call of K sweeps (one captured graph launch) on
coordinates already resident in HBM; the timed region covers exactly --steps
steps bracketed by torch.cuda.synchronize().
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
ORDER_NAMES = ["ori", "bfs", "rdr", "random"]
RANDOM_SEED = 1002
METRIC = "vertex-updates/sec and % HBM roofline per ordering (ORI/BFS/RDR/random), FP64 vs FP32"
COUNTERS = {"ocean": os.path.join(ROOT, "profiles", "sweep_ocean_rdr_f64_counters.md"),
            "graded16m": os.path.join(ROOT, "profiles", "sweep_graded16m_counters.md"),
            "batch512": os.path.join(ROOT, "profiles", "sweep_batch512_counters.md")}
# the kernels' source: counter summaries taken on other kernel code are not used
DEVICE_SRC = os.path.join(ROOT, "paper_1606_00803_amd", "csrc", "lms_kernels.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_bytes(n, n_free, nnz, s):
    """Algorithmic bytes of one sweep: read every coordinate pair once, write
    every free one once, read row_ptr and the neighbour indices once."""
    return 2 * s * n + 2 * s * n_free + 4 * (n + 1) + 4 * nnz


def quality_bytes(n, T, s):
    """Algorithmic bytes of one quality pass: three int32 corners and one
    float64 weight per triangle, every coordinate pair once."""
    return 20 * T + 2 * s * n


def device_source_hash():
    with open(DEVICE_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counters_traffic(kernel_name, prec, path):
    """HBM traffic per launch (FETCH_SIZE + WRITE_SIZE, calibrated) from a
    committed counter summary, when it was taken on the current kernel source;
    the summary lists every sweep variant the autotuner timed, per precision."""
    try:
        text = open(path).read()
    except OSError:
        return None
    src = re.search(r"^- source_sha256: (\S+)", text, flags=re.M)
    if not src or src.group(1) != device_source_hash():
        return None
    for name, p, traffic in re.findall(r"^\| `(\S+)` \| (f64|f32) \|[^|]*\| (\d+) \|", text, flags=re.M):
        if name == kernel_name and p == prec:
            return float(traffic)
    return None


class Timer:
    """HIP events on torch's current stream (the stream the library launches on)."""

    def __init__(self, torch):
        self.torch = torch
        self.s = torch.cuda.current_stream()
        self.e0 = torch.cuda.Event(enable_timing=True)
        self.e1 = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.w0 = time.perf_counter()
        self.e0.record(self.s)
        return self

    def __exit__(self, *a):
        self.e1.record(self.s)
        self.torch.cuda.synchronize()
        self.wall = time.perf_counter() - self.w0
        self.ms = self.e0.elapsed_time(self.e1)


def stream_copy_gbs(torch, mbytes=2048, reps=10):
    """Achieved bandwidth of a plain device copy (read + write bytes / time)."""
    n = max(1, int(mbytes * (1 << 20)) // 8)
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(2):
        b.copy_(a)
    with Timer(torch) as t:
        for _ in range(reps):
            b.copy_(a)
    del a, b
    return 2 * n * 8 * reps / (t.ms * 1e-3) / 1e9


def calibration_copy(torch, mb):
    """A device copy of known size (mb MiB), for scaling the memory counters;
    a 1 GiB fill in between evicts the source from the caches first."""
    if not mb:
        return
    a = torch.empty(mb << 17, dtype=torch.float64, device="cuda").fill_(1.0)
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(0.0)
    del flush
    torch.empty_like(a).copy_(a)
    torch.cuda.synchronize()
    del a


def run_fixed(torch, M, m, kind, prec, sweeps, steps, warmup, scheme="jacobi"):
    """Reorder, upload, time `steps` calls of `sweeps` sweeps.  Returns a dict."""
    from paper_1606_00803_amd import lms  # noqa: F401
    dt = torch.float64 if prec == "f64" else torch.float32
    x0 = torch.as_tensor(m.x, dtype=dt, device="cuda")
    y0 = torch.as_tensor(m.y, dtype=dt, device="cuda")
    x = torch.empty_like(x0)
    y = torch.empty_like(y0)
    M.permute(x0, y0, x, y)
    tx = torch.empty_like(x)
    ty = torch.empty_like(y)
    for _ in range(warmup):
        M.smooth(x, y, tx, ty, scheme=scheme, max_iters=sweeps, check_quality=False)
    # one event after every step as well: per-step median and minimum, with no
    # synchronisation inside the timed region
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    with Timer(torch) as t:
        for i in range(steps):
            M.smooth(x, y, tx, ty, scheme=scheme, max_iters=sweeps, check_quality=False)
            marks[i].record(t.s)
    per_step = [t.e0.elapsed_time(marks[0])] + [marks[i - 1].elapsed_time(marks[i]) for i in range(1, steps)]
    launch_us = marginal_launch_us(torch, M, x, y, tx, ty, scheme) if scheme == "jacobi" else None
    info = M.info()
    s = 8 if prec == "f64" else 4
    b = sweep_bytes(info["n"], info["n_free"], info["nnz"], s)
    launches = steps * sweeps
    sweep_us = t.ms * 1e3 / launches
    out = dict(sweep_kernel=sweep_variant(M.sweep_config(prec), scheme),
               vertex_updates_per_s=info["n_free"] * launches / t.wall,
               ms_per_step=t.wall * 1e3 / steps, sweep_us_events=sweep_us,
               step_ms_median=float(np.median(per_step)), step_ms_min=float(min(per_step)),
               achieved_gbs=b / (sweep_us * 1e-6) / 1e9,
               frac_hbm=b / (sweep_us * 1e-6) / 1e9 / HBM_PEAK_GBS, bytes_per_sweep=b,
               wall=t.wall, ev_ms=t.ms)
    if launch_us is not None:
        out["launch_us_marginal"] = launch_us
    del x0, y0, tx, ty
    return out, (x, y)


def fp32_vs_fp64(torch, M, m, sweeps, scheme="jacobi"):
    """Position error of the float32 form against the float64 form on the same
    GPU: both run `sweeps` sweeps from P_0 under the handle's ordering; the
    max and RMS distance per vertex over the mesh extent."""
    out = {}
    for dt in (torch.float64, torch.float32):
        x0 = torch.as_tensor(m.x, dtype=dt, device="cuda")
        y0 = torch.as_tensor(m.y, dtype=dt, device="cuda")
        x, y = torch.empty_like(x0), torch.empty_like(y0)
        M.permute(x0, y0, x, y)
        M.smooth(x, y, scheme=scheme, max_iters=sweeps, check_quality=False)
        out[dt] = (x.double().cpu().numpy(), y.double().cpu().numpy())
    ext = float(np.ptp(np.stack([m.x, m.y], axis=1), axis=0).max())
    d = np.hypot(out[torch.float32][0] - out[torch.float64][0], out[torch.float32][1] - out[torch.float64][1]) / ext
    return dict(max=float(d.max()), rms=float(np.sqrt(np.mean(d ** 2))), sweeps=sweeps,
                normalised_by="mesh extent (largest bounding-box side)")


def marginal_launch_us(torch, M, x, y, tx, ty, scheme, reps=5):
    """Duration of one launch of the sweep kernel the handle runs for fixed K:
    HIP events around `reps` calls of 2k and of 10k sweeps (k sweeps per
    launch), the difference over the 8k extra sweeps, times k.  Pack, unpack
    and the call's own overhead cancel; the gaps between launches stay."""
    k = sweeps_per_launch(M.sweep_config("f64" if x.dtype == torch.float64 else "f32").split(" ")[0])
    k1, k2 = 2 * k, 10 * k
    ms = {}
    for K in (k1, k2):
        M.smooth(x, y, tx, ty, scheme=scheme, max_iters=K, check_quality=False)   # captures the graph
        with Timer(torch) as t:
            for _ in range(reps):
                M.smooth(x, y, tx, ty, scheme=scheme, max_iters=K, check_quality=False)
        ms[K] = t.ms
    return (ms[k2] - ms[k1]) * 1e3 / (reps * (k2 - k1) / k)


# The GPU machine gives one process a share of 16 host threads, whatever the
# affinity mask shows; the oracle's OpenMP schedule uses at most that many.
HOST_THREAD_SHARE = 16


def host_cores():
    """(threads the oracle uses, logical CPUs in the affinity mask, logical CPUs of the host)."""
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    return max(1, min(visible, HOST_THREAD_SHARE)), visible, os.cpu_count() or visible


def relabelled(m, top, new2old):
    """The oracle's view of mesh m under an ordering: input vertex new2old[k]
    becomes label k (coordinates gathered, triangles renamed, neighbour lists
    rebuilt ascending in the new labels)."""
    from oracle import mesh as omesh
    from oracle import orderings as oord
    old2new = oord.inverse(new2old)
    tri = old2new[np.asarray(m.tri, dtype=np.int64)]
    return omesh.topology(m.n, tri), np.ascontiguousarray(m.x[new2old]), np.ascontiguousarray(m.y[new2old])


def cpu_baseline(m, sweeps, budget_s=3.0, one_core_s=2.0, orderings=("rdr", "ori", "bfs", "random"),
                 headline="rdr"):
    """The oracle's float64 Jacobi sweep (plain C, OpenMP static schedule over
    evenly divided vertices, as in the paper's Section 5.1) on the host, under
    each ordering the oracle computes itself: all the threads of the process's
    share, and one thread.  `value` is the headline ordering's rate."""
    from oracle import mesh as omesh
    from oracle import orderings as oord
    from oracle import quality as oq
    from oracle import smooth as osm
    cores, visible, logical = host_cores()
    top0 = omesh.topology(m.n, m.tri)
    free = int((top0.fixed == 0).sum())
    per = {}
    for kind in orderings:
        t0 = time.perf_counter()
        if kind == "ori":
            p = oord.ori(top0)
        elif kind == "bfs":
            p = oord.bfs(top0)
        elif kind == "rdr":
            p = oord.rdr(top0, oq.vertex_quality(m.x, m.y, m.tri, m.n))
        else:
            p = oord.random_order(m.n, RANDOM_SEED)
        t_order = time.perf_counter() - t0
        top, x, y = relabelled(m, top0, p)
        row = {"oracle_order_seconds": t_order}
        for label, threads, budget in (("all", cores, budget_s), ("one_core", 1, one_core_s)):
            # runs of k sweeps (fewer than the workload's when one run would
            # overshoot the budget) repeated for about `budget` seconds
            k = max(1, min(sweeps, int(budget * 2e7 * threads / max(1, free))))
            reps = 0
            w0 = time.perf_counter()
            while reps < 1 or time.perf_counter() - w0 < budget:
                osm.jacobi(top, x, y, k, threads=threads)
                reps += 1
            wall = time.perf_counter() - w0
            row[label] = dict(value=free * k * reps / wall, threads=threads,
                              sample=f"{k} sweeps x {reps} runs in {wall:.2f} s")
        per[kind] = row
        log(f"oracle {kind:7s}: {row['all']['value'] / 1e9:.3f} G upd/s on {cores} threads, "
            f"{row['one_core']['value'] / 1e9:.3f} G on one")
    h = per[headline]
    out = dict(value=h["all"]["value"], unit="vertex-updates/s", cores=cores, kind="oracle",
               sample=f"{sweeps}-sweep float64 Jacobi runs of the full workload ({m.n} vertices) in "
                      f"{headline.upper()} labels, {h['all']['sample']}, OpenMP static schedule over "
                      f"{cores} threads (the process's host share; {visible} CPUs in its affinity mask, "
                      f"{logical} on the host)",
               host_cpu=host_cpu_model(), affinity_cpus=visible, host_logical_cpus=logical,
               one_core_value=h["one_core"]["value"], per_ordering=per)
    # the paper's gain metric (T_algo - T_RDR) / T_algo on the CPU (Figure 13)
    if "rdr" in per:
        for label in ("all", "one_core"):
            out[f"rdr_gain_{label}"] = {a: 1.0 - per[a][label]["value"] / per["rdr"][label]["value"]
                                        for a in per if a != "rdr"}
    return out, top0


def host_cpu_model():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import subprocess
        r = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        info = dict(l.split(":", 1) for l in r.stdout.splitlines() if ":" in l)
        info = {k.strip(): v.strip() for k, v in info.items()}
        parts = [info.get("Model name") or model or "unknown CPU"]
        for key in ("Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)"):
            if key in info:
                parts.append(f"{key} {info[key]}")
        return ", ".join(parts)
    except Exception:
        return model


def result_line(value, steps, warmup, ms_per_step, dtype, config, roofline, cpu, **extra):
    out = {"metric": METRIC, "value": value, "unit": "vertex-updates/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic", "config": config,
           "roofline": roofline, "cpu_baseline": cpu}
    out.update(extra)
    return out


def sweep_variant(config, scheme="jacobi"):
    """The variant a fixed-K call ran, from the library's sweep_config string:
    its first name for Jacobi, the "colour=" one for multicolour."""
    if scheme == "jacobi":
        return config.split(" ")[0]
    m = re.search(r"(?:^| )colour=(\S+)", config)
    return m.group(1) if m else "colour"


def sweeps_per_launch(kernel_name):
    """A temporally blocked variant ("tb/.../k2/...") runs k sweeps per launch."""
    m = re.search(r"^tb/.*?/k(\d+)/", kernel_name)
    return int(m.group(1)) if m else 1


def roofline_of(r, prec="f64", workload="ocean"):
    # one launch processes k sweeps' worth of vertex updates: its algorithmic
    # bytes are k x B_sweep, over a launch that lasts k x the time per sweep
    k = sweeps_per_launch(r["sweep_kernel"])
    traffic = counters_traffic(r["sweep_kernel"], prec, COUNTERS[workload]) if workload in COUNTERS else None
    # the launch's own duration (marginal over fixed-K runs) when measured,
    # else the whole call's time per launch (pack, unpack and overhead included)
    launch_us = r.get("launch_us_marginal") or k * r["sweep_us_events"]
    achieved = k * r["bytes_per_sweep"] / (launch_us * 1e-6) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
           "kernel": "sweep " + r["sweep_kernel"], "sweeps_per_launch": k,
           "bytes_per_launch": k * r["bytes_per_sweep"], "avg_launch_us": launch_us,
           "avg_launch_us_whole_call": k * r["sweep_us_events"],
           "launch_duration": "marginal" if r.get("launch_us_marginal") else "whole call"}
    # against the bytes one pass must move at least, whatever its depth: every
    # coordinate read once, every free one written once, the index read once
    # (one B_sweep per launch); this fraction cannot exceed 1 on HBM-resident data
    out["pass_floor_bytes"] = r["bytes_per_sweep"]
    out["frac_pass_floor"] = r["bytes_per_sweep"] / (launch_us * 1e-6) / 1e9 / HBM_PEAK_GBS
    if traffic is not None and launch_us > 0:
        # the bytes the launch really moves (counters) over its measured duration
        out["traffic_gbs"] = traffic / (launch_us * 1e-6) / 1e9
        out["traffic_frac"] = out["traffic_gbs"] / HBM_PEAK_GBS
        out["traffic_per_algorithmic_byte"] = traffic / out["bytes_per_launch"]
    return out


def with_stream_copy(torch, roof):
    """Add the rate of a plain device copy that moves as many bytes (read +
    write) as one launch of the dominant kernel, and the fraction of it the
    kernel reaches: the practical ceiling at this size, beside the HBM peak."""
    gbs = stream_copy_gbs(torch, mbytes=roof["bytes_per_launch"] / 2 / (1 << 20), reps=50)
    roof["stream_copy_same_bytes_gbs"] = gbs
    roof["frac_of_stream_copy"] = roof["achieved"] / gbs
    return roof


# ---------------------------------------------------------------- workloads

def bench_ocean(torch, args):
    import meshgen
    from paper_1606_00803_amd import lms
    SWEEPS = 50
    t0 = time.perf_counter()
    m = meshgen.ocean()
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    M = lms.Mesh.build_csr(m.n, m.tri)
    t_csr = time.perf_counter() - t0
    info = M.info()
    log(f"ocean mesh n={info['n']} n_free={info['n_free']} T={m.T} nnz={info['nnz']} "
        f"colours={info['n_colors']} gen={t_gen:.2f}s csr={t_csr:.2f}s")
    calibration_copy(torch, args.calibration_copy_mb)
    results, reorder_s = {}, {}
    for kind in [o for o in args.orderings.split(",") if o]:
        t0 = time.perf_counter()
        M.reorder(kind, seed=RANDOM_SEED, x0=m.x, y0=m.y)
        reorder_s[kind] = time.perf_counter() - t0
        for prec in ("f64", "f32"):
            r, _ = run_fixed(torch, M, m, kind, prec, SWEEPS, args.steps, args.warmup)
            results[f"{kind}_{prec}"] = r
            log(f"{kind:7s} {prec}: {r['vertex_updates_per_s'] / 1e9:7.2f} G upd/s  sweep "
                f"{r['sweep_us_events']:7.2f} us  {r['achieved_gbs']:8.1f} GB/s  [{r['sweep_kernel']}]")
            if kind == "rdr" and prec == "f64":
                log("sweep variants (RDR, f64):", M.sweep_config("f64"))
    extras = {}
    if not args.no_extras:
        M.reorder("rdr", x0=m.x, y0=m.y)
        extras["fp32_vs_fp64_rdr"] = fp32_vs_fp64(torch, M, m, SWEEPS)
        log(f"float32 against float64 after {SWEEPS} sweeps: max {extras['fp32_vs_fp64_rdr']['max']:.3e}, "
            f"rms {extras['fp32_vs_fp64_rdr']['rms']:.3e} of extent")
        r, (x, y) = run_fixed(torch, M, m, "rdr", "f64", SWEEPS, args.steps, 1, scheme="multicolor")
        extras["multicolor_rdr_f64"] = {k: r[k] for k in ("vertex_updates_per_s", "sweep_us_events", "sweep_kernel")}
        extras["multicolor_rdr_f64"]["colours"] = info["n_colors"]
        M.quality(x, y)
        with Timer(torch) as t:
            for _ in range(args.steps):
                M.quality(x, y)
        qb = quality_bytes(info["n"], m.T, 8)
        extras["quality_pass"] = dict(us_per_call_incl_host_sync=t.wall * 1e6 / args.steps,
                                      algorithmic_bytes=qb)
        x0 = torch.as_tensor(m.x, dtype=torch.float64, device="cuda")
        y0 = torch.as_tensor(m.y, dtype=torch.float64, device="cuda")
        # to the paper's criterion: quality fused into the sweep passes (the
        # default), sweep + separate quality pass, and the multicolour scheme
        for label, flag, scheme in (("", "1", "jacobi"), ("_separate_quality", "0", "jacobi"),
                                    ("_multicolour", "1", "multicolor")):
            os.environ["LMS_FUSED_QUALITY"] = flag
            try:
                M.permute(x0, y0, x, y)
                M.smooth(x, y, max_iters=2000, tol=5e-6, scheme=scheme)   # tunes and captures the graphs
                M.permute(x0, y0, x, y)
                with Timer(torch) as t:
                    rr = M.smooth(x, y, max_iters=2000, tol=5e-6, scheme=scheme)
            finally:
                os.environ.pop("LMS_FUSED_QUALITY", None)
            extras["to_criterion_rdr_f64" + label] = dict(iters=rr["iters"], stopped_by=rr["stopped_by"],
                                                          q0=rr["q0"], q_final=rr["q_final"], seconds=t.wall)
            log(f"to the criterion{label.replace('_', ' ')}: {rr['iters']} sweeps in {t.wall * 1e3:.3f} ms")
        # locality of each ordering (host): reuse-distance quantiles of one
        # sweep's access trace (Table 2's measure) and cache lines per wavefront
        extras["reuse_profile"] = {}
        extras["reuse_profile_algorithm1"] = {}
        for kind in ORDER_NAMES:
            M.reorder(kind, seed=RANDOM_SEED, x0=m.x, y0=m.y)
            p = M.reuse_profile((0.5, 0.75, 0.9, 1.0))
            extras["reuse_profile"][kind] = dict(quantiles_50_75_90_100=p["quantiles"], mean=p["mean"],
                                                 accesses=p["accesses"], lines_per_wave=p["lines_per_wave"])
            log(f"reuse distance {kind:7s}: quantiles 50/75/90/100% {p['quantiles']}  "
                f"lines per wavefront {p['lines_per_wave']:.1f}")
            # the trace of Algorithm 1's loop body: the sweep plus the quality upkeep
            p = M.reuse_profile((0.5, 0.75, 0.9, 1.0), trace="algorithm1")
            extras["reuse_profile_algorithm1"][kind] = dict(quantiles_50_75_90_100=p["quantiles"], mean=p["mean"],
                                                            accesses_per_vertex=p["accesses"] / info["n"])
            log(f"reuse distance {kind:7s} (Algorithm 1 trace): quantiles 50/75/90/100% {p['quantiles']}")
        extras["stream_copy_gbs"] = stream_copy_gbs(torch)
        extras["host_seconds"] = dict(generate=t_gen, build_csr=t_csr,
                                      **{f"reorder_{k}": v for k, v in reorder_s.items()})
        # the same reorders with the breadth-first search and the relabelling
        # on the GPU (same result)
        dev_s = {}
        for kind in ORDER_NAMES:
            want = M.reorder(kind, seed=RANDOM_SEED, x0=m.x, y0=m.y)
            M.reorder_device(kind, seed=RANDOM_SEED, x0=m.x, y0=m.y)      # uploads the input arrays once
            t0 = time.perf_counter()
            got = M.reorder_device(kind, seed=RANDOM_SEED, x0=m.x, y0=m.y)
            dev_s[kind] = time.perf_counter() - t0
            assert np.array_equal(want, got)
            log(f"reorder {kind:7s}: host {reorder_s.get(kind, float('nan')):.3f} s, device {dev_s[kind]:.3f} s")
        extras["device_reorder_seconds"] = dev_s
        g = {k: results.get(f"{k}_f64", {}).get("vertex_updates_per_s") for k in ORDER_NAMES}
        if g.get("rdr") and g.get("ori") and g.get("bfs"):
            # the paper's gain metric (T_algo - T_RDR) / T_algo, here on the GPU
            extras["rdr_gain_f64"] = {a: 1.0 - g[a] / g["rdr"] for a in ("ori", "bfs", "random") if g.get(a)}
        # the paper's own figures, quoted with their hardware (context, not measured here)
        extras["paper_context"] = {
            "hardware": "4x Intel Xeon E7-8837 (Westmere-EX), 32 cores, OpenMP static schedule (Section 5.1)",
            "speedup_rdr_32_cores_vs_ori_1_core": 75, "gain_rdr_vs_bfs": 0.32, "gain_rdr_vs_ori": 0.30,
            "precision": "float64", "workload": "nine Triangle meshes, 299k-393k vertices (Table 1), to dQ < 5e-6"}
        del x, y, x0, y0
    if not args.no_extras and not args.no_large:
        del M
        torch.cuda.empty_cache()
        extras.update(large_configs(torch, args))
    cpu = None
    if not args.no_cpu_baseline:
        cpu, _ = cpu_baseline(m, SWEEPS)
        log(f"oracle on {cpu['cores']} host threads: {cpu['value'] / 1e9:.3f} G upd/s")
    h = results.get("rdr_f64") or next(iter(results.values()))
    return result_line(
        h["vertex_updates_per_s"], args.steps, args.warmup, h["ms_per_step"], "f64",
        {"workload": "ocean-like mesh: 1000x1000 jittered grid, ~30% disc-union holes, "
                     f"{SWEEPS} Jacobi sweeps per step, RDR ordering, float64",
         "n": info["n"], "n_free": info["n_free"], "n_tri": m.T, "nnz": info["nnz"],
         "sweeps_per_step": SWEEPS, "mesh_sha256": meshgen.mesh_hash(m)},
        with_stream_copy(torch, roofline_of(h, "f64", "ocean")), cpu, per_ordering=strip(results), extras=extras)


def strip(results):
    return {k: {kk: vv for kk, vv in v.items() if kk not in ("wall", "ev_ms")} for k, v in results.items()}


def config_rows(torch, M, m, workload, kinds, sweeps, steps, warmup):
    """Fixed-K runs of `sweeps` sweeps under each ordering and precision, each
    with the roofline block of its sweep kernel."""
    rows, reorder_s = {}, {}
    for kind in kinds:
        t0 = time.perf_counter()
        M.reorder(kind, seed=RANDOM_SEED, x0=m.x, y0=m.y)
        reorder_s[kind] = time.perf_counter() - t0
        for prec in ("f64", "f32"):
            r, _ = run_fixed(torch, M, m, kind, prec, sweeps, steps, warmup)
            roof = roofline_of(r, prec, workload)
            rows[f"{kind}_{prec}"] = dict(vertex_updates_per_s=r["vertex_updates_per_s"],
                                          ms_per_step=r["ms_per_step"], sweep_kernel=r["sweep_kernel"],
                                          roofline=roof)
            log(f"{workload} {kind:7s} {prec}: {r['vertex_updates_per_s'] / 1e9:7.2f} G upd/s  frac "
                f"{roof['frac']:.3f}  pass floor {roof['frac_pass_floor']:.3f}  "
                f"physical {roof.get('traffic_frac', float('nan')):.3f}  [{r['sweep_kernel']}]")
    return rows, reorder_s


def to_criterion(torch, M, m, workload):
    """Algorithm 1 to the paper's criterion (Section 5.1: dQ < 5e-6), quality
    fused into the sweep passes, float64 and float32 coordinates, under the
    handle's ordering: sweeps, the stop, and the wall time of the call."""
    out = {}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        x0 = torch.as_tensor(m.x, dtype=dt, device="cuda")
        y0 = torch.as_tensor(m.y, dtype=dt, device="cuda")
        x, y = torch.empty_like(x0), torch.empty_like(y0)
        M.permute(x0, y0, x, y)
        M.smooth(x, y, max_iters=2000, tol=5e-6)              # tunes, builds plans, captures graphs
        M.permute(x0, y0, x, y)
        with Timer(torch) as t:
            r = M.smooth(x, y, max_iters=2000, tol=5e-6)
        out[prec] = dict(iters=r["iters"], stopped_by=r["stopped_by"], q0=r["q0"], q_final=r["q_final"],
                         seconds=t.wall, stop_variant=(re.search(r"stop=(\S+)", M.sweep_config(prec)) or [None, None])[1])
        log(f"{workload} to the criterion ({prec}): {r['iters']} sweeps in {t.wall * 1e3:.2f} ms")
        del x0, y0, x, y
    return out


def large_configs(torch, args):
    """The two HBM-resident configurations, in the default run: the graded
    16M-vertex mesh (100 sweeps) and the 512-mesh batch (30 sweeps), under RDR
    and ORI in float64 and float32, each with its roofline blocks and the
    float32 position error against the float64 form on the same GPU."""
    import meshgen
    from paper_1606_00803_amd import lms
    out = {}
    t0 = time.perf_counter()
    m = meshgen.graded16m()
    t_gen = time.perf_counter() - t0
    M = lms.Mesh.build_csr(m.n, m.tri)
    info = M.info()
    log(f"graded mesh n={info['n']} n_free={info['n_free']} T={m.T} nnz={info['nnz']} gen={t_gen:.1f}s")
    rows, reorder_s = config_rows(torch, M, m, "graded16m", ("rdr", "ori"), 100, args.large_steps, 1)
    M.reorder("rdr", x0=m.x, y0=m.y)
    err = fp32_vs_fp64(torch, M, m, 100)
    log(f"graded16m float32 against float64 after 100 sweeps: max {err['max']:.3e}, rms {err['rms']:.3e}")
    crit = to_criterion(torch, M, m, "graded16m")
    # the breadth-first ordering on the host and on the device (same order)
    t0 = time.perf_counter()
    want = M.reorder("bfs")
    reorder_s["bfs"] = time.perf_counter() - t0
    M.reorder_device("bfs")                  # uploads the input arrays once
    t0 = time.perf_counter()
    got = M.reorder_device("bfs")
    reorder_s["bfs_device"] = time.perf_counter() - t0
    assert np.array_equal(want, got)
    log(f"graded16m reorder bfs: host {reorder_s['bfs']:.3f} s, device {reorder_s['bfs_device']:.3f} s")
    out["graded16m"] = dict(workload="graded mesh refined 4x toward a seeded curve, 100 Jacobi sweeps per step",
                            n=info["n"], n_free=info["n_free"], n_tri=m.T, nnz=info["nnz"], sweeps_per_step=100,
                            steps=args.large_steps, per_ordering=rows, fp32_vs_fp64_rdr=err, to_criterion_rdr=crit,
                            host_seconds=dict(generate=t_gen, **{f"reorder_{k}": v for k, v in reorder_s.items()}))
    del M, m
    t0 = time.perf_counter()
    ms = meshgen.batch()
    u, v_off, t_off = meshgen.concat(ms)
    B = lms.Mesh.build_csr_batched(v_off, t_off, np.concatenate([mm.tri for mm in ms]))
    t_gen = time.perf_counter() - t0
    info = B.info()
    log(f"batch: {len(ms)} meshes, n={info['n']} T={u.T} nnz={info['nnz']} ({t_gen:.1f}s)")
    rows, reorder_s = config_rows(torch, B, u, "batch512", ("rdr", "ori"), 30, args.large_steps, 1)
    B.reorder("rdr", x0=u.x, y0=u.y)
    err = fp32_vs_fp64(torch, B, u, 30)
    log(f"batch512 float32 against float64 after 30 sweeps: max {err['max']:.3e}, rms {err['rms']:.3e}")
    out["batch512"] = dict(workload=f"batch of {len(ms)} jittered grids, sizes log-uniform 1k-200k vertices, "
                                    "30 sweeps per step, one launch per pass over all meshes",
                           n=info["n"], n_free=info["n_free"], n_mesh=len(ms), nnz=info["nnz"], sweeps_per_step=30,
                           steps=args.large_steps, per_ordering=rows, fp32_vs_fp64_rdr=err,
                           host_seconds=dict(generate_and_build=t_gen,
                                             **{f"reorder_{k}": v for k, v in reorder_s.items()}))
    return out


def bench_graded16m(torch, args):
    import meshgen
    from paper_1606_00803_amd import lms
    SWEEPS = 100
    t0 = time.perf_counter()
    m = meshgen.graded16m()
    t_gen = time.perf_counter() - t0
    M = lms.Mesh.build_csr(m.n, m.tri)
    info = M.info()
    log(f"graded mesh n={info['n']} n_free={info['n_free']} T={m.T} nnz={info['nnz']} gen={t_gen:.1f}s")
    calibration_copy(torch, args.calibration_copy_mb)
    results, reorder_s, finals, quality = {}, {}, {}, {}
    for kind in [o for o in args.orderings.split(",") if o in ("rdr", "ori", "bfs", "random")]:
        t0 = time.perf_counter()
        M.reorder(kind, seed=RANDOM_SEED, x0=m.x, y0=m.y)
        reorder_s[kind] = time.perf_counter() - t0
        for prec in ("f64", "f32"):
            r, (x, y) = run_fixed(torch, M, m, kind, prec, SWEEPS, args.steps, args.warmup)
            results[f"{kind}_{prec}"] = r
            log(f"{kind:7s} {prec}: {r['vertex_updates_per_s'] / 1e9:7.2f} G upd/s  sweep "
                f"{r['sweep_us_events']:8.2f} us  {r['achieved_gbs']:8.1f} GB/s  [{r['sweep_kernel']}]")
            if kind == "rdr" and not args.no_extras:
                # one clean run of exactly SWEEPS sweeps from P_0 for the error metric
                dt = torch.float64 if prec == "f64" else torch.float32
                x0 = torch.as_tensor(m.x, dtype=dt, device="cuda")
                y0 = torch.as_tensor(m.y, dtype=dt, device="cuda")
                M.permute(x0, y0, x, y)
                M.smooth(x, y, max_iters=SWEEPS, check_quality=False)
                M.permute(x, y, x0, y0, inverse=True)
                finals[prec] = (x0.double().cpu().numpy(), y0.double().cpu().numpy())
                # the quality pass (Section 3.2) under RDR, on the permuted P_0
                M.permute(x0, y0, x, y)
                M.quality(x, y)
                with Timer(torch) as t:
                    for _ in range(10):
                        M.quality(x, y)
                qb = quality_bytes(info["n"], m.T, 8 if prec == "f64" else 4)
                us = t.ms * 1e3 / 10
                quality[prec] = dict(us_per_call=us, algorithmic_bytes=qb, achieved_gbs=qb / (us * 1e-6) / 1e9)
                log(f"quality pass (RDR) {prec}: {us:.1f} us/call (incl. host read-back), "
                    f"{qb / (us * 1e-6) / 1e9:.0f} GB/s")
            del x, y
    extras = dict(host_seconds=dict(generate=t_gen, **{f"reorder_{k}": v for k, v in reorder_s.items()}))
    for prec, q in quality.items():
        extras[f"quality_pass_rdr_{prec}"] = q
    cpu = None
    if not args.no_cpu_baseline and "f32" in finals:
        cpu, top = cpu_baseline(m, SWEEPS, budget_s=1.0, one_core_s=0.5, orderings=("ori",), headline="ori")
        from oracle import smooth as osm
        ex, ey = osm.jacobi(top, m.x, m.y, SWEEPS, threads=cpu["cores"])
        ext = float(np.ptp(m.xy, axis=0).max())
        d32 = np.hypot(finals["f32"][0] - ex, finals["f32"][1] - ey) / ext
        d64 = np.maximum(np.abs(finals["f64"][0] - ex), np.abs(finals["f64"][1] - ey)) / ext
        extras["fp32_error_vs_fp64_oracle"] = dict(max=float(d32.max()), rms=float(np.sqrt(np.mean(d32 ** 2))),
                                                   sweeps=SWEEPS, normalised_by="mesh extent")
        extras["fp64_max_error_vs_oracle"] = float(d64.max())
        log(f"FP32 error vs FP64 oracle after {SWEEPS} sweeps: max {d32.max():.3e}, rms "
            f"{np.sqrt(np.mean(d32 ** 2)):.3e} of extent; FP64 max {d64.max():.3e}")
    h = results.get("rdr_f32") or next(iter(results.values()))
    return result_line(
        h["vertex_updates_per_s"], args.steps, args.warmup, h["ms_per_step"], "f32",
        {"workload": f"graded mesh refined 4x toward a seeded curve: {SWEEPS} Jacobi sweeps per step, "
                     "RDR ordering, float32 storage and accumulation",
         "n": info["n"], "n_free": info["n_free"], "n_tri": m.T, "nnz": info["nnz"], "sweeps_per_step": SWEEPS},
        with_stream_copy(torch, roofline_of(h, "f32", "graded16m")), cpu, per_ordering=strip(results),
        extras=extras)


def bench_batch512(torch, args):
    import meshgen
    from paper_1606_00803_amd import lms
    SWEEPS = 30
    t0 = time.perf_counter()
    ms = meshgen.batch()
    u, v_off, t_off = meshgen.concat(ms)
    local = np.concatenate([mm.tri for mm in ms])
    B = lms.Mesh.build_csr_batched(v_off, t_off, local)
    info = B.info()
    log(f"batch: {len(ms)} meshes, n={info['n']} T={u.T} nnz={info['nnz']} ({time.perf_counter() - t0:.1f}s)")
    calibration_copy(torch, args.calibration_copy_mb)
    results = {}
    for kind in ("ori", "rdr"):
        B.reorder(kind, seed=RANDOM_SEED, x0=u.x, y0=u.y)
        for prec in ("f64", "f32"):
            r, _ = run_fixed(torch, B, u, kind, prec, SWEEPS, args.steps, args.warmup)
            results[f"{kind}_{prec}"] = r
            log(f"{kind:7s} {prec}: {r['vertex_updates_per_s'] / 1e9:7.2f} G upd/s  sweep "
                f"{r['sweep_us_events']:8.2f} us  {r['achieved_gbs']:8.1f} GB/s  [{r['sweep_kernel']}]")
    extras = {"fp32_vs_fp64_rdr": fp32_vs_fp64(torch, B, u, SWEEPS)}
    log(f"float32 against float64 after {SWEEPS} sweeps: max {extras['fp32_vs_fp64_rdr']['max']:.3e}, "
        f"rms {extras['fp32_vs_fp64_rdr']['rms']:.3e} of extent")
    h = results["rdr_f64"]
    line = result_line(
        h["vertex_updates_per_s"], args.steps, args.warmup, h["ms_per_step"], "f64",
        {"workload": f"batch of {len(ms)} jittered grids, sizes log-uniform 1k-200k vertices, "
                     f"{SWEEPS} sweeps each in one launch per sweep, RDR per mesh, float64",
         "n": info["n"], "n_mesh": len(ms), "sweeps_per_step": SWEEPS},
        with_stream_copy(torch, roofline_of(h, "f64", "batch512")), None, per_ordering=strip(results),
        extras=extras)
    if args.no_extras:
        return line
    # the same meshes split by size class, each class a batch of its own: the
    # class that fits in LDS (<= 4096 vertices) runs all sweeps in one launch
    # and may beat the per-sweep byte formula; the others run per sweep
    by_size = {}
    for label, lo, hi in (("n_le_4096", 0, 4096), ("n_4097_50000", 4097, 50000), ("n_gt_50000", 50001, 1 << 40)):
        sub = [mm for mm in ms if lo <= mm.n <= hi]
        if len(sub) < 2:
            continue
        cu, cv, ct = meshgen.concat(sub)
        CB = lms.Mesh.build_csr_batched(cv, ct, np.concatenate([mm.tri for mm in sub]))
        CB.reorder("rdr", x0=cu.x, y0=cu.y)
        by_size[label] = dict(meshes=len(sub), n=cu.n)
        for prec in ("f64", "f32"):
            r, _ = run_fixed(torch, CB, cu, "rdr", prec, SWEEPS, args.steps, args.warmup)
            by_size[label][prec] = dict(vertex_updates_per_s=r["vertex_updates_per_s"],
                                        frac_of_hbm_by_sweep_formula=r["frac_hbm"], path=r["sweep_kernel"])
            log(f"size class {label:13s} ({len(sub):3d} meshes, n={cu.n:9d}) {prec}: "
                f"{r['vertex_updates_per_s'] / 1e9:7.2f} G upd/s  {r['frac_hbm']:.2f} of the HBM peak "
                f"by the per-sweep bytes  [{r['sweep_kernel']}]")
        del CB
    extras["by_size_class_rdr"] = by_size
    # a batch of small meshes (every one fits in LDS): all sweeps in one launch,
    # against the per-sweep path
    small = meshgen.batch(count=8192, seed=44, n_min=256, n_max=2000)
    su, sv, st_ = meshgen.concat(small)
    SB = lms.Mesh.build_csr_batched(sv, st_, np.concatenate([mm.tri for mm in small]))
    SB.reorder("rdr", x0=su.x, y0=su.y)
    for flag, label in (("1", "one_launch"), ("0", "per_sweep"), (None, "tuned")):
        if flag is not None:
            os.environ["LMS_SMALL_BATCH"] = flag
        try:
            for prec in ("f64", "f32"):
                r, _ = run_fixed(torch, SB, su, "rdr", prec, SWEEPS, args.steps, args.warmup)
                extras[f"small_batch_{label}_{prec}"] = dict(vertex_updates_per_s=r["vertex_updates_per_s"],
                                                             ms_per_step=r["ms_per_step"], path=r["sweep_kernel"])
                log(f"small batch ({len(small)} meshes, n={su.n}) {label:10s} {prec}: "
                    f"{r['vertex_updates_per_s'] / 1e9:7.2f} G upd/s")
        finally:
            os.environ.pop("LMS_SMALL_BATCH", None)
    return line


def bench_graded64m(torch, args):
    import meshgen
    from paper_1606_00803_amd import lms
    log("generating the 64M-vertex graded mesh ...")
    t0 = time.perf_counter()
    m = meshgen.graded64m()
    t_gen = time.perf_counter() - t0
    log(f"generated in {t_gen:.1f}s; building the adjacency ...")
    M = lms.Mesh.build_csr(m.n, m.tri)
    info = M.info()
    log(f"graded64m n={info['n']} n_free={info['n_free']} T={m.T} colours={info['n_colors']} gen={t_gen:.1f}s")
    runs = {}
    host = dict(generate=t_gen)
    for kind in ("rdr", "random"):
        log(f"reordering ({kind}) ...")
        t0 = time.perf_counter()
        want = M.reorder(kind, seed=RANDOM_SEED + 3, x0=m.x, y0=m.y)
        host[f"reorder_{kind}"] = time.perf_counter() - t0
        log(f"reordered in {host[f'reorder_{kind}']:.1f}s on the host; again with the relabelling on the GPU ...")
        t0 = time.perf_counter()
        got = M.reorder_device(kind, seed=RANDOM_SEED + 3, x0=m.x, y0=m.y)
        host[f"reorder_device_{kind}"] = time.perf_counter() - t0
        assert np.array_equal(want, got)
        log(f"reordered in {host[f'reorder_device_{kind}']:.1f}s (GPU relabelling, first call uploads the input)")
        x0 = torch.as_tensor(m.x, dtype=torch.float32, device="cuda")
        y0 = torch.as_tensor(m.y, dtype=torch.float32, device="cuda")
        x = torch.empty_like(x0)
        y = torch.empty_like(y0)
        for scheme, fused in (("jacobi", "1"), ("jacobi", "0"), ("multicolor", "1")):
            os.environ["LMS_FUSED_QUALITY"] = fused
            try:
                log(f"{kind} {scheme}: tuning, tile plans, graphs ...")
                M.permute(x0, y0, x, y)
                M.smooth(x, y, scheme=scheme, max_iters=2, tol=5e-6)   # tune, plans, graphs
                log("timing to the criterion ...")
                M.permute(x0, y0, x, y)
                with Timer(torch) as t:
                    r = M.smooth(x, y, scheme=scheme, max_iters=2000, tol=5e-6)
            finally:
                os.environ.pop("LMS_FUSED_QUALITY", None)
            name = f"{kind}_{scheme}" + ("_separate_quality" if fused == "0" else "")
            runs[name] = dict(iters=r["iters"], stopped_by=r["stopped_by"], q0=r["q0"],
                              q_final=r["q_final"], seconds_to_criterion=t.wall,
                              vertex_updates_per_s_incl_quality=info["n_free"] * r["iters"] / t.wall)
            if fused == "1":
                # sweep-only rate (as many fixed sweeps, no quality) and the
                # cost of one quality pass, on the same state
                k = max(1, r["iters"])
                M.smooth(x, y, scheme=scheme, max_iters=2, check_quality=False)
                with Timer(torch) as t:
                    M.smooth(x, y, scheme=scheme, max_iters=k, check_quality=False)
                runs[name]["vertex_updates_per_s_sweeps_only"] = info["n_free"] * k / t.wall
                M.quality(x, y)
                with Timer(torch) as t:
                    for _ in range(5):
                        M.quality(x, y)
                runs[name]["quality_pass_us_incl_host_sync"] = t.wall * 1e6 / 5
            log(kind, name, runs[name])
        del x, y, x0, y0
    h = runs["rdr_jacobi"]
    return result_line(
        h["vertex_updates_per_s_incl_quality"], 1, 1, h["seconds_to_criterion"] * 1e3, "f32",
        {"workload": "graded ocean-like mesh ~64M vertices with holes and two refinement bands, "
                     "smoothed to dQ < 5e-6, float32 coordinates, float64 quality",
         "n": info["n"], "n_free": info["n_free"]},
        None, None, runs=runs, host_seconds=host)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ocean", choices=["ocean", "graded16m", "batch512", "graded64m"])
    ap.add_argument("--orderings", default=",".join(ORDER_NAMES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the per-ordering timings")
    ap.add_argument("--no-large", action="store_true",
                    help="leave the graded 16M-vertex mesh and the 512-mesh batch out of the default run")
    ap.add_argument("--large-steps", type=int, default=5, help="timed steps of each large configuration")
    ap.add_argument("--calibration-copy-mb", type=int, default=0,
                    help="first copy this many MiB device-to-device (a known-size kernel for counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1606_00803_amd import lms
    if not os.path.exists(lms.LIB_PATH):
        from paper_1606_00803_amd import build
        build.build()
    lms.load()
    assert torch.cuda.is_available(), "no GPU visible"
    fn = dict(ocean=bench_ocean, graded16m=bench_graded16m, batch512=bench_batch512,
              graded64m=bench_graded64m)[args.workload]
    out = fn(torch, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

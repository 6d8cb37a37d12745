"""Shared helpers of the GPU tests (not collected by pytest)."""
from __future__ import annotations

import os

import numpy as np

import meshgen
from oracle import mesh as omesh
from paper_1606_00803_amd import lms


def ensure_lib():
    if not os.path.exists(lms.LIB_PATH):
        from paper_1606_00803_amd import build
        build.build()
    return lms.load()


def extent(xy) -> float:
    xy = np.asarray(xy)
    return float(np.ptp(xy, axis=0).max())


def to_dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def run_library(m: meshgen.Mesh, kind: str, K: int, dtype=None, scheme: str = "jacobi",
                seed: int = 1002, M: lms.Mesh | None = None, **smooth_kw):
    """Build, reorder, permute on the device, smooth K sweeps, permute back.

    Returns (x, y, result, mesh handle) with x, y as float64 NumPy arrays in
    INPUT labels.
    """
    import torch
    dtype = dtype or torch.float64
    if M is None:
        M = lms.Mesh.build_csr(m.n, m.tri)
    M.reorder(kind, seed=seed, x0=m.x, y0=m.y)
    x0 = to_dev(m.x, dtype)
    y0 = to_dev(m.y, dtype)
    x = torch.empty_like(x0)
    y = torch.empty_like(y0)
    M.permute(x0, y0, x, y)
    kw = dict(max_iters=K, check_quality=False)
    kw.update(smooth_kw)
    r = M.smooth(x, y, scheme=scheme, **kw)
    bx = torch.empty_like(x)
    by = torch.empty_like(y)
    M.permute(x, y, bx, by, inverse=True)
    torch.cuda.synchronize()
    return (bx.double().cpu().numpy(), by.double().cpu().numpy(), r, M)


def oracle_topology(m: meshgen.Mesh):
    return omesh.topology(m.n, m.tri)

"""Python binding of the smoothing library's C ABI (include/lms.h).

Argument marshalling only: every step runs in ``liblms.so`` (host C++ for
the adjacency and orderings, HIP kernels for the sweeps and the quality).
Device arrays are PyTorch tensors on a ROCm device (float64 or float32,
contiguous, length n); work is enqueued on PyTorch's current stream.  There
is no fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "liblms.so")
HEADER = os.path.join(ROOT, "include", "lms.h")

ORI, BFS, RDR, RANDOM = 0, 1, 2, 3
FP64, FP32 = 0, 1
JACOBI, MULTICOLOR = 0, 1
STOP_MAX_ITERS, STOP_TOL, STOP_GOAL = 0, 1, 2
ORDERINGS = {"ori": ORI, "bfs": BFS, "rdr": RDR, "random": RANDOM}
SCHEMES = {"jacobi": JACOBI, "multicolor": MULTICOLOR}
STOP_NAMES = {STOP_MAX_ITERS: "max_iters", STOP_TOL: "tol", STOP_GOAL: "goal"}
TRACE_SWEEP, TRACE_ALGORITHM1 = 0, 1
TRACES = {"sweep": TRACE_SWEEP, "algorithm1": TRACE_ALGORITHM1}
STATUS_NAMES = {0: "LMS_OK", 1: "LMS_ERR_ARG", 2: "LMS_ERR_MESH", 3: "LMS_ERR_ALLOC",
                4: "LMS_ERR_HIP", 5: "LMS_ERR_STATE"}


class LmsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("check_quality", ctypes.c_int32),
                ("tol", ctypes.c_double), ("goal", ctypes.c_double), ("q_prev", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("stopped_by", ctypes.c_int32),
                ("q0", ctypes.c_double), ("q_final", ctypes.c_double), ("last_dq", ctypes.c_double)]


class ReuseStats(ctypes.Structure):
    _fields_ = [("accesses", ctypes.c_int64), ("cold", ctypes.c_int64), ("max", ctypes.c_int64),
                ("mean", ctypes.c_double), ("lines_per_wave", ctypes.c_double),
                ("max_lines_per_wave", ctypes.c_int64)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_free", ctypes.c_int32), ("n_mesh", ctypes.c_int32),
                ("n_colors", ctypes.c_int32), ("n_tri", ctypes.c_int64), ("nnz_full", ctypes.c_int64),
                ("nnz", ctypes.c_int64), ("ordering", ctypes.c_int32), ("max_degree", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i32, _i64, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64

_SIGS = {
    "lms_smooth_opts_default": (None, [ctypes.POINTER(Opts)]),
    "lms_build_csr": (ctypes.c_int, [_i32, _i64, _vp, _vp, ctypes.POINTER(_vp)]),
    "lms_build_csr_batched": (ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, ctypes.POINTER(_vp)]),
    "lms_reorder": (ctypes.c_int, [_vp, ctypes.c_int, _u64, _vp, _vp, _vp]),
    "lms_reorder_with_quality": (ctypes.c_int, [_vp, _vp, _vp]),
    "lms_permute": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _i32, _vp]),
    "lms_smooth": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(Opts), _vp, ctypes.POINTER(Result)]),
    "lms_sweep": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp]),
    "lms_quality": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp, _vp]),
    "lms_quality_batched": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "lms_quality_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, _vp, _vp]),
    "lms_sweep_config": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_char_p, _i32]),
    "lms_destroy": (ctypes.c_int, [_vp]),
    "lms_last_error": (ctypes.c_char_p, []),
    "lms_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(Info)]),
    "lms_get_csr": (ctypes.c_int, [_vp, _vp, _vp]),
    "lms_get_vertex_data": (ctypes.c_int, [_vp, _vp, _vp]),
    "lms_get_order": (ctypes.c_int, [_vp, _vp]),
    "lms_host_vertex_quality": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "lms_reorder_device": (ctypes.c_int, [_vp, _i32, _u64, _vp, _vp, _vp, _vp]),
    "lms_reuse_profile": (ctypes.c_int, [_vp, _vp, _i32, _vp, _i32, _i32, ctypes.POINTER(ReuseStats)]),
    "lms_reuse_profile_trace": (ctypes.c_int, [_vp, _i32, _vp, _i32, _vp, _i32, _i32, ctypes.POINTER(ReuseStats)]),
}


def header_functions() -> list[str]:
    """Names of the functions declared in include/lms.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lms_[a-z0-9_]+)\s*\(", text)))


def load(path: str | None = None):
    """Load liblms.so (built by paper_1606_00803_amd.build); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError(f"{p} not found: build it with `python -m paper_1606_00803_amd.build`")
    lib = ctypes.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise LmsError(status, load().lms_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_opts() -> Opts:
    o = Opts()
    load().lms_smooth_opts_default(ctypes.byref(o))
    return o


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, n: int, what: str):
    """(pointer, precision) of a device tensor of length n."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a GPU tensor")
    if t.dtype == torch.float64:
        p = FP64
    elif t.dtype == torch.float32:
        p = FP32
    else:
        raise TypeError(f"{what} must be float64 or float32")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{what} must be contiguous with {n} elements")
    return ctypes.c_void_p(t.data_ptr()), p


class Mesh:
    """A mesh handle (``lms_mesh_t``)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle

    # ---- construction -------------------------------------------------
    @classmethod
    def build_csr(cls, n: int, tri, fixed=None) -> "Mesh":
        tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        h = ctypes.c_void_p()
        _check(load().lms_build_csr(int(n), int(tri.shape[0]), _np_ptr(tri),
                                    None if fx is None else _np_ptr(fx), ctypes.byref(h)))
        return cls(h)

    @classmethod
    def build_csr_batched(cls, v_off, t_off, tri_local, fixed=None) -> "Mesh":
        v_off = np.ascontiguousarray(v_off, dtype=np.int64)
        t_off = np.ascontiguousarray(t_off, dtype=np.int64)
        tri = np.ascontiguousarray(tri_local, dtype=np.int32).reshape(-1, 3)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        h = ctypes.c_void_p()
        _check(load().lms_build_csr_batched(int(v_off.size - 1), _np_ptr(v_off), _np_ptr(t_off),
                                            _np_ptr(tri), None if fx is None else _np_ptr(fx),
                                            ctypes.byref(h)))
        return cls(h)

    def destroy(self):
        if self._h is not None and self._h.value:
            _check(load().lms_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("mesh handle destroyed")
        return self._h

    # ---- host-side --------------------------------------------------------
    def info(self) -> dict:
        i = Info()
        _check(load().lms_get_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}

    @property
    def n(self) -> int:
        return self.info()["n"]

    def reorder(self, kind, seed: int = 0, x0=None, y0=None) -> np.ndarray:
        kind = ORDERINGS[kind] if isinstance(kind, str) else int(kind)
        n = self.n
        out = np.empty(n, dtype=np.int32)
        xp = yp = None
        if x0 is not None:
            x0 = np.ascontiguousarray(x0, dtype=np.float64)
            y0 = np.ascontiguousarray(y0, dtype=np.float64)
            if x0.size != n or y0.size != n:
                raise ValueError("x0, y0 must have n elements")
            xp, yp = _np_ptr(x0), _np_ptr(y0)
        _check(load().lms_reorder(self.handle, kind, ctypes.c_uint64(seed & (2**64 - 1)), xp, yp,
                                  _np_ptr(out)))
        return out

    def reorder_device(self, kind, seed: int = 0, x0=None, y0=None) -> np.ndarray:
        """reorder() with the breadth-first search and the relabelling on the
        GPU (same result, bit for bit)."""
        kind = ORDERINGS[kind] if isinstance(kind, str) else int(kind)
        n = self.n
        out = np.empty(n, dtype=np.int32)
        xp = yp = None
        if x0 is not None:
            x0 = np.ascontiguousarray(x0, dtype=np.float64)
            y0 = np.ascontiguousarray(y0, dtype=np.float64)
            if x0.size != n or y0.size != n:
                raise ValueError("x0, y0 must have n elements")
            xp, yp = _np_ptr(x0), _np_ptr(y0)
        _check(load().lms_reorder_device(self.handle, kind, ctypes.c_uint64(seed & (2**64 - 1)), xp, yp,
                                         _np_ptr(out), _stream()))
        return out

    def reorder_with_quality(self, q) -> np.ndarray:
        q = np.ascontiguousarray(q, dtype=np.float64)
        if q.size != self.n:
            raise ValueError("q must have n elements")
        out = np.empty(self.n, dtype=np.int32)
        _check(load().lms_reorder_with_quality(self.handle, _np_ptr(q), _np_ptr(out)))
        return out

    def csr(self) -> tuple[np.ndarray, np.ndarray]:
        i = self.info()
        rp = np.empty(i["n"] + 1, dtype=np.int32)
        col = np.empty(max(i["nnz"], 1), dtype=np.int32)
        _check(load().lms_get_csr(self.handle, _np_ptr(rp), _np_ptr(col)))
        return rp, col[:i["nnz"]]

    def vertex_data(self) -> tuple[np.ndarray, np.ndarray]:
        n = self.n
        fx = np.empty(n, dtype=np.uint8)
        col = np.empty(n, dtype=np.int32)
        _check(load().lms_get_vertex_data(self.handle, _np_ptr(fx), _np_ptr(col)))
        return fx, col

    def order(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        _check(load().lms_get_order(self.handle, _np_ptr(out)))
        return out

    def host_vertex_quality(self, x, y) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        q = np.empty(self.n, dtype=np.float64)
        _check(load().lms_host_vertex_quality(self.handle, _np_ptr(x), _np_ptr(y), _np_ptr(q)))
        return q

    def reuse_profile(self, fractions=(0.5, 0.75, 0.9, 1.0), line_bytes: int = 128,
                      record_bytes: int = 16, trace: str = "sweep") -> dict:
        """Locality of the current ordering (reuse-distance quantiles of an
        access trace: "sweep", one sweep of Eq. 1, or "algorithm1", the sweep
        with Algorithm 1's quality upkeep; cache-line spans per wavefront);
        host only."""
        f = np.ascontiguousarray(fractions, dtype=np.float64)
        q = np.zeros(f.size, dtype=np.int64)
        st = ReuseStats()
        if trace == "sweep":
            _check(load().lms_reuse_profile(self.handle, _np_ptr(f), int(f.size), _np_ptr(q), int(line_bytes),
                                            int(record_bytes), ctypes.byref(st)))
        else:
            kind = TRACES[trace] if isinstance(trace, str) else int(trace)
            _check(load().lms_reuse_profile_trace(self.handle, kind, _np_ptr(f), int(f.size), _np_ptr(q),
                                                  int(line_bytes), int(record_bytes), ctypes.byref(st)))
        return dict(accesses=st.accesses, cold=st.cold, quantiles=[int(v) for v in q], mean=st.mean,
                    max=st.max, lines_per_wave=st.lines_per_wave, max_lines_per_wave=st.max_lines_per_wave)

    # ---- device-side ------------------------------------------------------
    def permute(self, sx, sy, dx, dy, inverse: bool = False):
        n = self.n
        a, p = _dev(sx, n, "sx")
        b, _ = _dev(sy, n, "sy")
        c, p2 = _dev(dx, n, "dx")
        d, _ = _dev(dy, n, "dy")
        if p != p2 or sy.dtype != sx.dtype or dy.dtype != dx.dtype:
            raise TypeError("all four arrays must have the same dtype")
        _check(load().lms_permute(self.handle, a, b, c, d, p, 1 if inverse else 0, _stream()))

    def sweep(self, sx, sy, dx, dy):
        n = self.n
        a, p = _dev(sx, n, "sx")
        b, _ = _dev(sy, n, "sy")
        c, p2 = _dev(dx, n, "dx")
        d, _ = _dev(dy, n, "dy")
        if p != p2 or sy.dtype != sx.dtype or dy.dtype != dx.dtype:
            raise TypeError("all four arrays must have the same dtype")
        _check(load().lms_sweep(self.handle, a, b, c, d, p, _stream()))

    def smooth(self, x, y, tx=None, ty=None, scheme="jacobi", max_iters: int = 1000,
               check_quality: bool = True, tol: float = 5e-6, goal: float = math.inf,
               q_prev: float | None = None) -> dict:
        n = self.n
        a, p = _dev(x, n, "x")
        b, _ = _dev(y, n, "y")
        if y.dtype != x.dtype:
            raise TypeError("x and y must have the same dtype")
        c = d = None
        if tx is not None or ty is not None:
            c, _ = _dev(tx, n, "tx")
            d, _ = _dev(ty, n, "ty")
            if tx.dtype != x.dtype or ty.dtype != x.dtype:
                raise TypeError("tx, ty must match x's dtype")
        o = Opts(int(max_iters), 1 if check_quality else 0, float(tol), float(goal),
                 math.nan if q_prev is None else float(q_prev))
        r = Result()
        sch = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        _check(load().lms_smooth(self.handle, a, b, c, d, p, sch, ctypes.byref(o), _stream(),
                                 ctypes.byref(r)))
        return dict(iters=r.iters, stopped_by=STOP_NAMES.get(r.stopped_by, r.stopped_by),
                    q0=r.q0, q_final=r.q_final, last_dq=r.last_dq)

    def quality(self, x, y, q_vertex=None) -> float:
        n = self.n
        a, p = _dev(x, n, "x")
        b, _ = _dev(y, n, "y")
        qv = None
        if q_vertex is not None:
            import torch
            if q_vertex.dtype != torch.float64:
                raise TypeError("q_vertex must be float64")
            qv, _ = _dev(q_vertex, n, "q_vertex")
        out = ctypes.c_double()
        _check(load().lms_quality(self.handle, a, b, p, ctypes.byref(out), qv, _stream()))
        return out.value

    def quality_noalloc(self, x, y, q_out) -> None:
        """lms_quality_noalloc: Q into the float64 device tensor q_out[0],
        asynchronously on the current stream."""
        n = self.n
        a, p = _dev(x, n, "x")
        b, _ = _dev(y, n, "y")
        import torch
        if q_out.dtype != torch.float64 or not q_out.is_cuda or q_out.numel() < 1:
            raise TypeError("q_out must be a float64 device tensor of at least one element")
        _check(load().lms_quality_noalloc(self.handle, a, b, p, q_out.data_ptr(), _stream()))

    def sweep_config(self, precision="f64") -> str:
        buf = ctypes.create_string_buffer(8192)
        p = FP64 if precision in ("f64", FP64) else FP32
        _check(load().lms_sweep_config(self.handle, p, buf, 8192))
        return buf.value.decode()

    def quality_batched(self, x, y) -> np.ndarray:
        i = self.info()
        a, p = _dev(x, i["n"], "x")
        b, _ = _dev(y, i["n"], "y")
        out = np.empty(i["n_mesh"], dtype=np.float64)
        _check(load().lms_quality_batched(self.handle, a, b, p, _np_ptr(out), _stream()))
        return out

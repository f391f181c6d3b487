"""Python binding of the gfx950 threshold RHG library (include/rhg.h).

Argument marshalling only: every step of generation runs in librhg.so's HIP
kernels.  Functions carry the C names; a non-OK status raises RhgError.
Device buffers may be PyTorch tensors (their data_ptr is passed) and the
context may run on a PyTorch stream (pass torch.cuda.current_stream()).
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librhg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rhg.h")

RHG_OK, RHG_EINVAL, RHG_ENOMEM, RHG_EDEVICE, RHG_ERANGE, RHG_ETRUNC, RHG_EBUSY = 0, -1, -2, -3, -4, -5, -6
RHG_FP64, RHG_FP32_RECHECK = 0, 1
RHG_OPT_FP32_EXHAUSTIVE = 1
RHG_OPT_SHARD_COUNT = 2
RHG_OPT_SHARD_INDEX = 3
RHG_OPT_LITERAL_ABLATION = 4


class RhgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, status_str(status), status))


class rhg_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("alpha", ctypes.c_double), ("kbar", ctypes.c_double),
                ("R", ctypes.c_double), ("seed", ctypes.c_uint64), ("precision", ctypes.c_int),
                ("num_bands", ctypes.c_uint32), ("band_ratio", ctypes.c_double)]


class rhg_stats(ctypes.Structure):
    _fields_ = [("edges", ctypes.c_uint64), ("candidates", ctypes.c_uint64), ("rechecks", ctypes.c_uint64),
                ("windows", ctypes.c_uint64), ("disagreements", ctypes.c_uint64),
                ("ms", ctypes.c_double * 8), ("bytes_moved", ctypes.c_uint64),
                ("count_kernel_ms", ctypes.c_double), ("literal_undecided", ctypes.c_uint64),
                ("literal_wrong", ctypes.c_uint64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "ms"}
        d["ms"] = list(self.ms)
        return d


class rhg_server_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("batched", ctypes.c_uint64), ("groups", ctypes.c_uint64),
                ("fallbacks", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def params(n: int, alpha: float = 1.0, kbar: float = 10.0, R: float = 0.0, seed: int = 1,
           precision: int = RHG_FP64, num_bands: int = 0, band_ratio: float = 0.0) -> rhg_params:
    return rhg_params(int(n), float(alpha), float(kbar), float(R), int(seed), int(precision), int(num_bands),
                      float(band_ratio))


_lib = None
_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


def load(path: Optional[str] = None):
    """Load librhg.so; raises if it has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    try:
        # Share the process's HIP runtime with PyTorch: its wheel carries its own
        # libamdhip64.so.7; loading it first makes librhg.so bind to the same
        # runtime, so PyTorch streams and device pointers are valid here.
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(p):
        raise RuntimeError("librhg.so not built (run __graft_entry__.build() or paper_1606_09481_amd/build.py)")
    L = ctypes.CDLL(p)
    vp, i32, u64, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "rhg_ctx_create": (i32, [i32, vp, P(vp)]),
        "rhg_ctx_set_allocator": (i32, [vp, _ALLOC, _FREE, vp]),
        "rhg_ctx_set_option": (i32, [vp, i32, ctypes.c_int64]),
        "rhg_ctx_destroy": (None, [vp]),
        "rhg_target_radius": (i32, [u64, d, d, P(d)]),
        "rhg_band_boundaries": (i32, [d, ctypes.c_uint32, d, vp]),
        "rhg_generate": (i32, [vp, P(rhg_params), P(vp)]),
        "rhg_generate_from_coords": (i32, [vp, u64, vp, vp, d, i32, i32, P(vp)]),
        "rhg_generate_from_table": (i32, [vp, u64, vp, vp, vp, d, i32, i32, P(vp)]),
        "rhg_move": (i32, [vp, u64, d, d, vp, vp, vp, vp]),
        "rhg_update_after_move": (i32, [vp, u64, vp, vp, d, i32, vp, vp, u64, P(vp)]),
        "rhg_csr_from_pairs": (i32, [vp, u64, vp, u64, vp, vp]),
        "rhg_count": (i32, [vp, P(rhg_params), P(vp), P(u64)]),
        "rhg_emit": (i32, [vp, vp, vp, u64]),
        "rhg_generate_noalloc": (i32, [vp, P(rhg_params), vp, u64, P(u64)]),
        "rhg_generate_soft": (i32, [vp, P(rhg_params), d, P(vp)]),
        "rhg_count_soft": (i32, [vp, P(rhg_params), d, P(vp), P(u64)]),
        "rhg_generate_soft_from_table": (i32, [vp, u64, vp, vp, vp, d, d, u64, i32, P(vp)]),
        "rhg_graph_num_edges": (i32, [vp, P(u64)]),
        "rhg_graph_num_points": (i32, [vp, P(u64)]),
        "rhg_graph_radius": (i32, [vp, P(d)]),
        "rhg_graph_edges_device": (i32, [vp, P(vp)]),
        "rhg_graph_copy_edges": (i32, [vp, vp, u64]),
        "rhg_graph_copy_points": (i32, [vp, vp, vp, vp, P(d)]),
        "rhg_graph_stats": (i32, [vp, P(rhg_stats)]),
        "rhg_graph_free": (None, [vp]),
        "rhg_server_create": (i32, [i32, u64, P(vp)]),
        "rhg_server_submit": (i32, [vp, P(rhg_params), P(u64)]),
        "rhg_server_wait": (i32, [vp, u64, i32, P(vp), P(d)]),
        "rhg_server_counters": (i32, [vp, P(rhg_server_stats)]),
        "rhg_server_estimate_bytes": (i32, [P(rhg_params), P(u64)]),
        "rhg_server_destroy": (None, [vp]),
        "rhg_status_str": (ctypes.c_char_p, [i32]),
        "rhg_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions():
    """Names of the functions include/rhg.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rhg_[a-z0-9_]+)\s*\(", txt)))


def _check(status: int, where: str):
    if status != RHG_OK:
        raise RhgError(status, where)


def status_str(status: int) -> str:
    return load().rhg_status_str(int(status)).decode()


def _ptr(x) -> ctypes.c_void_p:
    """Address of a numpy array, a torch tensor, an int address or None."""
    if x is None:
        return ctypes.c_void_p(0)
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(ctypes.c_void_p)
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    raise TypeError("unsupported buffer %r" % type(x))


# ---- context -----------------------------------------------------------------
def rhg_ctx_create(device: int = 0, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    s = None
    if stream is not None:
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _check(load().rhg_ctx_create(int(device), ctypes.c_void_p(s), ctypes.byref(h)), "rhg_ctx_create")
    return h


def rhg_ctx_set_option(ctx, option: int, value: int):
    _check(load().rhg_ctx_set_option(ctx, int(option), int(value)), "rhg_ctx_set_option")


def rhg_ctx_set_allocator(ctx, alloc, free, user=None):
    """alloc(nbytes) -> device address, free(address); Python callables (kept alive on ctx)."""
    ca = _ALLOC(lambda nb, u: alloc(int(nb)) or 0)
    cf = _FREE(lambda p, u: free(int(p)))
    _keep.setdefault(ctx.value, []).extend([ca, cf])
    _check(load().rhg_ctx_set_allocator(ctx, ca, cf, None), "rhg_ctx_set_allocator")


_keep = {}


def rhg_ctx_destroy(ctx):
    load().rhg_ctx_destroy(ctx)
    _keep.pop(ctx.value, None)


# ---- parameters ----------------------------------------------------------------
def rhg_target_radius(n: int, alpha: float, kbar: float) -> float:
    R = ctypes.c_double()
    _check(load().rhg_target_radius(int(n), float(alpha), float(kbar), ctypes.byref(R)), "rhg_target_radius")
    return R.value


def rhg_band_boundaries(R: float, num_bands: int, band_ratio: float = 0.9) -> np.ndarray:
    c = np.empty(int(num_bands) + 1, dtype=np.float64)
    _check(load().rhg_band_boundaries(float(R), int(num_bands), float(band_ratio), _ptr(c)), "rhg_band_boundaries")
    return c


# ---- generation ------------------------------------------------------------------
def rhg_generate(ctx, p: rhg_params) -> ctypes.c_void_p:
    g = ctypes.c_void_p()
    _check(load().rhg_generate(ctx, ctypes.byref(p), ctypes.byref(g)), "rhg_generate")
    return g


def rhg_generate_from_coords(ctx, theta, r, R: float, precision: int = RHG_FP64) -> ctypes.c_void_p:
    """theta, r: float64 numpy arrays (host) or torch float64 tensors on the GPU."""
    on_dev = int(not isinstance(theta, np.ndarray))
    if isinstance(theta, np.ndarray):
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        r = np.ascontiguousarray(r, dtype=np.float64)
    n = len(theta)
    g = ctypes.c_void_p()
    _check(load().rhg_generate_from_coords(ctx, n, _ptr(theta), _ptr(r), float(R), int(precision), on_dev,
                                           ctypes.byref(g)), "rhg_generate_from_coords")
    return g


def rhg_generate_from_table(ctx, theta, r, table5xn, R: float, precision: int = RHG_FP64) -> ctypes.c_void_p:
    on_dev = int(not isinstance(theta, np.ndarray))
    if isinstance(theta, np.ndarray):
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        r = np.ascontiguousarray(r, dtype=np.float64)
        table5xn = np.ascontiguousarray(table5xn, dtype=np.float64)
    n = len(theta)
    g = ctypes.c_void_p()
    _check(load().rhg_generate_from_table(ctx, n, _ptr(theta), _ptr(r), _ptr(table5xn), float(R), int(precision),
                                          on_dev, ctypes.byref(g)), "rhg_generate_from_table")
    return g


def rhg_move(ctx, theta, r, tau_phi, tau_r, alpha: float, R: float):
    """One movement step in place.  theta, r, tau_phi, tau_r: float64 torch
    tensors on the GPU of equal length (or device addresses with n given by
    theta's length); theta, r and tau_r are updated on the context stream."""
    n = int(theta.numel()) if hasattr(theta, "numel") else len(theta)
    for x in (r, tau_phi, tau_r):
        if hasattr(x, "numel") and int(x.numel()) != n:
            raise ValueError("rhg_move: arrays of different lengths")
    _check(load().rhg_move(ctx, n, float(alpha), float(R), _ptr(theta), _ptr(r), _ptr(tau_phi), _ptr(tau_r)),
           "rhg_move")


def rhg_update_after_move(ctx, theta, r, R: float, moved, old_pairs, m_old: int,
                          precision: int = RHG_FP64) -> ctypes.c_void_p:
    """Graph after a move from the graph before it.  theta, r: float64 torch
    tensors on the GPU (coordinates after the move); moved: uint8 tensor on
    the GPU, nonzero for moved points (original order); old_pairs: int32
    device tensor (or device address) holding the m_old pairs of the graph
    before the move."""
    n = int(theta.numel())
    for x in (r, moved):
        if int(x.numel()) != n:
            raise ValueError("rhg_update_after_move: arrays of different lengths")
    if not isinstance(old_pairs, int) and int(old_pairs.numel()) < 2 * int(m_old):
        raise ValueError("rhg_update_after_move: old_pairs holds fewer than m_old pairs")
    g = ctypes.c_void_p()
    _check(load().rhg_update_after_move(ctx, n, _ptr(theta), _ptr(r), float(R), int(precision), _ptr(moved),
                                        _ptr(old_pairs), int(m_old), ctypes.byref(g)), "rhg_update_after_move")
    return g


def rhg_csr_from_pairs(ctx, n: int, pairs, m: int, row_ptr, col):
    """Symmetric CSR of m device pairs: row_ptr (uint64/int64 tensor, n + 1)
    and col (int32 tensor, 2m) on the GPU; pairs a device tensor or address."""
    if int(row_ptr.numel()) < int(n) + 1 or (int(m) and int(col.numel()) < 2 * int(m)):
        raise ValueError("rhg_csr_from_pairs: output arrays too small")
    _check(load().rhg_csr_from_pairs(ctx, int(n), _ptr(pairs), int(m), _ptr(row_ptr), _ptr(col)),
           "rhg_csr_from_pairs")


def rhg_count(ctx, p: rhg_params) -> Tuple[ctypes.c_void_p, int]:
    g = ctypes.c_void_p()
    m = ctypes.c_uint64()
    _check(load().rhg_count(ctx, ctypes.byref(p), ctypes.byref(g), ctypes.byref(m)), "rhg_count")
    return g, m.value


def rhg_emit(ctx, plan, dev_pairs, capacity_pairs: int):
    """dev_pairs: a torch int32 tensor on the GPU (>= 2*m elements) or a device address."""
    _check(load().rhg_emit(ctx, plan, _ptr(dev_pairs), int(capacity_pairs)), "rhg_emit")


def rhg_generate_soft(ctx, p: rhg_params, T: float) -> ctypes.c_void_p:
    """General model at temperature T (Sec. II, Eq. 2); p.seed also seeds the pairs' uniforms."""
    g = ctypes.c_void_p()
    _check(load().rhg_generate_soft(ctx, ctypes.byref(p), float(T), ctypes.byref(g)), "rhg_generate_soft")
    return g


def rhg_count_soft(ctx, p: rhg_params, T: float) -> Tuple[ctypes.c_void_p, int]:
    g = ctypes.c_void_p()
    m = ctypes.c_uint64()
    _check(load().rhg_count_soft(ctx, ctypes.byref(p), float(T), ctypes.byref(g), ctypes.byref(m)),
           "rhg_count_soft")
    return g, m.value


def rhg_generate_soft_from_table(ctx, theta, r, table5xn, R: float, T: float, seed: int) -> ctypes.c_void_p:
    on_dev = int(not isinstance(theta, np.ndarray))
    if isinstance(theta, np.ndarray):
        theta = np.ascontiguousarray(theta, dtype=np.float64)
        r = np.ascontiguousarray(r, dtype=np.float64)
        table5xn = np.ascontiguousarray(table5xn, dtype=np.float64)
    n = len(theta)
    g = ctypes.c_void_p()
    _check(load().rhg_generate_soft_from_table(ctx, n, _ptr(theta), _ptr(r), _ptr(table5xn), float(R), float(T),
                                               int(seed) & (2**64 - 1), on_dev, ctypes.byref(g)),
           "rhg_generate_soft_from_table")
    return g


def rhg_generate_noalloc(ctx, p: rhg_params, dev_pairs, capacity_pairs: int) -> int:
    """One seeded request (n <= 8192) into dev_pairs (torch int32 tensor on the
    GPU, or a device address) without any device allocation; returns m.
    Raises RhgError(RHG_ETRUNC) when m > capacity_pairs (its .m holds m)."""
    m = ctypes.c_uint64()
    s = load().rhg_generate_noalloc(ctx, ctypes.byref(p), _ptr(dev_pairs), int(capacity_pairs), ctypes.byref(m))
    if s != RHG_OK:
        e = RhgError(s, "rhg_generate_noalloc")
        e.m = m.value
        raise e
    return m.value


# ---- graph handle ------------------------------------------------------------------
def rhg_graph_num_edges(g) -> int:
    m = ctypes.c_uint64()
    _check(load().rhg_graph_num_edges(g, ctypes.byref(m)), "rhg_graph_num_edges")
    return m.value


def rhg_graph_num_points(g) -> int:
    n = ctypes.c_uint64()
    _check(load().rhg_graph_num_points(g, ctypes.byref(n)), "rhg_graph_num_points")
    return n.value


def rhg_graph_radius(g) -> float:
    R = ctypes.c_double()
    _check(load().rhg_graph_radius(g, ctypes.byref(R)), "rhg_graph_radius")
    return R.value


def rhg_graph_edges_device(g) -> int:
    p = ctypes.c_void_p()
    _check(load().rhg_graph_edges_device(g, ctypes.byref(p)), "rhg_graph_edges_device")
    return p.value or 0


def rhg_graph_copy_edges(g, out: Optional[np.ndarray] = None) -> np.ndarray:
    m = rhg_graph_num_edges(g)
    if out is None:
        out = np.empty((m, 2), dtype=np.int32)
    cap = out.size // 2
    _check(load().rhg_graph_copy_edges(g, _ptr(out), cap), "rhg_graph_copy_edges")
    return out[:m]


def rhg_graph_copy_points(g):
    """(theta, r, table(5, n), K) as the distance test used them."""
    n = rhg_graph_num_points(g)
    th = np.empty(n, dtype=np.float64)
    r = np.empty(n, dtype=np.float64)
    t = np.empty((5, n), dtype=np.float64)
    K = ctypes.c_double()
    _check(load().rhg_graph_copy_points(g, _ptr(th), _ptr(r), _ptr(t), ctypes.byref(K)), "rhg_graph_copy_points")
    return th, r, t, K.value


def rhg_graph_stats(g) -> dict:
    s = rhg_stats()
    _check(load().rhg_graph_stats(g, ctypes.byref(s)), "rhg_graph_stats")
    return s.as_dict()


def rhg_graph_free(g):
    load().rhg_graph_free(g)


# ---- serving -------------------------------------------------------------------------
def rhg_server_create(device: int = 0, mem_budget_bytes: int = 8 << 30) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().rhg_server_create(int(device), int(mem_budget_bytes), ctypes.byref(h)), "rhg_server_create")
    return h


def rhg_server_submit(s, p: rhg_params) -> int:
    t = ctypes.c_uint64()
    _check(load().rhg_server_submit(s, ctypes.byref(p), ctypes.byref(t)), "rhg_server_submit")
    return t.value


def rhg_server_wait(s, ticket: int, timeout_ms: int = -1):
    """(graph, latency_ms); raises RhgError(RHG_EBUSY) if not done within timeout_ms >= 0."""
    g = ctypes.c_void_p()
    lat = ctypes.c_double()
    _check(load().rhg_server_wait(s, int(ticket), int(timeout_ms), ctypes.byref(g), ctypes.byref(lat)),
           "rhg_server_wait")
    return g, lat.value


def rhg_server_estimate_bytes(p: rhg_params) -> int:
    b = ctypes.c_uint64()
    _check(load().rhg_server_estimate_bytes(ctypes.byref(p), ctypes.byref(b)), "rhg_server_estimate_bytes")
    return b.value


def rhg_server_counters(s) -> dict:
    out = rhg_server_stats()
    _check(load().rhg_server_counters(s, ctypes.byref(out)), "rhg_server_counters")
    return out.as_dict()


def rhg_server_destroy(s):
    load().rhg_server_destroy(s)


def rhg_status_str(status: int) -> str:
    return status_str(status)


def rhg_version() -> str:
    return load().rhg_version().decode()

"""FP64 CPU oracle for threshold random hyperbolic graphs (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product (the HIP library and its
binding under ``paper_1606_09481_amd/``) never does, and the two share no
code: this wrapper loads ``liboracle.so`` built from ``rhg_oracle.c`` with
plain gcc.

Every function names the passage of von Looz et al. (HPEC 2016) it follows;
see ``rhg_oracle.c`` for the arithmetic.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rhg_oracle.c")
# RHG_ORACLE_LIB: another build of rhg_oracle.c to load instead (the mutation
# test loads builds with planted mistakes and requires a pin to fail)
_BUILT = os.path.join(_HERE, "liboracle.so")
_LIB = os.environ.get("RHG_ORACLE_LIB") or _BUILT

TWO_PI = 2.0 * np.pi  # fl(2*pi), the sampler's angle period


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_BUILT):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-pthread", "-o", _BUILT + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_BUILT + ".tmp", _BUILT)
    return _BUILT


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d, i64, u64, i32, vp = ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        pd = ctypes.POINTER(ctypes.c_double)
        L.orc_kbar_approx.restype = d
        L.orc_kbar_approx.argtypes = [d, d, d]
        L.orc_target_radius.restype = i32
        L.orc_target_radius.argtypes = [d, d, d, pd]
        L.orc_default_bands.restype = i32
        L.orc_default_bands.argtypes = [u64]
        L.orc_boundaries.restype = None
        L.orc_boundaries.argtypes = [d, i32, d, vp]
        L.orc_band_of_radius.restype = i32
        L.orc_band_of_radius.argtypes = [d, vp, i32]
        L.orc_splitmix64.restype = u64
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_sample.restype = i32
        L.orc_sample.argtypes = [u64, d, d, u64, vp, vp]
        L.orc_sample_range.restype = i32
        L.orc_sample_range.argtypes = [u64, u64, d, d, u64, vp, vp]
        L.orc_table.restype = None
        L.orc_table.argtypes = [u64, vp, vp, vp, vp, vp, vp, vp]
        L.orc_coshdist.restype = d
        L.orc_coshdist.argtypes = [vp, vp, vp, vp, vp, i64, i64]
        L.orc_is_edge.restype = i32
        L.orc_is_edge.argtypes = [vp, vp, vp, vp, vp, i64, i64, d]
        L.orc_brute.restype = i64
        L.orc_brute.argtypes = [i64, vp, vp, vp, vp, vp, d, ctypes.POINTER(ctypes.c_void_p)]
        L.orc_brute_rows.restype = i64
        L.orc_brute_rows.argtypes = [i64, vp, vp, vp, vp, vp, d, vp, i64, i32, ctypes.POINTER(ctypes.c_void_p)]
        L.orc_window.restype = i32
        L.orc_window.argtypes = [d, d, d, pd]
        L.orc_band_sweep.restype = i64
        L.orc_band_sweep.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, d, d, i32, d, i32, i64, i64,
                                     ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_uint64)]
        L.orc_sort_edges.restype = None
        L.orc_sort_edges.argtypes = [vp, i64]
        L.orc_move.restype = None
        L.orc_move.argtypes = [u64, d, d, vp, vp, vp, vp]
        L.orc_free.restype = None
        L.orc_free.argtypes = [vp]
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.orc_pair_uniform.restype = d
        L.orc_pair_uniform.argtypes = [u64, i64, i64]
        L.orc_fd_prob.restype = d
        L.orc_fd_prob.argtypes = [d, d, d]
        L.orc_soft_is_edge.restype = i32
        L.orc_soft_is_edge.argtypes = [vp, vp, vp, vp, vp, i64, i64, d, d, u64]
        L.orc_soft_brute.restype = i64
        L.orc_soft_brute.argtypes = [i64, vp, vp, vp, vp, vp, d, d, u64, PP, PP, ctypes.POINTER(ctypes.c_int64)]
        L.orc_soft_band_sweep.restype = i64
        L.orc_soft_band_sweep.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, d, d, u64, i32, d, i32, PP, PP,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64)]
        _lib = L
    return _lib


def default_threads() -> int:
    """Host threads for the threaded oracle routines: the machine's cores, at
    most 16 (the CPU share one GPU job may use on a shared host)."""
    return max(1, min(16, os.cpu_count() or 1))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Parameters (getTargetRadius, Sec. III-B; slab boundaries, Sec. III-A Eq. 4)
# --------------------------------------------------------------------------
def kbar_approx(n: float, alpha: float, R: float) -> float:
    """Average-degree approximation with zeta = 1 (Sec. III-B)."""
    return lib().orc_kbar_approx(float(n), float(alpha), float(R))


def target_radius(n: float, alpha: float, kbar: float) -> float:
    """getTargetRadius: R on the decreasing branch with kbar_approx(R) = kbar."""
    R = ctypes.c_double()
    if lib().orc_target_radius(float(n), float(alpha), float(kbar), ctypes.byref(R)) != 0:
        raise ValueError("average degree not reachable for these (n, alpha, kbar)")
    return R.value


def default_bands(n: int) -> int:
    """ceil(log2 n) slabs (Sec. III-A, 'log n' boundaries)."""
    return int(lib().orc_default_bands(int(n)))


def boundaries(R: float, B: int, p: float = 0.9) -> np.ndarray:
    """c_0 = 0 < c_1 < ... < c_B = R with geometric widths (Eq. 4)."""
    c = np.empty(B + 1, dtype=np.float64)
    lib().orc_boundaries(float(R), int(B), float(p), _ptr(c))
    return c


def band_of(r: float, c: np.ndarray) -> int:
    c = np.ascontiguousarray(c, dtype=np.float64)
    return int(lib().orc_band_of_radius(float(r), _ptr(c), len(c) - 1))


# --------------------------------------------------------------------------
# Sampling (Eq. 1) and the per-point table
# --------------------------------------------------------------------------
def splitmix64(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64(int(seed) & (2**64 - 1), int(k)))


_CHUNK = 1 << 20


def _chunks(n: int, threads: int):
    """Splits [0, n) into ranges for host threads (each point is independent)."""
    if threads <= 0:
        threads = default_threads()
    if n <= _CHUNK or threads == 1:
        return [(0, n)], 1
    return [(a, min(n, a + _CHUNK)) for a in range(0, n, _CHUNK)], threads


def _run(jobs, threads):
    if threads == 1:
        for j in jobs:
            j()
        return
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda j: j(), jobs))


def sample(n: int, alpha: float, R: float, seed: int, threads: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    theta = np.empty(n, dtype=np.float64)
    r = np.empty(n, dtype=np.float64)
    L = lib()
    # an empty range only checks the parameters
    if L.orc_sample_range(0, 0, float(alpha), float(R), int(seed), _ptr(theta), _ptr(r)) != 0:
        raise ValueError("outside the sampler's domain (R in (0, 354], sinh(alpha R / 2) finite)")
    ranges, threads = _chunks(n, threads)
    _run([lambda a=a, b=b: L.orc_sample_range(a, b, float(alpha), float(R), int(seed), _ptr(theta), _ptr(r))
          for a, b in ranges], threads)
    return theta, r


def table(theta: np.ndarray, r: np.ndarray, threads: int = 0) -> np.ndarray:
    """(5, n) array: exp(r), exp(-r), sinh r, sin(theta/2), cos(theta/2)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    n = len(theta)
    t = np.empty((5, n), dtype=np.float64)
    L = lib()
    ranges, threads = _chunks(n, threads)
    _run([lambda a=a, b=b: L.orc_table(b - a, _ptr(theta[a:]), _ptr(r[a:]), _ptr(t[0, a:]), _ptr(t[1, a:]),
                                       _ptr(t[2, a:]), _ptr(t[3, a:]), _ptr(t[4, a:]))
          for a, b in ranges], threads)
    return t


def coshdist(tab: np.ndarray, u: int, v: int) -> float:
    """cosh of the hyperbolic distance (Eq. 3) in the fixed FP64 evaluation order."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    return lib().orc_coshdist(_ptr(tab[0]), _ptr(tab[1]), _ptr(tab[2]), _ptr(tab[3]), _ptr(tab[4]), int(u), int(v))


def is_edge(tab: np.ndarray, u: int, v: int, K: float) -> bool:
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    return bool(lib().orc_is_edge(_ptr(tab[0]), _ptr(tab[1]), _ptr(tab[2]), _ptr(tab[3]), _ptr(tab[4]),
                                  int(u), int(v), float(K)))


EDOMAIN = -2  # R outside (0, 354] (or K = cosh R beyond cosh 354), a query index out of range


def _take(ptr: ctypes.c_void_p, m: int) -> np.ndarray:
    if m == EDOMAIN:
        raise ValueError("outside the oracle's domain (R in (0, 354], queries in 0..n-1)")
    if m < 0:
        raise MemoryError("oracle allocation failed")
    out = np.empty((m, 2), dtype=np.int32)
    if m > 0:
        ctypes.memmove(out.ctypes.data, ptr.value, m * 8)
    lib().orc_free(ptr)
    return out


def brute(tab: np.ndarray, K: float) -> np.ndarray:
    """All pairs i < j with coshdist < K; (m, 2) int32, lexicographically sorted."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    p = ctypes.c_void_p()
    m = lib().orc_brute(tab.shape[1], _ptr(tab[0]), _ptr(tab[1]), _ptr(tab[2]), _ptr(tab[3]), _ptr(tab[4]),
                        float(K), ctypes.byref(p))
    return _take(p, m)


def brute_rows(tab: np.ndarray, K: float, queries, threads: int = 0) -> np.ndarray:
    """For each listed query q, all (q, w) with w != q and coshdist < K (all-pairs definition on those rows)."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    q = np.ascontiguousarray(queries, dtype=np.int64)
    if threads <= 0:
        threads = default_threads()
    p = ctypes.c_void_p()
    m = lib().orc_brute_rows(tab.shape[1], _ptr(tab[0]), _ptr(tab[1]), _ptr(tab[2]), _ptr(tab[3]), _ptr(tab[4]),
                             float(K), _ptr(q), len(q), int(threads), ctypes.byref(p))
    return _take(p, m)


def window(rv: float, c: float, K: float) -> Optional[float]:
    """getMinMaxPhi half-width (widened); None means the whole slab."""
    d = ctypes.c_double()
    whole = lib().orc_window(float(rv), float(c), float(K), ctypes.byref(d))
    return None if whole else d.value


def band_sweep(theta: np.ndarray, r: np.ndarray, tab: np.ndarray, R: float, K: float, B: Optional[int] = None,
               p: float = 0.9, threads: int = 0, q0: int = 0, q1: Optional[int] = None,
               with_candidates: bool = False):
    """Algorithm 1 band query; (m, 2) int32 edges (lo, hi), unsorted (block order)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    n = len(theta)
    if B is None:
        B = default_bands(n)
    if q1 is None:
        q1 = n
    if threads <= 0:
        threads = default_threads()
    ptr = ctypes.c_void_p()
    cand = ctypes.c_uint64()
    m = lib().orc_band_sweep(n, _ptr(theta), _ptr(r), _ptr(tab[0]), _ptr(tab[1]), _ptr(tab[2]), _ptr(tab[3]),
                             _ptr(tab[4]), float(R), float(K), int(B), float(p), int(threads), int(q0), int(q1),
                             ctypes.byref(ptr), ctypes.byref(cand))
    e = _take(ptr, m)
    return (e, int(cand.value)) if with_candidates else e


def sort_edges(e: np.ndarray) -> np.ndarray:
    """Lexicographic (lo, hi) order, in place on a copy."""
    e = np.ascontiguousarray(e, dtype=np.int32).copy()
    lib().orc_sort_edges(_ptr(e), len(e))
    return e


def cosh_R(R: float) -> float:
    """K = cosh R, the threshold the distance test compares against (host libm)."""
    import math
    return math.cosh(R)


# --------------------------------------------------------------------------
# Dynamic model (Sec. III-C, Algorithm 2)
# --------------------------------------------------------------------------
def move(theta: np.ndarray, r: np.ndarray, tau_phi: np.ndarray, tau_r: np.ndarray, alpha: float,
         R: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """One movement step: rotation by tau_phi and Algorithm 2's radial step
    tau_r (in units of cosh(alpha r)), reflected at 0 and R.  Returns new
    (theta, r, tau_r); the inputs are not modified."""
    th = np.ascontiguousarray(theta, dtype=np.float64).copy()
    rr = np.ascontiguousarray(r, dtype=np.float64).copy()
    tp = np.ascontiguousarray(tau_phi, dtype=np.float64)
    tr = np.ascontiguousarray(tau_r, dtype=np.float64).copy()
    lib().orc_move(len(th), float(alpha), float(R), _ptr(th), _ptr(rr), _ptr(tp), _ptr(tr))
    return th, rr, tr



# --------------------------------------------------------------------------
# General model at temperature T > 0 (Sec. II, Eq. 2)
# --------------------------------------------------------------------------
def pair_uniform(seed: int, lo: int, hi: int) -> float:
    """The uniform in (0, 1] that decides pair {lo, hi} (lo < hi)."""
    return lib().orc_pair_uniform(int(seed) & (2**64 - 1), int(lo), int(hi))


def fd_prob(V: float, R: float, T: float) -> float:
    """Eq. 2: 1 / (exp((acosh V - R) / (2T)) + 1) (acosh V taken as 0 for V <= 1)."""
    return lib().orc_fd_prob(float(V), float(R), float(T))


def soft_is_edge(tab: np.ndarray, u: int, v: int, R: float, T: float, seed: int) -> bool:
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    return bool(lib().orc_soft_is_edge(_ptr(tab[0]), _ptr(tab[1]), _ptr(tab[2]), _ptr(tab[3]), _ptr(tab[4]),
                                       int(u), int(v), float(R), float(T), int(seed) & (2**64 - 1)))


def _take_soft(ptr, m, tptr, nt):
    if m == EDOMAIN:
        for q in (ptr, tptr):
            if q.value:
                lib().orc_free(q)
        raise ValueError("outside the oracle's domain (0 < T < 1, R in (0, 354])")
    e = _take(ptr, m)
    ties = _take(tptr, int(nt.value)) if m >= 0 else None
    return e, ties


def soft_brute(tab: np.ndarray, R: float, T: float, seed: int, with_ties: bool = False):
    """All pairs i < j, each an edge iff its uniform is below Eq. 2's
    probability; (m, 2) int32 sorted.  with_ties: also the near ties (pairs
    whose uniform lies within the rounding band of the probability)."""
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    p, tp, nt = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
    m = lib().orc_soft_brute(tab.shape[1], _ptr(tab[0]), _ptr(tab[1]), _ptr(tab[2]), _ptr(tab[3]), _ptr(tab[4]),
                             float(R), float(T), int(seed) & (2**64 - 1), ctypes.byref(p), ctypes.byref(tp),
                             ctypes.byref(nt))
    e, ties = _take_soft(p, m, tp, nt)
    return (e, ties) if with_ties else e


def soft_band_sweep(theta: np.ndarray, r: np.ndarray, tab: np.ndarray, R: float, T: float, seed: int,
                    B: Optional[int] = None, p: float = 0.9, threads: int = 0, with_ties: bool = False,
                    with_candidates: bool = False):
    """Band sweep of the general model (windows for R + 80 T); edges in block order."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    tab = np.ascontiguousarray(tab, dtype=np.float64)
    n = len(theta)
    if B is None:
        B = default_bands(n)
    if threads <= 0:
        threads = default_threads()
    ptr, tp, nt, cand = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64(), ctypes.c_uint64()
    m = lib().orc_soft_band_sweep(n, _ptr(theta), _ptr(r), _ptr(tab[0]), _ptr(tab[1]), _ptr(tab[2]),
                                  _ptr(tab[3]), _ptr(tab[4]), float(R), float(T), int(seed) & (2**64 - 1), int(B),
                                  float(p), int(threads), ctypes.byref(ptr), ctypes.byref(tp), ctypes.byref(nt),
                                  ctypes.byref(cand))
    e, ties = _take_soft(ptr, m, tp, nt)
    out = [e]
    if with_ties:
        out.append(ties)
    if with_candidates:
        out.append(int(cand.value))
    return out[0] if len(out) == 1 else tuple(out)

"""Edge-set comparison between the HIP path and the oracle.

The edge list is integer output decided by floating point, so the oracle
decides every pair on exactly the table bits the device's distance test read
(rhg_graph_copy_points exports them: angles, radii, exp(r), exp(-r), sinh r,
sin(theta/2), cos(theta/2) and cosh R).  The decisions are then the same
IEEE binary64 operations on both sides and the edge sets must be identical:
no pair is allowed to differ.  Separately, the device's own table is checked
against the host's libm (within 2 ulp per entry), which is a check of the
table kernel, not of the query.
"""
from __future__ import annotations

import numpy as np


def keys(e: np.ndarray) -> np.ndarray:
    e = np.asarray(e).reshape(-1, 2).astype(np.int64)
    return (e[:, 0] << 32) | e[:, 1]


def canonical(e: np.ndarray) -> np.ndarray:
    return np.sort(keys(e))


def assert_valid(e: np.ndarray, n: int):
    e = np.asarray(e).reshape(-1, 2)
    assert np.all(e[:, 0] < e[:, 1]), "lo < hi"
    assert e.size == 0 or (e.min() >= 0 and e.max() < n), "indices in range"
    k = canonical(e)
    assert np.all(k[1:] != k[:-1]), "each edge once"


def assert_same(gpu: np.ndarray, ref: np.ndarray):
    a, b = canonical(gpu), canonical(ref)
    if len(a) == len(b) and np.array_equal(a, b):
        return
    diff = np.setxor1d(a, b)
    raise AssertionError("edge sets differ: %d vs %d edges, %d pairs in one only, e.g. %s" % (
        len(a), len(b), len(diff), [(int(x >> 32), int(x & 0xffffffff)) for x in diff[:5]]))


def ulps(a, b) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.spacing(np.maximum(np.abs(a), np.abs(b)))


def assert_table_close(orc, th: np.ndarray, r: np.ndarray, t: np.ndarray, max_ulps: float = 2):
    """The device table of (th, r) is within max_ulps of the host libm's,
    entry by entry (exp(r), exp(-r), sin and cos of the half angle), and its
    sinh column is (exp(r) - exp(-r)) / 2 of its own exponentials."""
    to = orc.table(th, r)
    u = ulps(t[[0, 1, 3, 4]], to[[0, 1, 3, 4]])
    assert u.max() <= max_ulps, "table entry %d ulp from the host libm" % u.max()
    assert np.array_equal(t[2], 0.5 * (t[0] - t[1])), "sinh column is not (exp(r) - exp(-r)) / 2"


def oracle_edges(orc, g, rhg, sweep: bool = True, threads: int = 0):
    """The oracle's edge set of graph g on the exact bits the device used:
    the band sweep (sweep=True) or all pairs (sweep=False).  Also returns
    (theta, r, table, K) as exported."""
    th, r, t, K = rhg.rhg_graph_copy_points(g)
    R = rhg.rhg_graph_radius(g)
    ref = orc.band_sweep(th, r, t, R, K, threads=threads) if sweep else orc.brute(t, K)
    return ref, (th, r, t, K)


def incident(e: np.ndarray, vertices: np.ndarray) -> np.ndarray:
    """Edges of e touching any of the vertices (canonical keys)."""
    e = np.asarray(e).reshape(-1, 2)
    sel = np.isin(e[:, 0], vertices) | np.isin(e[:, 1], vertices)
    return canonical(e[sel])

"""Edge-set comparison between the HIP path and the oracle.

The edge list is integer output decided by floating point.  When both sides
read the same table bits (rhg_generate_from_table) the decisions are the same
FP64 operations and the sets must be identical.  When each side computes its
own table (device libm vs host libm, each within 2 ulp of exact), a pair whose
cosh-distance lies within the rounding of those tables of cosh R may be
decided either way; such pairs are reported and checked to be within that
bound, every other pair must agree.
"""
from __future__ import annotations

import numpy as np

U = 2.0 ** -53


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
    assert len(a) == len(b) and np.array_equal(a, b), "edge sets differ (%d vs %d)" % (len(a), len(b))


def ambiguity_bound(tab: np.ndarray, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    ep, em, sh, hs, hc = tab
    d = hs[u] * hc[v] - hc[u] * hs[v]
    V = 0.5 * (ep[u] * em[v] + em[u] * ep[v]) + 2 * (sh[u] * sh[v]) * d * d
    dd = 16 * U
    return V, 64 * U * V + 2 * sh[u] * sh[v] * (2 * np.abs(d) * dd + dd * dd)


def assert_same_up_to_rounding(gpu: np.ndarray, ref: np.ndarray, tab_ref: np.ndarray, K: float,
                               max_ambiguous: int = 16):
    """Identical sets, except pairs within the table-rounding bound of cosh R."""
    a, b = canonical(gpu), canonical(ref)
    assert np.all(a[1:] != a[:-1]), "duplicate edges in GPU output"
    if len(a) == len(b) and np.array_equal(a, b):
        return 0
    diff = np.setxor1d(a, b)
    u = (diff >> 32).astype(np.int64)
    v = (diff & 0xffffffff).astype(np.int64)
    V, bound = ambiguity_bound(tab_ref, u, v)
    bad = np.abs(V - K) > bound
    assert not bad.any(), "pairs decided differently far from the threshold: %s" % list(zip(u[bad], v[bad]))[:5]
    assert len(diff) <= max_ambiguous, "too many ambiguous pairs: %d" % len(diff)
    return len(diff)


def incident(e: np.ndarray, vertices: np.ndarray) -> np.ndarray:
    """Edges of e touching any of the vertices (canonical keys)."""
    e = np.asarray(e).reshape(-1, 2)
    sel = np.isin(e[:, 0], vertices) | np.isin(e[:, 1], vertices)
    return canonical(e[sel])

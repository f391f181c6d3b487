"""Pins for the oracle's band sweep (Algorithm 1: slabs, angle sort, getMinMaxPhi,
binary search, outward-only scan).

The band method computes exactly the edge set of the plain pairwise
definition; it only skips pairs that cannot be neighbours.  So the sweep is
pinned to brute force over all pairs on small inputs -- random, model
distributed, adversarial (points on slab boundaries, at the origin and the
rim, angles at 0 and 2pi, duplicates, tight clusters) and pairs constructed
to sit within a few ulps of the threshold -- and to invariants: the result
does not depend on the number of slabs or their ratio, B = 1 is brute force,
and relabelling the points relabels the edges.  The getMinMaxPhi window is
also checked directly: every true neighbour lies inside it.
"""
import math

import mpmath
import numpy as np
import pytest

import inputs

mpmath.mp.dps = 50


def _edges_equal(a, b):
    return a.shape == b.shape and np.array_equal(a, b)


def _check(orc, th, r, R, B=None, p=0.9):
    t = orc.table(th, r)
    K = math.cosh(R)
    eb = orc.brute(t, K)
    es = orc.sort_edges(orc.band_sweep(th, r, t, R, K, B=B, p=p, threads=4))
    assert _edges_equal(eb, es), (len(eb), len(es))
    # each edge once, lo < hi
    assert np.all(es[:, 0] < es[:, 1])
    return eb


@pytest.mark.parametrize("n,alpha,kbar,seed", [
    (3000, 1.0, 10, 1), (3000, 0.55, 6, 2), (4000, 1.5, 20, 3), (2000, 0.75, 50, 4), (5000, 1.0, 4, 5),
])
def test_sweep_equals_brute_model(orc, n, alpha, kbar, seed):
    R = orc.target_radius(n, alpha, kbar)
    th, r = orc.sample(n, alpha, R, seed)
    e = _check(orc, th, r, R)
    assert len(e) > 0


@pytest.mark.parametrize("seed", range(4))
def test_sweep_equals_brute_adversarial(orc, seed):
    n, R = 3000, 14.0
    B = orc.default_bands(n)
    c = orc.boundaries(R, B, 0.9)
    th, r = inputs.adversarial_coords(n, R, c, seed)
    _check(orc, th, r, R)


@pytest.mark.parametrize("seed", range(3))
def test_sweep_equals_brute_uniform_radii(orc, seed):
    # radii uniform on [0, R]: many deep points with whole-slab windows
    th, r = inputs.uniform_coords(1500, 12.0, seed)
    _check(orc, th, r, 12.0)


def test_sweep_tiny_and_degenerate(orc):
    # n = 2, all points equal, all at the origin, all on the rim at one angle
    _check(orc, np.array([0.1, 0.2]), np.array([3.0, 3.0]), 5.0)
    _check(orc, np.array([0.1, 0.2]), np.array([5.0, 5.0]), 5.0)
    _check(orc, np.full(50, 1.0), np.full(50, 7.0), 7.0)
    _check(orc, np.linspace(0, 6, 60), np.zeros(60), 9.0)
    _check(orc, np.full(40, 2 * np.pi), np.full(40, 9.0), 9.0)
    e = _check(orc, np.array([0.0, 2 * np.pi]), np.array([9.0, 9.0]), 9.0)
    assert len(e) == 1                              # 0 and fl(2pi) are the same angle


def _threshold_pairs(R, n_pairs, seed, ulp_steps=(-3, -1, 0, 1, 3)):
    """Pairs of points whose exact distance is R up to a few ulps of angle."""
    g = np.random.default_rng(seed)
    th, r = [], []
    K = mpmath.cosh(mpmath.mpf(R))
    for _ in range(n_pairs):
        while True:
            ru = float(R - g.exponential(1.0))
            rv = float(R - g.exponential(1.0))
            if ru > 0.5 and rv > 0.5 and ru + rv > R + 0.1:
                break
        a, b = mpmath.mpf(ru), mpmath.mpf(rv)
        cosd = (mpmath.cosh(a) * mpmath.cosh(b) - K) / (mpmath.sinh(a) * mpmath.sinh(b))
        d = float(mpmath.acos(cosd))
        t0 = float(g.random() * (2 * np.pi - 2 * d)) if g.random() < 0.8 else float(g.random() * d)
        for k in ulp_steps:
            t1 = t0 + d
            for _ in range(abs(k)):
                t1 = np.nextafter(t1, np.inf if k > 0 else -np.inf)
            th += [t0, t1 % (2 * np.pi)]
            r += [ru, rv]
    return np.array(th), np.array(r)


@pytest.mark.parametrize("R,seed", [(14.0, 0), (20.0, 1), (26.5, 2)])
def test_sweep_near_threshold_pairs(orc, R, seed):
    th, r = _threshold_pairs(R, 60, seed)
    th2, r2 = inputs.outer_heavy_coords(1500, R, seed + 7)
    th = np.concatenate([th, th2])
    r = np.concatenate([r, r2])
    e = _check(orc, th, r, R)
    # the constructed pairs straddle the threshold: both outcomes occur
    t = orc.table(th, r)
    K = math.cosh(R)
    dec = [orc.is_edge(t, 2 * i, 2 * i + 1, K) for i in range(300)]
    assert any(dec) and not all(dec)


@pytest.mark.parametrize("B,p", [(1, 0.9), (2, 0.9), (None, 0.5), (None, 0.99), (40, 0.9), (7, 0.7)])
def test_sweep_invariant_under_slabs(orc, B, p):
    n, alpha, kbar = 3000, 0.75, 12
    R = orc.target_radius(n, alpha, kbar)
    th, r = orc.sample(n, alpha, R, 42)
    _check(orc, th, r, R, B=B, p=p)


def test_sweep_permutation_invariant(orc):
    n, R = 2500, 15.0
    th, r = orc.sample(n, 1.0, R, 9)
    t = orc.table(th, r)
    K = math.cosh(R)
    e1 = orc.sort_edges(orc.band_sweep(th, r, t, R, K))
    perm = np.random.default_rng(3).permutation(n)
    e2 = orc.band_sweep(th[perm], r[perm], t[:, perm], R, K)
    e2 = np.sort(perm[e2], axis=1).astype(np.int32)   # permuted point k is original point perm[k]
    assert np.array_equal(e1, orc.sort_edges(e2))


def test_sweep_query_subset_partitions(orc):
    n, R = 4000, 15.0
    th, r = orc.sample(n, 1.0, R, 10)
    t = orc.table(th, r)
    K = math.cosh(R)
    full = orc.sort_edges(orc.band_sweep(th, r, t, R, K))
    parts = [orc.band_sweep(th, r, t, R, K, q0=a, q1=b) for a, b in [(0, 1000), (1000, 1001), (1001, 4000)]]
    assert np.array_equal(full, orc.sort_edges(np.concatenate(parts)))


def test_window_contains_all_neighbours(orc):
    # getMinMaxPhi superset property, per (query, slab), against brute force
    n, R = 2000, 16.0
    th, r = orc.sample(n, 0.75, R, 12)
    t = orc.table(th, r)
    K = math.cosh(R)
    B = orc.default_bands(n)
    c = orc.boundaries(R, B, 0.9)
    e = orc.brute(t, K)
    band = np.array([orc.band_of(x, c) for x in r])
    checked = 0
    for u, v in e:
        for q, w in ((u, v), (v, u)):
            j = band[w]
            if j < band[q]:
                continue
            delta = orc.window(r[q], c[j], K) if j > 0 else None
            if delta is None:
                continue
            dth = abs(th[q] - th[w])
            dth = min(dth, 2 * np.pi - dth)
            assert dth <= delta, (q, w, dth, delta)
            checked += 1
    assert checked > 1000


def test_candidate_count_reasonable(orc):
    # the windows are tight: candidates per edge is a small constant (the
    # point of the method), far below the n/2 per query of brute force
    n, alpha, kbar = 20000, 1.0, 10
    R = orc.target_radius(n, alpha, kbar)
    th, r = orc.sample(n, alpha, R, 1)
    t = orc.table(th, r)
    e, cand = orc.band_sweep(th, r, t, R, math.cosh(R), with_candidates=True)
    assert cand < 3 * len(e)


def _window_edge_pairs(orc, R, n_q, seed, steps=range(-6, 7)):
    """Candidates sitting exactly on a slab's inner boundary c_j at the exact
    getMinMaxPhi angle from a query, plus or minus a few ulps: the pairs whose
    inclusion depends on the window being wide enough."""
    g = np.random.default_rng(seed)
    B = orc.default_bands(4000)
    c = orc.boundaries(R, B, 0.9)
    K = mpmath.cosh(mpmath.mpf(R))
    th, r = [], []
    for _ in range(n_q):
        j = int(g.integers(B // 2, B))
        rv = float(g.uniform(c[j], R))          # the query is in slab j or outside it
        cj = float(c[j])
        a, b = mpmath.mpf(rv), mpmath.mpf(cj)
        s = (K - mpmath.cosh(a - b)) / (2 * mpmath.sinh(a) * mpmath.sinh(b))
        if s >= 1:
            continue
        d = float(2 * mpmath.asin(mpmath.sqrt(s)))
        t0 = float(g.uniform(0.5, 2 * np.pi - 0.5 - d))
        th.append(t0)
        r.append(rv)
        for k in steps:
            t1 = t0 + d
            for _ in range(abs(k)):
                t1 = np.nextafter(t1, np.inf if k > 0 else -np.inf)
            th.append(t1)
            r.append(cj)
            t2 = t0 - d
            for _ in range(abs(k)):
                t2 = np.nextafter(t2, -np.inf if k > 0 else np.inf)
            th.append(t2)
            r.append(cj)
    return np.array(th), np.array(r), B


@pytest.mark.parametrize("R,seed", [(14.0, 3), (22.0, 4), (27.0, 5)])
def test_sweep_window_edge_pairs(orc, R, seed):
    th, r, B = _window_edge_pairs(orc, R, 150, seed)
    t = orc.table(th, r)
    K = math.cosh(R)
    eb = orc.brute(t, K)
    es = orc.sort_edges(orc.band_sweep(th, r, t, R, K, B=B))
    assert np.array_equal(eb, es), (len(eb), len(es))


def test_golden_fixture(orc):
    """The stored small graph (written by tests/golden/make_golden.py) still comes out."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "n2000_a1_k10_seed1.txt")
    with open(path) as f:
        f.readline()
        R = float.fromhex(f.readline().split()[1].split("=")[1])
        stored = np.loadtxt(f, dtype=np.int32).reshape(-1, 2)
    assert R == orc.target_radius(2000, 1.0, 10.0)
    th, r = orc.sample(2000, 1.0, R, 1)
    t = orc.table(th, r)
    assert np.array_equal(orc.sort_edges(orc.band_sweep(th, r, t, R, math.cosh(R))), stored)


def _restricted(eb, rows):
    """Row views (q, w) of the all-pairs edge list for each listed q, in list order."""
    out = []
    for q in rows:
        a = eb[eb[:, 0] == q][:, 1]
        b = eb[eb[:, 1] == q][:, 0]
        w = np.sort(np.concatenate([a, b]))
        out.append(np.stack([np.full(len(w), q, dtype=np.int32), w.astype(np.int32)], axis=1))
    return np.concatenate(out) if out else np.empty((0, 2), np.int32)


@pytest.mark.parametrize("case", ["model_hubs", "duplicates", "ragged", "adversarial"])
def test_brute_rows_equals_brute_restricted(orc, case):
    """The per-row all-pairs routine the full-size tests lean on is the plain
    definition restricted to the listed rows: every neighbour of each listed
    query, each once, in list order then increasing neighbour, with repeated
    and adjacent listed rows, hubs, exact duplicate points and ragged n."""
    rng = np.random.default_rng(17)
    if case == "model_hubs":
        n, alpha, kbar = 3001, 0.55, 8
        R = orc.target_radius(n, alpha, kbar)
        th, r = orc.sample(n, alpha, R, 7)
    elif case == "duplicates":
        n, R = 1500, 12.0
        th, r = inputs.uniform_coords(n, R, 3)
        for k in range(0, 300, 2):  # exact duplicate points, some of them listed rows
            th[k + 1], r[k + 1] = th[k], r[k]
    elif case == "ragged":
        n, alpha, kbar = 997, 1.0, 12
        R = orc.target_radius(n, alpha, kbar)
        th, r = orc.sample(n, alpha, R, 9)
    else:
        n, R = 2000, 14.0
        th, r = inputs.adversarial_coords(n, R, orc.boundaries(R, orc.default_bands(n), 0.9), 5)
    t = orc.table(th, r)
    K = math.cosh(R)
    eb = orc.brute(t, K)
    order = np.argsort(r, kind="stable")
    rows = np.concatenate([order[:6], order[-4:], rng.choice(n, 20, replace=False), [0, 1, n - 1, 0]])
    for threads in (1, 4):
        got = orc.brute_rows(t, K, rows, threads=threads)
        want = _restricted(eb, rows)
        # the routine emits each row's neighbours in increasing order within the row
        assert got.shape == want.shape and np.array_equal(got, want), (case, threads, got.shape, want.shape)
    assert len(orc.brute_rows(t, K, np.array([], dtype=np.int64))) == 0
    # hubs have many neighbours; at least one listed row is adjacent to another listed row
    assert got.shape[0] > 0

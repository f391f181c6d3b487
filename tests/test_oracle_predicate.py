"""Pins for the oracle's distance test (hyperbolic law of cosines, Sec. II Eq. 3).

The oracle evaluates cosh dist in a fixed FP64 order from the per-point table.
It is pinned here against things other than itself:

* closed forms: equal angles give distance |r_u - r_v|; opposite angles give
  r_u + r_v; a point at the origin is at distance r_other from everything;
* the literal Eq. 3 evaluated from (theta, r) in 60-digit arithmetic, within
  an error bound derived from the FP64 rounding of the table and the
  operations (relative 16u, the effect of an absolute 8u error in the
  half-angle sine, and of the absolute 3u cosh r error of sinh r taken as
  (e^r - e^-r) / 2), also for points near the centre;
* exact symmetry in (u, v), which the outward-only scan relies on.
"""
import math

import mpmath
import numpy as np
import pytest

U = 2.0 ** -53
mpmath.mp.dps = 60


def _tab(orc, th, r):
    return orc.table(np.asarray(th, dtype=np.float64), np.asarray(r, dtype=np.float64))


def exact_cosh_dist(th_u, r_u, th_v, r_v):
    a = [mpmath.mpf(float(x)) for x in (th_u, r_u, th_v, r_v)]
    return mpmath.cosh(a[1]) * mpmath.cosh(a[3]) - mpmath.sinh(a[1]) * mpmath.sinh(a[3]) * mpmath.cos(a[0] - a[2])


def error_bound(tab, u, v, V):
    sh = tab[2]
    d = tab[3][u] * tab[4][v] - tab[4][u] * tab[3][v]
    ad = 8 * U
    # sinh r is (e^r - e^-r) / 2 of the table's exponentials: an absolute
    # error of at most 3 u cosh r each (cosh r = (e^r + e^-r) / 2), which
    # enters through 2 sinh r_u sinh r_v sin^2
    ch = 0.5 * (tab[0] + tab[1])
    dsh = 2 * d * d * 3 * U * 1.01 * (ch[u] * sh[v] + sh[u] * ch[v])
    return 16 * U * V + 2 * sh[u] * sh[v] * (2 * abs(d) * ad + ad * ad) + dsh


def test_closed_forms(orc):
    g = np.random.default_rng(0)
    n = 400
    th = g.random(n) * 2 * np.pi
    r = g.random(n) * 30
    for i in range(0, n, 2):
        # same angle
        t = _tab(orc, [th[i], th[i]], [r[i], r[i + 1]])
        V = orc.coshdist(t, 0, 1)
        ref = float(mpmath.cosh(mpmath.mpf(float(r[i])) - mpmath.mpf(float(r[i + 1]))))
        assert abs(V - ref) <= 8 * U * V
        # origin
        t = _tab(orc, [th[i], th[i + 1]], [0.0, r[i + 1]])
        V = orc.coshdist(t, 0, 1)
        assert abs(V - math.cosh(r[i + 1])) <= 8 * U * V
        # opposite angles (pi apart)
        t = _tab(orc, [0.0, np.pi], [r[i], r[i + 1]])
        V = orc.coshdist(t, 0, 1)
        ref = float(mpmath.cosh(mpmath.mpf(float(r[i])) + mpmath.mpf(float(r[i + 1]))))
        assert abs(V - ref) <= 16 * U * V


@pytest.mark.parametrize("R", [15.68, 26.5, 29.3])
def test_against_high_precision(orc, R):
    g = np.random.default_rng(int(R * 10))
    n = 300
    # rim-heavy radii and small angular offsets: the regime of real windows
    r = np.clip(R - g.exponential(1.5, n), 0, R)
    th = g.random(n) * 2 * np.pi
    pairs = [(i, (i + 1) % n) for i in range(n)]
    th2 = th.copy()
    for i in range(0, n, 2):          # half of the pairs a few window widths apart
        th2[(i + 1) % n] = (th[i] + g.standard_normal() * math.exp(-R / 2) * 4) % (2 * np.pi)
    t = _tab(orc, th2, r)
    K = math.cosh(R)
    for u, v in pairs:
        V = orc.coshdist(t, u, v)
        ex = exact_cosh_dist(th2[u], r[u], th2[v], r[v])
        err = abs(mpmath.mpf(V) - ex)
        assert err <= error_bound(t, u, v, V), (u, v, V, float(ex))
        if abs(ex - K) > error_bound(t, u, v, V):
            assert orc.is_edge(t, u, v, K) == bool(ex < K)


def test_small_radii_against_high_precision(orc):
    # sinh r from e^r - e^-r cancels for small r: pairs of a point near the
    # centre and one anywhere, at every angle, stay within the bound
    g = np.random.default_rng(9)
    n = 200
    r = np.concatenate([10.0 ** g.uniform(-9, -1, n // 2), g.random(n // 2) * 20])
    th = g.random(n) * 2 * np.pi
    t = _tab(orc, th, r)
    for u in range(n // 2):
        for v in (n // 2 + u, (u + 1) % (n // 2)):
            V = orc.coshdist(t, u, v)
            ex = exact_cosh_dist(th[u], r[u], th[v], r[v])
            assert abs(mpmath.mpf(V) - ex) <= error_bound(t, u, v, V), (u, v, r[u], r[v])


def test_symmetry_bitwise(orc):
    g = np.random.default_rng(5)
    n = 5000
    th = g.random(n) * 2 * np.pi
    r = g.random(n) * 28
    t = _tab(orc, th, r)
    for i in range(0, n - 1):
        assert orc.coshdist(t, i, i + 1) == orc.coshdist(t, i + 1, i)


def test_strict_threshold_and_self(orc):
    t = _tab(orc, [0.5, 0.5], [3.0, 3.0])
    V = orc.coshdist(t, 0, 1)
    assert V == 1.0                              # coincident points: distance 0
    assert not orc.is_edge(t, 0, 0, 10.0)        # no self loops
    assert orc.is_edge(t, 0, 1, np.nextafter(1.0, 2.0))
    assert not orc.is_edge(t, 0, 1, 1.0)         # strict: V < K

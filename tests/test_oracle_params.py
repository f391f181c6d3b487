"""Pins for the oracle's parameter functions.

getTargetRadius (Sec. III-B) is pinned against the model itself: the exact
expected degree, by numerical quadrature of the edge probability over two
points drawn from Eq. 1 with uniform angles, must match the requested
average degree to within the approximation's accuracy.  The slab boundaries
(Sec. III-A, Eq. 4) are pinned by their defining invariants.
"""
import math

import numpy as np
import pytest
from scipy import integrate


def expected_degree(n, alpha, R):
    """(n-1) * P(edge) for two independent model points: the angular
    difference is uniform, so P(edge | r1, r2) = Theta(r1, r2)/pi where
    Theta is the largest angle at which the pair is still within R."""
    norm = math.cosh(alpha * R) - 1.0

    def f(r):  # Eq. 1 density, written against the boundary to keep it well scaled
        return alpha * math.sinh(alpha * r) / norm

    def theta_max(r1, r2):
        if r1 + r2 <= R:
            return math.pi
        s = (math.cosh(R) - math.cosh(r1 - r2)) / (2.0 * math.sinh(r1) * math.sinh(r2))
        return 2.0 * math.asin(math.sqrt(min(1.0, max(0.0, s))))

    def inner(r1):
        val, _ = integrate.quad(lambda r2: f(r2) * theta_max(r1, r2), 0.0, R, points=[max(0.0, R - r1)],
                                limit=400, epsabs=0, epsrel=1e-11)
        return f(r1) * val

    pts = [R - k for k in (1.0, 2.0, 4.0, 8.0) if R - k > 0]
    val, _ = integrate.quad(inner, 0.0, R, points=pts, limit=400, epsabs=0, epsrel=1e-10)
    return (n - 1) * val / math.pi


@pytest.mark.parametrize("n,alpha,kbar,tol", [
    (1e4, 1.0, 10, 1e-3),
    (1e6, 1.0, 20, 1e-3),
    (1e7, 0.75, 100, 1e-3),
    (4e6, 1.0, 64, 1e-3),
    (4e6, 1.5, 64, 1e-3),
    (4e6, 0.55, 64, 1.5e-2),   # the approximation is known to drift near alpha = 1/2
])
def test_target_radius_matches_model_degree(orc, n, alpha, kbar, tol):
    R = orc.target_radius(n, alpha, kbar)
    E = expected_degree(n, alpha, R)
    assert abs(E - kbar) / kbar < tol, (R, E)


def test_target_radius_on_decreasing_branch(orc):
    # larger average degree -> smaller disk, and the returned R solves the approximation
    Rs = [orc.target_radius(1e5, 1.0, k) for k in (2, 5, 10, 50, 200)]
    assert all(a > b for a, b in zip(Rs, Rs[1:]))
    for k in (2, 10, 200):
        R = orc.target_radius(1e5, 1.0, k)
        assert abs(orc.kbar_approx(1e5, 1.0, R) - k) / k < 1e-9
        # decreasing there
        assert orc.kbar_approx(1e5, 1.0, R + 1e-3) < orc.kbar_approx(1e5, 1.0, R - 1e-3)


@pytest.mark.parametrize("args", [(1e4, 0.5, 10), (1e4, 0.3, 10), (1e4, 1.0, 0.0), (1e4, 1.0, -1.0),
                                  (1e4, 1.0, 1e12), (1.0, 1.0, 1.0), (1e4, float("nan"), 10)])
def test_target_radius_rejects(orc, args):
    with pytest.raises(ValueError):
        orc.target_radius(*args)


def test_target_radius_grows_like_2_ln_n(orc):
    # for fixed kbar, R - 2 ln n tends to a constant (the e^{-R/2} term dominates)
    d = [orc.target_radius(n, 1.0, 10) - 2 * math.log(n) for n in (1e6, 1e8, 1e10)]
    assert abs(d[1] - d[2]) < 1e-3 and abs(d[0] - d[1]) < 2e-2


@pytest.mark.parametrize("R,B,p", [(15.68, 14, 0.9), (26.5, 24, 0.9), (10.0, 1, 0.9), (30.0, 40, 0.5),
                                   (20.0, 7, 0.99)])
def test_boundaries_invariants(orc, R, B, p):
    c = orc.boundaries(R, B, p)
    assert len(c) == B + 1 and c[0] == 0.0 and c[-1] == R
    w = np.diff(c)
    assert np.all(w > 0)
    if B >= 3:
        ratios = w[1:-1] / w[:-2]
        assert np.allclose(ratios, p, rtol=1e-12)
    # the last width is whatever closes the sum at R: equal to c_1 p^{B-1} up to rounding
    assert abs(w[-1] - w[0] * p ** (B - 1)) < 1e-9 * R


def test_band_of_half_open(orc):
    c = orc.boundaries(20.0, 10, 0.9)
    for i in range(10):
        assert orc.band_of(c[i], c) == i                     # c_i belongs to slab i
        if i > 0:
            assert orc.band_of(np.nextafter(c[i], 0.0), c) == i - 1
    assert orc.band_of(20.0, c) == 9                          # r = R: last slab
    assert orc.band_of(0.0, c) == 0


def test_default_bands(orc):
    assert orc.default_bands(2) == 1
    assert orc.default_bands(10_000) == 14
    assert orc.default_bands(1_000_000) == 20
    assert orc.default_bands(10_000_000) == 24
    assert orc.default_bands(1 << 20) == 20
    assert orc.default_bands((1 << 20) + 1) == 21

"""The radius domain R <= 354, on both sides of the boundary.

Eq. 3 is evaluated as cosh(r_u - r_v) + 2 sinh r_u sinh r_v sin^2(dtheta/2).
Its largest product, 2 sinh^2 R ~ e^{2R}/2, overflows near R = 355.2; past
that, two coincident points on the rim meet inf * 0 = NaN and would be
declared non-adjacent although their distance is 0.  Both the oracle and the
library therefore accept 0 < R <= 354 and refuse anything larger.  Checked
here on the CPU: the overflow point itself (so the bound is derived, not
assumed), the oracle's entry points at the bound and one ulp past it, the
predicate's answers at the bound, and the library's host-side validation.
"""
import math

import numpy as np
import pytest

from paper_1606_09481_amd import rhg

R_MAX = 354.0
PAST = float(np.nextafter(R_MAX, np.inf))


def test_bound_sits_below_the_overflow():
    # 2 sinh^2 R: finite at the bound with room to spare, infinite a little past 355.2
    s = np.sinh(np.float64(R_MAX))
    assert np.isfinite(np.float64(2.0) * s * s)
    assert np.isfinite(np.float64(2.0) * s * s * np.float64(8.0))  # headroom for the rounding of sinh
    with np.errstate(over="ignore"):
        s2 = np.sinh(np.float64(355.3))
        assert not np.isfinite(np.float64(2.0) * s2 * s2)
        # where the bound was not closed: the product overflows and 0 * inf is NaN
        assert math.isnan(float(np.float64(2.0) * s2 * s2 * np.float64(0.0)))


def test_predicate_at_the_bound(orc):
    # coincident rim points are adjacent (distance 0); opposite ones are not
    th = np.array([1.0, 1.0, 1.0 + math.pi, 2.0])
    r = np.array([R_MAX, R_MAX, R_MAX, R_MAX - 1e-9])
    t = orc.table(th, r)
    K = math.cosh(R_MAX)
    V = orc.coshdist(t, 0, 1)
    assert V == 1.0
    assert orc.is_edge(t, 0, 1, K)
    assert not orc.is_edge(t, 0, 2, K) and np.isfinite(orc.coshdist(t, 0, 2))
    e = orc.brute(t, K)
    assert [tuple(x) for x in e] == [(0, 1)]
    es = orc.sort_edges(orc.band_sweep(th, r, t, R_MAX, K, B=3))
    assert np.array_equal(es, e)


def test_oracle_refuses_past_the_bound(orc):
    th, r = orc.sample(50, 1.0, R_MAX, 3)
    assert np.all(r <= R_MAX)
    with pytest.raises(ValueError):
        orc.sample(50, 1.0, PAST, 3)
    with pytest.raises(ValueError):
        orc.sample(50, 5.0, 300.0, 3)  # sinh(alpha R / 2) overflows
    t = orc.table(th, r)
    orc.band_sweep(th, r, t, R_MAX, math.cosh(R_MAX))
    with pytest.raises(ValueError):
        orc.band_sweep(th, r, t, PAST, math.cosh(PAST))
    with pytest.raises(ValueError):
        orc.brute(t, math.cosh(PAST))
    with pytest.raises(ValueError):
        orc.brute_rows(t, math.cosh(PAST), [0, 1])
    with pytest.raises(ValueError):
        orc.brute_rows(t, math.cosh(R_MAX), [0, 50])  # a query outside 0..n-1


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(rhg.LIB_PATH):
        from paper_1606_09481_amd import build
        build.build()
    return rhg.load()


def test_library_refuses_past_the_bound(lib):
    # rhg_server_estimate_bytes validates exactly as a generation does (host only)
    assert rhg.rhg_server_estimate_bytes(rhg.params(1000, 1.0, R=R_MAX)) > 0
    for R in (PAST, 355.3, 700.0, float("inf")):
        with pytest.raises(rhg.RhgError) as ei:
            rhg.rhg_server_estimate_bytes(rhg.params(1000, 1.0, R=R))
        assert ei.value.status == rhg.RHG_EINVAL
    with pytest.raises(rhg.RhgError) as ei:  # the seeded sampler needs sinh(alpha R / 2) finite
        rhg.rhg_server_estimate_bytes(rhg.params(1000, 5.0, R=300.0))
    assert ei.value.status == rhg.RHG_EINVAL

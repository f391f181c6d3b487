"""Pins of the oracle's general model at temperature T > 0 (Sec. II, Eq. 2).

Eq. 2 gives a pair at distance x the edge probability
f(x) = 1 / (exp((x - R) / (2T)) + 1).  The oracle decides each unordered pair
with its own uniform from the counter generator.  Checked here against what
the model and the mathematics fix, not against the oracle's own formula:

* closed forms of Eq. 2: f = 1/2 at x = R, 1/4 and 3/4 at x = R +- 2T ln 3,
  1/20 at R + 2T ln 19, whatever T;
* the edge frequency of a pair at those distances over many seeds
  (a binomial test: catches a wrong sign, a factor 2 on T, T in place of 1/T);
* the uniforms: in (0, 1], uniform (KS), distinct per pair;
* the limit T -> 0 is the threshold graph (the threshold oracle is pinned
  on its own), except pairs within 80 T of distance R;
* the mean degree over seeds against the model's expected degree by
  quadrature of Eq. 1 and Eq. 2 (integrator cross-checked against the
  threshold model's quadrature as T -> 0);
* the band sweep with the enlarged radius equals all pairs, on model,
  adversarial and uniform-radius inputs and for several slab counts;
* symmetry of the decision, and the domain 0 < T < 1.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

from inputs import adversarial_coords, uniform_coords
from test_oracle_params import expected_degree


def _pair_table(orc, x_list, R):
    """Pairs (2k, 2k+1) at opposite angles with equal radii x/2: distance x exactly (r_u + r_v)."""
    th = np.empty(2 * len(x_list))
    r = np.empty(2 * len(x_list))
    for k, x in enumerate(x_list):
        th[2 * k], th[2 * k + 1] = 1.0, 1.0 + math.pi
        r[2 * k] = r[2 * k + 1] = x / 2.0
    return th, r, orc.table(th, r)


@pytest.mark.parametrize("T", [0.05, 0.3, 0.8])
def test_closed_forms(orc, T):
    R = 20.0
    for x, want in [(R, 0.5), (R + 2 * T * math.log(3), 0.25), (R - 2 * T * math.log(3), 0.75),
                    (R + 2 * T * math.log(19), 0.05)]:
        assert orc.fd_prob(math.cosh(x), R, T) == pytest.approx(want, rel=1e-9)
    # coincident points (V = 1, and V rounded below 1): distance 0
    assert orc.fd_prob(1.0, R, T) == pytest.approx(1.0 / (1.0 + math.exp(-R / (2 * T))), rel=1e-15)
    assert orc.fd_prob(1.0 - 2 ** -52, R, T) == orc.fd_prob(1.0, R, T)
    # decreasing in the distance
    V = np.cosh(np.linspace(0.0, R + 80 * T, 200))
    f = np.array([orc.fd_prob(v, R, T) for v in V])
    assert np.all(np.diff(f) <= 0) and f[-1] < 1e-15


@pytest.mark.parametrize("T", [0.1, 0.5])
def test_edge_frequency_at_known_distances(orc, T):
    R = 18.0
    xs = [R - 2 * T * math.log(3), R, R + 2 * T * math.log(3), R + 2 * T * math.log(19)]
    want = [0.75, 0.5, 0.25, 0.05]
    th, r, t = _pair_table(orc, xs, R)
    seeds = 20000
    for k, p in enumerate(want):
        hits = sum(orc.soft_is_edge(t, 2 * k, 2 * k + 1, R, T, s) for s in range(seeds))
        sd = math.sqrt(p * (1 - p) / seeds)
        assert abs(hits / seeds - p) < 5 * sd, (xs[k], hits / seeds, p)


def test_uniforms(orc):
    u = np.array([orc.pair_uniform(11, i, j) for i in range(0, 300) for j in range(i + 1, i + 40)])
    assert u.min() > 0.0 and u.max() <= 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    assert len(np.unique(u)) == len(u)
    # a different seed gives different numbers for the same pair
    assert orc.pair_uniform(11, 3, 7) != orc.pair_uniform(12, 3, 7)


def test_symmetric_decision(orc):
    R, T = 14.0, 0.3
    th, r = orc.sample(300, 1.0, R, 2)
    t = orc.table(th, r)
    rng = np.random.default_rng(0)
    for _ in range(2000):
        u, v = rng.integers(0, 300, 2)
        assert orc.soft_is_edge(t, u, v, R, T, 5) == orc.soft_is_edge(t, v, u, R, T, 5)
    assert not orc.soft_is_edge(t, 4, 4, R, T, 5)


@pytest.mark.parametrize("kind", ["model", "adversarial"])
def test_low_temperature_limit_is_the_threshold_graph(orc, kind):
    # pairs further than 80 T from distance R have f within e^-40 of 0 or 1,
    # so only they may differ; the adversarial set puts many pairs at exactly
    # R (a point at the centre and one on the rim), which connect half the time
    n, alpha = 3000, 0.8
    R = orc.target_radius(n, alpha, 12)
    if kind == "model":
        th, r = orc.sample(n, alpha, R, 4)
    else:
        th, r = adversarial_coords(n, R, orc.boundaries(R, orc.default_bands(n)), 4)
    t = orc.table(th, r)
    hard = {tuple(x) for x in orc.brute(t, math.cosh(R))}
    for T in (1e-9, 1e-6):
        soft = {tuple(x) for x in orc.soft_brute(t, R, T, 9)}
        diff = hard ^ soft
        for (u, v) in diff:
            x = math.acosh(max(1.0, orc.coshdist(t, u, v)))
            assert abs(x - R) <= 80 * T or orc.pair_uniform(9, u, v) == 1.0, (u, v, x - R)
        if kind == "model":
            assert len(diff) <= 2


def _soft_expected_degree(n, alpha, R, T, nr=240, nphi=400):
    """(n - 1) * int int rho(r1) rho(r2) (1/pi) int_0^pi f(x) dphi dr1 dr2 (Eq. 1, Eq. 2, Eq. 3)."""
    xr, wr = np.polynomial.legendre.leggauss(nr)
    rr = 0.5 * R * (xr + 1.0)
    w_r = 0.5 * R * wr * alpha * np.sinh(alpha * rr) / (math.cosh(alpha * R) - 1.0)
    # phi on a log scale: the probability changes over angles as small as e^{-R}
    lo = -2.0 * R - 5.0
    xp, wp = np.polynomial.legendre.leggauss(nphi)
    s = lo + (math.log(math.pi) - lo) * 0.5 * (xp + 1.0)
    phi = np.exp(s)
    w_phi = (math.log(math.pi) - lo) * 0.5 * wp * phi / math.pi
    sin2 = np.sin(phi / 2.0) ** 2
    tot = 0.0
    for i in range(nr):
        a = np.cosh(rr[i] - rr)[:, None]
        b = 2.0 * np.sinh(rr[i]) * np.sinh(rr)[:, None]
        x = np.arccosh(np.maximum(a + b * sin2[None, :], 1.0))
        f = special.expit(-(x - R) / (2.0 * T))
        tot += w_r[i] * float(np.sum(w_r[:, None] * f * w_phi[None, :]))
    return (n - 1) * tot


def test_quadrature_matches_the_threshold_model_as_T_goes_to_zero(orc):
    n, alpha = 2000, 1.0
    R = orc.target_radius(n, alpha, 10)
    hard = expected_degree(n, alpha, R)
    soft = _soft_expected_degree(n, alpha, R, 1e-4)
    assert soft == pytest.approx(hard, rel=2e-3)


@pytest.mark.parametrize("alpha,T", [(1.0, 0.3), (0.75, 0.5), (1.0, 0.05)])
def test_mean_degree_over_seeds(orc, alpha, T):
    n = 2000
    R = orc.target_radius(n, alpha, 10)
    degs = []
    for seed in range(1, 41):
        th, r = orc.sample(n, alpha, R, seed)
        t = orc.table(th, r)
        e = orc.soft_band_sweep(th, r, t, R, T, seed, threads=4)
        degs.append(2.0 * len(e) / n)
    degs = np.array(degs)
    E = _soft_expected_degree(n, alpha, R, T)
    se = degs.std(ddof=1) / math.sqrt(len(degs))
    assert abs(degs.mean() - E) < 4 * se, (degs.mean(), E, se)
    # and the temperature matters: the threshold model's degree is well apart
    if T >= 0.3:
        assert abs(degs.mean() - expected_degree(n, alpha, R)) > 8 * se


@pytest.mark.parametrize("kind,B", [("model", None), ("model", 1), ("model", 40), ("adversarial", 3),
                                    ("uniform", None)])
@pytest.mark.parametrize("T", [0.02, 0.2, 0.6])
def test_band_sweep_equals_all_pairs(orc, kind, B, T):
    n, alpha = 2500, 0.9
    R = orc.target_radius(n, alpha, 8)
    if kind == "model":
        th, r = orc.sample(n, alpha, R, 3)
    elif kind == "adversarial":
        th, r = adversarial_coords(n, R, orc.boundaries(R, 3), 6)
    else:
        th, r = uniform_coords(n, R, 7)
    t = orc.table(th, r)
    ref, ties = orc.soft_brute(t, R, T, 21, with_ties=True)
    got, gties = orc.soft_band_sweep(th, r, t, R, T, 21, B=B, with_ties=True)
    assert np.array_equal(orc.sort_edges(got), ref)
    assert np.array_equal(orc.sort_edges(gties), ties)


def test_domain(orc):
    th, r = orc.sample(100, 1.0, 10.0, 1)
    t = orc.table(th, r)
    for T in (0.0, -0.1, 1.0, float("nan")):
        with pytest.raises(ValueError):
            orc.soft_brute(t, 10.0, T, 1)
        with pytest.raises(ValueError):
            orc.soft_band_sweep(th, r, t, 10.0, T, 1)

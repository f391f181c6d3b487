"""Pins of the oracle's movement step (dynamic model, Sec. III-C, Algorithm 2,
Theorem 1), against what the mathematics fixes rather than the oracle's own
formula:

* the defining relation of the radial step in the coordinate w = cosh(alpha r):
  w' = w + tau_r inside the disk, mirrored at the end it crosses (w' = 2 - w -
  tau_r at the centre, 2 cosh(alpha R) - w - tau_r at the rim, two crossings
  subtract a whole period), with tau_r negated once per reflection;
* the rotation: theta' = theta + tau_phi exactly when no wrap occurs,
  theta' in [0, 2 pi) and congruent to theta + tau_phi otherwise;
* tau = 0 returns the point exactly;
* Theorem 1: after many steps with symmetric random steps, the radii still
  follow F(r) = (cosh(alpha r) - 1) / (cosh(alpha R) - 1) and the angles are
  uniform (Kolmogorov-Smirnov); two controls show the test has power: a
  one-sided step breaks the law, and so does the step as printed (on
  sinh(alpha r), which is not uniform near the centre).
"""
import numpy as np
import pytest
from scipy import stats

TWO_PI = 2.0 * np.pi


def _w(r, alpha):
    return np.cosh(alpha * r)


def _pts(orc, n, alpha, R, seed):
    return orc.sample(n, alpha, R, seed)


def test_radial_step_inside(orc):
    alpha, R = 0.8, 18.0
    th, r = _pts(orc, 4000, alpha, R, 11)
    rng = np.random.default_rng(1)
    W = _w(R, alpha)
    w = _w(r, alpha)
    tau = rng.uniform(-1, 1, len(r)) * np.minimum(w - 1.0, W - w) * 0.9  # stays inside
    th2, r2, t2 = orc.move(th, r, np.zeros_like(r), tau, alpha, R)
    assert np.array_equal(t2, tau)
    err = np.abs(_w(r2, alpha) - (w + tau))
    assert np.all(err <= 1e-13 * (w + np.abs(tau)))
    assert np.all((r2 >= 0) & (r2 <= R))
    assert np.array_equal(th2, th)  # tau_phi = 0 with th in [0, 2 pi): unchanged


def test_radial_step_near_centre(orc):
    """Small radii: the step keeps relative precision (no cancellation in cosh - 1)."""
    alpha, R = 1.0, 15.0
    r = np.array([1e-6, 1e-4, 1e-2, 0.1, 0.5])
    tau = np.sinh(alpha * r / 2) ** 2  # = (w - 1) / 2, without forming cosh - 1
    _, r2, _ = orc.move(np.zeros(5), r, np.zeros(5), tau, alpha, R)
    # w' - 1 = 1.5 (w - 1)  <=>  sinh^2(alpha r'/2) = 1.5 sinh^2(alpha r/2)
    lhs = np.sinh(alpha * r2 / 2) ** 2
    rhs = 1.5 * np.sinh(alpha * r / 2) ** 2
    assert np.all(np.abs(lhs - rhs) <= 1e-14 * rhs)


def test_reflection_at_rim_and_centre(orc):
    alpha, R = 1.0, 12.0
    W = _w(R, alpha)
    r = np.array([11.9, 11.5, 0.3, 1.0])
    w = _w(r, alpha)
    tau = np.array([W - w[0] + 1000.0, (W - w[1]) * 1.5, -(w[2] - 1.0) * 3.0, -(w[3] - 1.0) - 0.25])
    _, r2, t2 = orc.move(np.zeros(4), r, np.zeros(4), tau, alpha, R)
    assert np.array_equal(t2, -tau)
    w2 = _w(r2, alpha)
    want = np.array([2 * W - w[0] - tau[0], 2 * W - w[1] - tau[1], 2 - w[2] - tau[2], 2 - w[3] - tau[3]])
    assert np.all(np.abs(w2 - want) <= 1e-12 * (w + np.abs(tau)))


def test_two_reflections(orc):
    alpha, R = 1.0, 8.0
    W = _w(R, alpha)
    r = np.array([4.0, 7.0])
    w = _w(r, alpha)
    P = 2 * (W - 1)
    tau = np.array([P + 0.5 * (W - w[0]), -(P + 0.25 * (w[1] - 1))])  # one full period plus a step inside
    _, r2, t2 = orc.move(np.zeros(2), r, np.zeros(2), tau, alpha, R)
    assert np.array_equal(t2, tau)  # two reflections: direction kept
    want = w + tau - np.sign(tau) * P
    assert np.all(np.abs(_w(r2, alpha) - want) <= 1e-12 * (w + np.abs(tau)))


def test_rotation(orc):
    rng = np.random.default_rng(5)
    th = rng.uniform(0, TWO_PI, 5000)
    tp = rng.uniform(-7, 7, 5000)
    th2, _, _ = orc.move(th, np.full(5000, 1.0), tp, np.zeros(5000), 1.0, 10.0)
    assert np.all((th2 >= 0) & (th2 < TWO_PI))
    inside = (th + tp >= 0) & (th + tp < TWO_PI)
    assert np.array_equal(th2[inside], (th + tp)[inside])
    k = np.round((th + tp - th2) / TWO_PI)
    assert np.all(np.abs(th + tp - th2 - k * TWO_PI) <= 1e-14 * (TWO_PI + np.abs(tp)))


def test_zero_step_is_identity(orc):
    alpha, R = 0.75, 20.0
    th, r = _pts(orc, 3000, alpha, R, 2)
    th2, r2, t2 = orc.move(th, r, np.zeros_like(r), np.zeros_like(r), alpha, R)
    assert np.array_equal(th2, th)
    assert np.array_equal(r2, r) and np.array_equal(t2, np.zeros_like(r))  # a zero step moves nothing


def _radius_cdf(alpha, R):
    return lambda x: (np.cosh(alpha * np.clip(x, 0, R)) - 1.0) / (np.cosh(alpha * R) - 1.0)


@pytest.mark.parametrize("alpha,R", [(1.0, 3.0), (1.0, 6.0), (0.6, 9.0)])
def test_theorem1_density_preserved(orc, alpha, R):
    """Symmetric random steps as large as the whole disk: 30 steps keep Eq. 1's radius law and uniform angles."""
    n = 60_000
    th, r = _pts(orc, n, alpha, R, 3)
    rng = np.random.default_rng(9)
    W = _w(R, alpha)
    tp = rng.uniform(-1, 1, n)
    tr = rng.uniform(-1, 1, n) * (W - 1.0) * 0.7
    for _ in range(30):
        th, r, tr = orc.move(th, r, tp, tr, alpha, R)
    assert stats.kstest(r, _radius_cdf(alpha, R)).pvalue > 1e-3
    assert stats.kstest(th / TWO_PI, "uniform").pvalue > 1e-3


def test_theorem1_controls_have_power(orc):
    """The KS check above detects (a) one-sided steps and (b) the step taken on sinh(alpha r) as printed
    (alpha R = 3: enough mass near the centre, where sinh and cosh differ)."""
    alpha, R, n = 1.0, 3.0, 60_000
    th, r = _pts(orc, n, alpha, R, 4)
    W = _w(R, alpha)
    rng = np.random.default_rng(10)
    # (a) every node steps outward by 0.3 of the range: one step piles mass near the rim
    _, r1, _ = orc.move(th, r, np.zeros(n), np.full(n, 0.3 * (W - 1.0)), alpha, R)
    assert stats.kstest(r1, _radius_cdf(alpha, R)).pvalue < 1e-6
    # (b) the printed form: x = sinh(alpha r) shifted and reflected in [0, sinh(alpha R)]
    X = np.sinh(alpha * R)
    x = np.sinh(alpha * r)
    t = rng.uniform(-1, 1, n) * X * 0.7
    for _ in range(30):
        y = x + t
        k = np.floor(y / X)
        odd = (np.abs(k) % 2) == 1
        x = np.where(odd, (k + 1) * X - y, y - k * X)
        t = np.where(odd, -t, t)
    r2 = np.arcsinh(x) / alpha
    assert stats.kstest(r2, _radius_cdf(alpha, R)).pvalue < 1e-6

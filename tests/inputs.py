"""Seeded synthetic coordinate sets shared by the oracle tests and the GPU tests.

This module holds none of the method's arithmetic: it only draws and arranges
numbers (numpy's PCG64 generator) into angle/radius arrays with awkward
structure -- exact duplicates, angles at 0 and at the largest allowed angle,
radii exactly on caller-supplied values (slab boundaries, 0, R), tight angular
clusters.  Model-distributed points come from each side's own sampler, not
from here.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi  # largest angle accepted (fl(2*pi)); angles live in [0, TWO_PI]


def uniform_coords(n: int, R: float, seed: int):
    """Angles uniform in [0, 2pi), radii uniform in [0, R] (not the model law)."""
    g = np.random.default_rng(seed)
    return g.random(n) * TWO_PI, g.random(n) * R


def outer_heavy_coords(n: int, R: float, seed: int, scale: float = 1.0):
    """Radii R - Exp(scale) clipped at 0: most points near the rim, a few deep inside."""
    g = np.random.default_rng(seed)
    r = R - g.exponential(scale, n)
    return g.random(n) * TWO_PI, np.clip(r, 0.0, R)


def adversarial_coords(n: int, R: float, special_radii, seed: int):
    """Awkward points: radii on the given values, 0 and R; angles at 0, TWO_PI and
    in tight clusters; exact duplicate points; the rest rim-heavy."""
    g = np.random.default_rng(seed)
    theta, r = outer_heavy_coords(n, R, seed + 1000)
    special = np.asarray(list(special_radii) + [0.0, R], dtype=np.float64)
    k = n // 8
    idx = g.choice(n, size=k, replace=False)
    r[idx] = special[g.integers(0, len(special), size=k)]
    idx = g.choice(n, size=n // 16, replace=False)
    theta[idx] = np.where(g.random(len(idx)) < 0.5, 0.0, TWO_PI)
    # clusters: groups of 8 points within 1e-15 .. 1e-9 of a centre angle
    for c in range(max(1, n // 64)):
        centre = g.random() * TWO_PI
        ids = g.choice(n, size=8, replace=False)
        theta[ids] = np.clip(centre + g.standard_normal(8) * 10.0 ** g.uniform(-15, -9), 0.0, TWO_PI)
    # exact duplicates
    for c in range(max(1, n // 50)):
        a, b = g.choice(n, size=2, replace=False)
        theta[b], r[b] = theta[a], r[a]
    return theta, r

"""Writes the stored edge lists under tests/golden/ by calling only the oracle.

The paper prints no worked example (no coordinates, no edge list), so the
fixtures here are regression anchors for the oracle itself: a small model
graph (n = 2000, alpha = 1, average degree 10 -> R by getTargetRadius,
SplitMix64 seed 1), its R, and its edge list from the all-pairs definition.
Run: python tests/golden/make_golden.py
"""
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402


def main():
    n, alpha, kbar, seed = 2000, 1.0, 10.0, 1
    R = oracle.target_radius(n, alpha, kbar)
    th, r = oracle.sample(n, alpha, R, seed)
    t = oracle.table(th, r)
    e = oracle.brute(t, math.cosh(R))
    path = os.path.join(HERE, "n2000_a1_k10_seed1.txt")
    with open(path, "w") as f:
        f.write("# threshold RHG, n=2000 alpha=1.0 kbar=10 seed=1 (SplitMix64), all-pairs oracle\n")
        f.write("# R=%s m=%d\n" % (float(R).hex(), len(e)))
        np.savetxt(f, e, fmt="%d")


if __name__ == "__main__":
    main()

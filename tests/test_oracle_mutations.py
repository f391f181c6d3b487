"""Planted mistakes in the oracle must each fail one of its pins.

Each case copies oracle/rhg_oracle.c, plants one plausible mistake (a
dropped term, a wrong sign, an off-by-one constant, a missing widening, a
broken reading of the paper), builds it with the oracle's own flags, and runs
the pin modules named for it against that build (RHG_ORACLE_LIB) in a
subprocess: the run must fail.  A mistake the pins let through would mean a
wrong oracle could pass, and with it a wrong GPU path.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "rhg_oracle.c")

# (name, original text, planted text, pin modules that must catch it)
MUTATIONS = [
    ("half-angle difference sign", "double d = t->hs[u] * t->hc[v] - t->hc[u] * t->hs[v];",
     "double d = t->hs[u] * t->hc[v] + t->hc[u] * t->hs[v];", ["test_oracle_predicate.py"]),
    ("factor 2 of the angular term", "return a + 2.0 * b;", "return a + b;", ["test_oracle_predicate.py"]),
    ("halving of cosh(r_u - r_v)", "double a = 0.5 * (t1 + t2);", "double a = (t1 + t2);",
     ["test_oracle_predicate.py"]),
    ("strict threshold", "return orc_V(&t, u, v) < K;", "return orc_V(&t, u, v) <= K;",
     ["test_oracle_predicate.py"]),
    ("sinh from the exponentials", "sh[i] = 0.5 * (ep[i] - em[i]);", "sh[i] = 0.5 * (ep[i] + em[i]);",
     ["test_oracle_sampling.py"]),
    ("window without widening", "double Kw = K * (1.0 + 1e-9);\n    double s = (Kw - cosh(rv - c)) / den;\n    if (s >= 1.0) return 1;\n    if (s < 0.0) s = 0.0;\n    double d = 2.0 * asin(sqrt(s));\n    d = d * (1.0 + 1e-9) + 1e-13;",
     "double s = (K - cosh(rv - c)) / den;\n    if (s >= 1.0) return 1;\n    if (s < 0.0) s = 0.0;\n    double d = 2.0 * asin(sqrt(s));",
     ["test_oracle_sweep.py"]),
    ("same-slab pairs once", "if (j == X->band[v] && w < v) continue; /* same slab",
     "if (0) continue; /* same slab", ["test_oracle_sweep.py"]),
    ("radius inverse CDF factor 2", "double ri = 2.0 * asinh(sqrt(u2) * sR) / alpha;",
     "double ri = asinh(sqrt(u2) * sR) / alpha;", ["test_oracle_sampling.py"]),
    ("angle range", "theta[i] = u1 * ORC_TWO_PI;", "theta[i] = u1 * ORC_PI;", ["test_oracle_sampling.py"]),
    ("SplitMix64 constant", "z = (z ^ (z >> 30)) * UINT64_C(0xBF58476D1CE4E5B9);",
     "z = (z ^ (z >> 30)) * UINT64_C(0xBF58476D1CE4E5B8);", ["test_oracle_sampling.py"]),
    ("getTargetRadius (pi - 1) term", "- (ORC_PI - 1.0) * za", "- (ORC_PI + 1.0) * za",
     ["test_oracle_params.py"]),
    ("slab width ratio", "width *= p;", "width /= p;", ["test_oracle_params.py"]),
    ("reflection at the ends", "double s2 = odd ? (k + 1.0) * S - y : y - k * S;",
     "double s2 = y - k * S;", ["test_oracle_dynamic.py"]),
    ("Eq. 2 factor 2 on T", "double y = (x - R) / (2.0 * T);", "double y = (x - R) / T;",
     ["test_oracle_soft.py"]),
    ("Eq. 2 sign", "double y = (x - R) / (2.0 * T);", "double y = (R - x) / (2.0 * T);", ["test_oracle_soft.py"]),
    ("general model cutoff", "X.Kc = cosh(R + 80.0 * T);", "X.Kc = cosh(R + 2.0 * T);", ["test_oracle_soft.py"]),
    ("acosh below 1", "double x = V > 1.0 ? acosh(V) : 0.0;", "double x = acosh(V);", ["test_oracle_soft.py"]),
]


@pytest.mark.parametrize("name,orig,planted,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(tmp_path, name, orig, planted, pins):
    src = open(SRC).read()
    assert src.count(orig) == 1, "mutation site not found once: %s" % orig
    mut = tmp_path / "rhg_oracle_mut.c"
    mut.write_text(src.replace(orig, planted))
    lib = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-pthread", "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, RHG_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", p) for p in pins]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "planted mistake '%s' passed every pin in %s:\n%s" % (name, pins, r.stdout[-2000:])
    assert "failed" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]

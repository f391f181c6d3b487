"""Parity beyond 32-bit batch offsets and beyond 32-bit table offsets.

* n = 1.2*10^8, alpha = 0.55, kbar = 8: hub batches whose 64 windows in one
  slab hold more than 2^32 candidates (the window scan and the walk's
  offsets then run in 64 bits, rebased per work unit);
* n = 2^28 + 3, alpha = 1, kbar = 4: table byte offsets above 2^32 (64-bit
  addressing of the table).

As at the benchmark sizes, the oracle answers for sampled vertices (random,
innermost hubs, outermost) by the all-pairs definition on those rows; the
device gets the oracle's own table (table mode), so the incident edges must
be identical, in both precision forms, and the whole output must be valid.
"""
import math
import time

import numpy as np
import pytest

from paper_1606_09481_amd import rhg
from test_gpu_fullsize import _device_view, _incident_device

pytestmark = pytest.mark.gpu


def _rows(r, n, rng, k_rand=32, k_end=8):
    inner = np.argpartition(r, k_end)[:k_end]
    outer = np.argpartition(r, n - k_end)[n - k_end:]
    return np.unique(np.concatenate([rng.choice(n, k_rand, replace=False), inner, outer]))


@pytest.mark.parametrize("n,alpha,kbar,precs", [(120_000_001, 0.55, 8.0, (rhg.RHG_FP64, rhg.RHG_FP32_RECHECK)),
                                                 ((1 << 28) + 3, 1.0, 4.0, (rhg.RHG_FP64,))])
def test_big_n_table_mode(orc, n, alpha, kbar, precs):
    t0 = time.time()
    print("case", n, alpha, kbar, flush=True)
    R = orc.target_radius(n, alpha, kbar)
    th, r = orc.sample(n, alpha, R, 1)
    t = orc.table(th, r)
    rows = _rows(r, n, np.random.default_rng(n))
    ref = orc.brute_rows(t, math.cosh(R), rows)
    ref = np.unique(np.sort(ref.reshape(-1, 2), axis=1).astype(np.int64) @ np.array([1 << 32, 1], np.int64))
    print("oracle: %d incident edges of %d vertices (%.0f s)" % (len(ref), len(rows), time.time() - t0), flush=True)
    rhg.load()
    c = rhg.rhg_ctx_create(0)
    try:
        for prec in precs:
            g = rhg.rhg_generate_from_table(c, th, r, t, R, prec)
            try:
                m = rhg.rhg_graph_num_edges(g)
                got = _incident_device(_device_view(rhg.rhg_graph_edges_device(g), 2 * m), m, rows, n)
                st = rhg.rhg_graph_stats(g)
            finally:
                rhg.rhg_graph_free(g)
            print("precision %d: m %d, candidates %d (%.0f s)" % (prec, m, st["candidates"], time.time() - t0),
                  flush=True)
            assert len(got) == len(ref) and np.array_equal(got, ref), "precision %d" % prec
    finally:
        rhg.rhg_ctx_destroy(c)

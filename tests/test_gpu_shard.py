"""One query share of a generation, as one of S devices would run it
(RHG_OPT_SHARD_COUNT / RHG_OPT_SHARD_INDEX).

Every point is still sampled, sorted and planned; only the 64-query batches of
share k (cut on the candidate prefix of the plan) are counted and emitted.
Each edge is found by exactly one query (Alg. 1 queries outward; the own slab
by the forward rule), so:
  * the S shares' edge lists are pairwise disjoint and their union is the
    whole graph, which the other parity tests pin to the oracle;
  * their edge and candidate counts add up to the whole graph's;
for both precision forms, ragged cuts, more shares than batches (empty
shares), and S = 1 (byte-identical to the ordinary generation).  A share index
outside [0, S) is refused.
"""
import numpy as np
import pytest

from paper_1606_09481_amd import rhg

pytestmark = pytest.mark.gpu


def _ctx(S=None, k=None):
    rhg.load()
    c = rhg.rhg_ctx_create(0)
    if S is not None:
        rhg.rhg_ctx_set_option(c, rhg.RHG_OPT_SHARD_COUNT, S)
        rhg.rhg_ctx_set_option(c, rhg.RHG_OPT_SHARD_INDEX, k)
    return c


def _generate(c, p):
    g = rhg.rhg_generate(c, p)
    try:
        e = rhg.rhg_graph_copy_edges(g).reshape(-1, 2).astype(np.int64)
        st = rhg.rhg_graph_stats(g)
    finally:
        rhg.rhg_graph_free(g)
    return e, st


def _keys(e):
    return np.sort((e[:, 0] << 32) | e[:, 1])


@pytest.mark.parametrize("n,alpha,kbar,S", [(60_000, 0.75, 20, 3), (60_000, 0.75, 20, 8), (40_001, 0.55, 12, 5),
                                            (1_000, 1.0, 10, 64)])
@pytest.mark.parametrize("prec", [rhg.RHG_FP64, rhg.RHG_FP32_RECHECK])
def test_shares_partition_the_graph(n, alpha, kbar, S, prec):
    print("case", n, alpha, kbar, S, prec, flush=True)
    p = rhg.params(n, alpha, kbar=kbar, seed=3, precision=prec)
    c = _ctx()
    try:
        full, st_full = _generate(c, p)
    finally:
        rhg.rhg_ctx_destroy(c)
    parts, m_sum, cand_sum = [], 0, 0
    for k in range(S):
        c = _ctx(S, k)
        try:
            e, st = _generate(c, p)
        finally:
            rhg.rhg_ctx_destroy(c)
        assert st["edges"] == len(e)
        m_sum += len(e)
        cand_sum += st["candidates"]
        parts.append(e)
    assert m_sum == len(full)
    assert cand_sum == st_full["candidates"]
    u = _keys(np.concatenate(parts))
    assert np.all(u[1:] != u[:-1]), "an edge found by two shares"
    assert np.array_equal(u, _keys(full)), "the shares' union is not the whole graph"
    if S > 16:
        assert sum(len(e) == 0 for e in parts) > 0  # more shares than batches: some are empty


def test_single_share_is_the_generation():
    p = rhg.params(30_000, 1.0, kbar=16, seed=4)
    c = _ctx()
    c1 = _ctx(1, 0)
    try:
        a, _ = _generate(c, p)
        b, _ = _generate(c1, p)
    finally:
        rhg.rhg_ctx_destroy(c)
        rhg.rhg_ctx_destroy(c1)
    assert np.array_equal(a, b)


def test_share_options_checked():
    c = _ctx()
    try:
        for opt, v in [(rhg.RHG_OPT_SHARD_COUNT, 0), (rhg.RHG_OPT_SHARD_COUNT, 1 << 20), (rhg.RHG_OPT_SHARD_INDEX, -1)]:
            with pytest.raises(rhg.RhgError) as ei:
                rhg.rhg_ctx_set_option(c, opt, v)
            assert ei.value.status == rhg.RHG_EINVAL
        rhg.rhg_ctx_set_option(c, rhg.RHG_OPT_SHARD_COUNT, 4)
        rhg.rhg_ctx_set_option(c, rhg.RHG_OPT_SHARD_INDEX, 4)
        with pytest.raises(rhg.RhgError) as ei:
            rhg.rhg_generate(c, rhg.params(10_000, 1.0, kbar=10, seed=1))
        assert ei.value.status == rhg.RHG_EINVAL
        rhg.rhg_ctx_set_option(c, rhg.RHG_OPT_SHARD_INDEX, 3)
        g = rhg.rhg_generate(c, rhg.params(10_000, 1.0, kbar=10, seed=1))
        rhg.rhg_graph_free(g)
    finally:
        rhg.rhg_ctx_destroy(c)

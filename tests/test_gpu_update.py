"""GPU parity of the graph update after a move (dynamic model, Sec. III-C):
rhg_update_after_move keeps the edges between unmoved points and re-queries
the moved points in every slab and both directions.  Its edge list must be
the threshold graph of the moved coordinates exactly: the same edge set as
rhg_generate_from_coords on the same device arrays (the same bits of the same
distance test decide every pair) and as the oracle's band sweep on the table
the device used.  Cases: the paper's 12% of moved nodes, none, all, half,
hub-heavy alpha = 0.55, the FP32 filter, a ragged n, n = 10^6, and an old
list in shuffled order; the kept pairs come first, in their old order.
"""
import math

import numpy as np
import pytest

import parity
from paper_1606_09481_amd import rhg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    rhg.load()
    torch.cuda.set_device(0)
    c = rhg.rhg_ctx_create(0, torch.cuda.current_stream())
    yield c
    rhg.rhg_ctx_destroy(c)


def _dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    return (t if dtype is None else t.to(dtype)).cuda()


def _moved_state(orc, n, alpha, R, frac, seed):
    """Coordinates before and after a move of round(frac n) random nodes
    (steps of the paper's experiment; the others keep tau = 0)."""
    import torch
    th, r = orc.sample(n, alpha, R, seed)
    rng = np.random.default_rng(seed)
    k = int(round(frac * n))
    who = rng.choice(n, k, replace=False)
    tp = np.zeros(n)
    tr = np.zeros(n)
    tp[who] = rng.uniform(-1, 1, k)
    tr[who] = rng.uniform(-10, 1, k)
    dth, dr = _dev(th), _dev(r)
    dth1, dr1 = dth.clone(), dr.clone()
    return dth, dr, dth1, dr1, _dev(tp), _dev(tr), who


def _update_case(ctx, orc, n, alpha, kbar, frac, seed, prec=rhg.RHG_FP64, shuffle=False, oracle=True):
    import torch
    print("case", n, alpha, kbar, frac, seed, prec, shuffle, flush=True)
    R = orc.target_radius(n, alpha, kbar)
    dth, dr, dth1, dr1, dtp, dtr, who = _moved_state(orc, n, alpha, R, frac, seed)
    g0 = rhg.rhg_generate_from_coords(ctx, dth, dr, R)
    e0 = rhg.rhg_graph_copy_edges(g0)
    rhg.rhg_graph_free(g0)
    if shuffle:
        e0 = e0[np.random.default_rng(seed + 1).permutation(len(e0))]
    old = _dev(e0.reshape(-1))
    rhg.rhg_move(ctx, dth1, dr1, dtp, dtr, alpha, R)
    moved = torch.zeros(n, dtype=torch.uint8, device="cuda")
    if len(who):
        moved[_dev(who.astype(np.int64))] = 1
    torch.cuda.synchronize()
    g1 = rhg.rhg_update_after_move(ctx, dth1, dr1, R, moved, old, len(e0), prec)
    e1 = rhg.rhg_graph_copy_edges(g1)
    rhg.rhg_graph_free(g1)
    g2 = rhg.rhg_generate_from_coords(ctx, dth1, dr1, R, prec)
    e2 = rhg.rhg_graph_copy_edges(g2)
    th2, r2, tab, K = rhg.rhg_graph_copy_points(g2)
    rhg.rhg_graph_free(g2)
    parity.assert_valid(e1, n)
    parity.assert_same(e1, e2)
    # the kept pairs come first, in their old order
    mv = np.zeros(n, bool)
    mv[who] = True
    kept = e0[~(mv[e0[:, 0]] | mv[e0[:, 1]])]
    assert np.array_equal(e1[:len(kept)], kept)
    if oracle:
        parity.assert_same(e1, orc.band_sweep(th2, r2, tab, R, K))
    return len(e0), len(e1), len(kept)


@pytest.mark.parametrize("n,alpha,kbar,frac,seed", [(20_000, 1.0, 10.0, 0.12, 1), (20_000, 1.0, 10.0, 0.0, 2),
                                                   (20_000, 1.0, 10.0, 1.0, 3), (30_001, 1.5, 20.0, 0.5, 4),
                                                   (50_000, 0.55, 8.0, 0.12, 5), (4_097, 0.8, 30.0, 0.3, 6)])
def test_update_matches_generation_and_oracle(ctx, orc, n, alpha, kbar, frac, seed):
    m0, m1, mk = _update_case(ctx, orc, n, alpha, kbar, frac, seed)
    print("old %d, new %d, kept %d" % (m0, m1, mk), flush=True)


def test_update_fp32_filter_and_shuffled_old_list(ctx, orc):
    _update_case(ctx, orc, 40_000, 0.9, 16.0, 0.12, 7, prec=rhg.RHG_FP32_RECHECK, shuffle=True)


def test_update_1e6(ctx, orc):
    """n = 10^6, kbar = 20, the paper's 12%: the edge set of the regeneration
    (the unit order is sector-sorted at this size)."""
    _update_case(ctx, orc, 1_000_000, 1.0, 20.0, 0.12, 8, oracle=False)


def test_update_rejects_bad_pairs(ctx, orc):
    import torch
    n = 1000
    R = orc.target_radius(n, 1.0, 10.0)
    th, r = orc.sample(n, 1.0, R, 9)
    dth, dr = _dev(th), _dev(r)
    moved = torch.zeros(n, dtype=torch.uint8, device="cuda")
    bad = _dev(np.array([0, 1, 2, n], dtype=np.int32))  # the second pair names point n
    with pytest.raises(rhg.RhgError) as ei:
        rhg.rhg_update_after_move(ctx, dth, dr, R, moved, bad, 2)
    assert ei.value.status == rhg.RHG_EINVAL
    with pytest.raises(rhg.RhgError) as ei:
        rhg.rhg_update_after_move(ctx, dth, dr, R, moved, 0, 2)  # null list with pairs
    assert ei.value.status == rhg.RHG_EINVAL
    g = rhg.rhg_update_after_move(ctx, dth, dr, R, moved, 0, 0)  # no old edges, nothing moved: no edges
    assert rhg.rhg_graph_num_edges(g) == 0
    rhg.rhg_graph_free(g)


@pytest.mark.parametrize("n", [2, 3, 64, 65, 129])
def test_update_tiny_and_ragged(ctx, orc, n):
    """One or two batches, a ragged last batch: every case of half and all moved."""
    kbar = min(1.5, (n - 1) / 2.0)
    for frac, seed in ((0.5, 20 + n), (1.0, 40 + n)):
        _update_case(ctx, orc, n, 1.0, kbar, frac, seed)


def test_update_from_empty_old_list(ctx, orc):
    """No old edges and every point flagged: the update is a whole generation."""
    import torch
    n = 5_000
    R = orc.target_radius(n, 1.0, 10.0)
    th, r = orc.sample(n, 1.0, R, 31)
    dth, dr = _dev(th), _dev(r)
    moved = torch.ones(n, dtype=torch.uint8, device="cuda")
    g = rhg.rhg_update_after_move(ctx, dth, dr, R, moved, 0, 0)
    e = rhg.rhg_graph_copy_edges(g)
    rhg.rhg_graph_free(g)
    g2 = rhg.rhg_generate_from_coords(ctx, dth, dr, R)
    e2 = rhg.rhg_graph_copy_edges(g2)
    rhg.rhg_graph_free(g2)
    parity.assert_valid(e, n)
    parity.assert_same(e, e2)


def test_update_fp32_exhaustive_no_disagreement(ctx, orc):
    """The FP32 filter's self-check in update mode: no pair decided by the
    filter differs from the FP64 test."""
    rhg.rhg_ctx_set_option(ctx, rhg.RHG_OPT_FP32_EXHAUSTIVE, 1)
    try:
        n, alpha, kbar = 30_000, 0.8, 20.0
        R = orc.target_radius(n, alpha, kbar)
        import torch
        dth, dr, dth1, dr1, dtp, dtr, who = _moved_state(orc, n, alpha, R, 0.2, 50)
        g0 = rhg.rhg_generate_from_coords(ctx, dth, dr, R)
        m0 = rhg.rhg_graph_num_edges(g0)
        rhg.rhg_move(ctx, dth1, dr1, dtp, dtr, alpha, R)
        moved = torch.zeros(n, dtype=torch.uint8, device="cuda")
        moved[_dev(who.astype(np.int64))] = 1
        g1 = rhg.rhg_update_after_move(ctx, dth1, dr1, R, moved, rhg.rhg_graph_edges_device(g0), m0,
                                       rhg.RHG_FP32_RECHECK)
        st = rhg.rhg_graph_stats(g1)
        rhg.rhg_graph_free(g1)
        rhg.rhg_graph_free(g0)
        assert st["disagreements"] == 0 and st["candidates"] > 0
    finally:
        rhg.rhg_ctx_set_option(ctx, rhg.RHG_OPT_FP32_EXHAUSTIVE, 0)

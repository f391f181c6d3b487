"""Request server (rhg_server_*) on the GPU, through the C ABI.

* A mixed stream of requests -- small ones that share one-launch groups and
  large ones on the multi-launch path, both precisions, kbar- and R-given,
  non-default slab settings -- returns for every request exactly the bytes
  rhg_generate returns for the same parameters alone.
* One served small request against the all-pairs oracle on the table bits
  it used (identical edge sets).
* Admission: estimated memory in flight never exceeds the budget; a request
  larger than the whole budget still runs (alone).
* Ticket semantics: bounded waits, unknown and already-collected tickets.
"""
import math

import numpy as np
import pytest

import parity
from paper_1606_09481_amd import rhg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    rhg.load()
    c = rhg.rhg_ctx_create(0)
    yield c
    rhg.rhg_ctx_destroy(c)


def _edges(g):
    e = rhg.rhg_graph_copy_edges(g)
    st = rhg.rhg_graph_stats(g)
    rhg.rhg_graph_free(g)
    return e, st


def _mix(seed, count, n_lo=300, n_hi=65536, large=()):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        alpha = float(rng.uniform(0.55, 1.5))
        kbar = float(rng.integers(6, 65))
        if kbar > n / 8:
            continue
        try:
            R = rhg.rhg_target_radius(n, alpha, kbar)
        except rhg.RhgError:
            continue  # average degree out of reach for this (n, alpha): draw again
        prec = rhg.RHG_FP32_RECHECK if (len(out) % 3 == 1 and R <= 43) else rhg.RHG_FP64
        kind = len(out) % 5
        if kind == 2:
            p = rhg.params(n, alpha, R=R, seed=int(rng.integers(1, 2**63)), precision=prec)
        elif kind == 3:
            p = rhg.params(n, alpha, kbar=kbar, seed=int(rng.integers(1, 2**63)), precision=prec, num_bands=3,
                           band_ratio=1.0)
        else:
            p = rhg.params(n, alpha, kbar=kbar, seed=int(rng.integers(1, 2**63)), precision=prec)
        out.append(p)
    for (n, alpha, kbar, prec) in large:
        out.insert(len(out) // 2, rhg.params(n, alpha, kbar=kbar, seed=int(rng.integers(1, 2**63)), precision=prec))
    return out


def _describe(p):
    return "n=%d alpha=%.3f kbar=%.1f R=%.4f seed=%d prec=%d B=%d p=%.2f" % (
        p.n, p.alpha, p.kbar, p.R, p.seed, p.precision, p.num_bands, p.band_ratio)


def test_mix_equals_alone(ctx):
    reqs = _mix(11, 60, large=[(100_000, 0.8, 20, rhg.RHG_FP64), (250_000, 1.0, 10, rhg.RHG_FP32_RECHECK)])
    reqs.append(reqs[5])  # the same request twice in one mix
    srv = rhg.rhg_server_create(0, 4 << 30)
    try:
        tickets = [rhg.rhg_server_submit(srv, p) for p in reqs]
        served = []
        for t in tickets:
            g, lat = rhg.rhg_server_wait(srv, t)
            assert lat >= 0.0
            served.append(_edges(g))
        cnt = rhg.rhg_server_counters(srv)
    finally:
        rhg.rhg_server_destroy(srv)
    print("counters", cnt, flush=True)
    assert cnt["completed"] == len(reqs)
    assert cnt["batched"] >= len(reqs) - 4 and cnt["groups"] >= 1
    for p, (e, st) in zip(reqs, served):
        g = rhg.rhg_generate(ctx, p)
        ref, st_ref = _edges(g)
        assert e.shape == ref.shape, _describe(p)
        assert np.array_equal(e, ref), _describe(p)
        assert st["candidates"] == st_ref["candidates"] and st["windows"] == st_ref["windows"], _describe(p)
        assert st["rechecks"] == st_ref["rechecks"], _describe(p)
    assert np.array_equal(served[5][0], served[-1][0])


def test_served_small_request_vs_bruteforce(orc):
    n, alpha, kbar, seed = 6000, 0.9, 12, 5
    srv = rhg.rhg_server_create(0, 1 << 30)
    try:
        g, _ = rhg.rhg_server_wait(srv, rhg.rhg_server_submit(srv, rhg.params(n, alpha, kbar=kbar, seed=seed)))
        R = rhg.rhg_graph_radius(g)
        ref, (th, r, t, K) = parity.oracle_edges(orc, g, rhg, sweep=False)
        e, _ = _edges(g)
        cnt = rhg.rhg_server_counters(srv)
    finally:
        rhg.rhg_server_destroy(srv)
    assert cnt["batched"] == 1
    parity.assert_valid(e, n)
    parity.assert_same(e, ref)  # the all-pairs oracle on the table bits the served request used
    assert K == math.cosh(R)
    tho, _ = orc.sample(n, alpha, R, seed)
    assert np.array_equal(th, tho)
    parity.assert_table_close(orc, th, r, t)


def _est_bytes(n, kbar):
    return rhg.rhg_server_estimate_bytes(rhg.params(n, 1.0, kbar=kbar))


def test_admission_budget(ctx):
    budget = 24 << 20
    reqs = [p for p in _mix(12, 40, n_lo=4000, n_hi=16384) if p.R <= 0]
    assert len(reqs) >= 24 and max(rhg.rhg_server_estimate_bytes(p) for p in reqs) < budget
    srv = rhg.rhg_server_create(0, budget)
    try:
        tickets = [rhg.rhg_server_submit(srv, p) for p in reqs]
        out = [_edges(rhg.rhg_server_wait(srv, t)[0])[0] for t in tickets]
        cnt = rhg.rhg_server_counters(srv)
    finally:
        rhg.rhg_server_destroy(srv)
    print("counters", cnt, flush=True)
    assert cnt["peak_bytes"] <= budget
    assert cnt["completed"] == len(reqs)
    for p, e in zip(reqs[:8], out[:8]):
        ref, _ = _edges(rhg.rhg_generate(ctx, p))
        assert np.array_equal(e, ref), _describe(p)


def test_request_larger_than_budget_runs_alone(ctx):
    srv = rhg.rhg_server_create(0, 8 << 20)
    p_big = rhg.params(300_000, 1.0, kbar=10, seed=3)
    p_small = rhg.params(3000, 1.0, kbar=10, seed=4)
    try:
        t1 = rhg.rhg_server_submit(srv, p_big)
        t2 = rhg.rhg_server_submit(srv, p_small)
        e2, _ = _edges(rhg.rhg_server_wait(srv, t2)[0])
        e1, _ = _edges(rhg.rhg_server_wait(srv, t1)[0])
        cnt = rhg.rhg_server_counters(srv)
    finally:
        rhg.rhg_server_destroy(srv)
    assert cnt["completed"] == 2
    assert cnt["peak_bytes"] == max(_est_bytes(300_000, 10), _est_bytes(3000, 10))
    assert np.array_equal(e1, _edges(rhg.rhg_generate(ctx, p_big))[0])
    assert np.array_equal(e2, _edges(rhg.rhg_generate(ctx, p_small))[0])


def test_group_edges_of_sizes(ctx):
    """Requests at the sizes where batches and the group cutoff change (a few
    points, one batch and a point more, 65536 and 65537 points: the last
    grouped size and the first one that is not), submitted together: each
    equals rhg_generate alone."""
    reqs = [rhg.params(n, 1.0, R=4.0 + 0.5 * k, seed=100 + n) for k, n in enumerate((2, 3, 63, 64, 65, 127, 129))]
    reqs += [rhg.params(n, 0.9, kbar=12.0, seed=7 + n) for n in (65536, 65537)]
    srv = rhg.rhg_server_create(0, 4 << 30)
    try:
        tickets = [rhg.rhg_server_submit(srv, p) for p in reqs]
        served = [_edges(rhg.rhg_server_wait(srv, t)[0]) for t in tickets]
        cnt = rhg.rhg_server_counters(srv)
    finally:
        rhg.rhg_server_destroy(srv)
    print("counters", cnt, flush=True)
    assert cnt["completed"] == len(reqs) and cnt["batched"] >= len(reqs) - 1
    for p, (e, _) in zip(reqs, served):
        ref, _ = _edges(rhg.rhg_generate(ctx, p))
        assert e.shape == ref.shape and np.array_equal(e, ref), _describe(p)


def test_ticket_semantics():
    srv = rhg.rhg_server_create(0, 1 << 30)
    try:
        t = rhg.rhg_server_submit(srv, rhg.params(2_000_000, 0.75, kbar=40, seed=9))
        try:
            g, _ = rhg.rhg_server_wait(srv, t, 0)
        except rhg.RhgError as err:
            assert err.status == rhg.RHG_EBUSY
            g, _ = rhg.rhg_server_wait(srv, t, -1)
        assert rhg.rhg_graph_num_edges(g) > 0
        rhg.rhg_graph_free(g)
        with pytest.raises(rhg.RhgError) as ei:
            rhg.rhg_server_wait(srv, t, 0)  # already collected
        assert ei.value.status == rhg.RHG_EINVAL
        with pytest.raises(rhg.RhgError) as ei:
            rhg.rhg_server_wait(srv, 987654321, 0)
        assert ei.value.status == rhg.RHG_EINVAL
        with pytest.raises(rhg.RhgError) as ei:
            rhg.rhg_server_submit(srv, rhg.params(1, 1.0, kbar=10))
        assert ei.value.status == rhg.RHG_EINVAL
        # never collected: freed by destroy
        rhg.rhg_server_submit(srv, rhg.params(5000, 1.0, kbar=10, seed=1))
    finally:
        rhg.rhg_server_destroy(srv)

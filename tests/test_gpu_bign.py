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
from test_gpu_fullsize import _device_view

pytestmark = pytest.mark.gpu


def _incident_device(out, m, rows, n):
    """Canonical keys of the device edges touching `rows`, plus whole-output checks."""
    import torch
    flag = torch.zeros(n, dtype=torch.bool, device=out.device)
    flag[torch.as_tensor(rows, device=out.device)] = True
    sel = []
    chunk = 1 << 25
    for a in range(0, m, chunk):
        b = min(m, a + chunk)
        e = out[2 * a:2 * b].view(-1, 2).long()
        assert bool((e[:, 0] < e[:, 1]).all()), "lo < hi"
        assert int(e[:, 0].min()) >= 0 and int(e[:, 1].max()) < n, "indices in range"
        mk = flag[e[:, 0]] | flag[e[:, 1]]
        sel.append(e[mk].cpu())
    e = torch.cat(sel).numpy()
    k = (e[:, 0] << 32) | e[:, 1]
    ks = np.sort(k)
    assert np.all(ks[1:] != ks[:-1]), "each edge once"
    return ks


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


def _sorted_keys(g):
    """Sorted canonical keys lo * 2^32 + hi of a graph's edges, on the device."""
    import torch
    m = rhg.rhg_graph_num_edges(g)
    e = _device_view(rhg.rhg_graph_edges_device(g), 2 * m).view(-1, 2).long()
    assert bool((e[:, 0] < e[:, 1]).all()), "lo < hi"
    return torch.sort((e[:, 0] << 32) | e[:, 1]).values


def test_big_n_update_after_move():
    """n = 2^28 + 3 (64-bit table offsets) in update mode: the graph after a
    move of 12% of the nodes, updated from the graph before it, has exactly
    the edge set of its regeneration (sorted and compared on the device)."""
    import torch
    n, alpha, kbar = (1 << 28) + 3, 1.0, 4.0
    print("case update", n, alpha, kbar, flush=True)
    rhg.load()
    torch.cuda.set_device(0)
    c = rhg.rhg_ctx_create(0, torch.cuda.current_stream())
    try:
        R = rhg.rhg_target_radius(n, alpha, kbar)
        gen = torch.Generator(device="cuda").manual_seed(11)
        u = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen)
        th = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen) * (2 * math.pi)
        r = (2.0 * torch.asinh(torch.sqrt(u) * math.sinh(alpha * R / 2.0)) / alpha).clamp_(max=R)  # Eq. 1
        del u
        g0 = rhg.rhg_generate_from_coords(c, th, r, R)
        m0 = rhg.rhg_graph_num_edges(g0)
        sel = torch.rand(n, device="cuda", generator=gen) < 0.12
        tp = torch.where(sel, torch.rand(n, dtype=torch.float64, device="cuda", generator=gen) * 2 - 1, 0.0)
        tr = torch.where(sel, torch.rand(n, dtype=torch.float64, device="cuda", generator=gen) * 11 - 10, 0.0)
        rhg.rhg_move(c, th, r, tp, tr, alpha, R)
        del tp, tr
        moved = sel.to(torch.uint8)
        torch.cuda.synchronize()
        gu = rhg.rhg_update_after_move(c, th, r, R, moved, rhg.rhg_graph_edges_device(g0), m0)
        rhg.rhg_graph_free(g0)
        ku = _sorted_keys(gu)
        rhg.rhg_graph_free(gu)
        gr = rhg.rhg_generate_from_coords(c, th, r, R)
        kr = _sorted_keys(gr)
        rhg.rhg_graph_free(gr)
        print("edges before %d, after %d" % (m0, len(kr)), flush=True)
        assert len(ku) == len(kr) and bool(torch.equal(ku, kr))
        assert bool((ku[1:] != ku[:-1]).all()), "each edge once"
    finally:
        rhg.rhg_ctx_destroy(c)
        torch.cuda.empty_cache()

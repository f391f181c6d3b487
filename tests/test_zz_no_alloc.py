"""The allocation-free entry point rhg_generate_noalloc, through the C ABI.

Its output must be the bytes that rhg_count + rhg_emit (the entry point it is
a variant of) write for the same parameters, on two calls in a row on one
context, the second with a smaller n (the fixed scratch keeps the first
call's contents).  Nothing may be written past the m pairs; a buffer that is
too small gives RHG_ETRUNC with m reported and nothing written; n above the
limit is refused before any launch.
"""
import numpy as np
import pytest

from paper_1606_09481_amd import rhg

pytestmark = pytest.mark.gpu

SENTINEL = -7


@pytest.fixture(scope="module")
def ctx():
    import torch
    rhg.load()
    torch.cuda.set_device(0)
    c = rhg.rhg_ctx_create(0, torch.cuda.current_stream())
    yield c
    rhg.rhg_ctx_destroy(c)


def _count_emit(ctx, p):
    import torch
    plan, m = rhg.rhg_count(ctx, p)
    try:
        out = torch.empty(2 * m + 2, dtype=torch.int32, device="cuda")
        rhg.rhg_emit(ctx, plan, out, m)
        torch.cuda.synchronize()
    finally:
        rhg.rhg_graph_free(plan)
    return out[:2 * m].cpu().numpy(), m


def _noalloc(ctx, p, capacity):
    import torch
    out = torch.full((2 * capacity + 64,), SENTINEL, dtype=torch.int32, device="cuda")
    m = rhg.rhg_generate_noalloc(ctx, p, out, capacity)
    torch.cuda.synchronize()
    host = out.cpu().numpy()
    assert np.all(host[2 * m:] == SENTINEL), "written past the m pairs"
    return host[:2 * m], m


def _describe(p):
    return "n=%d alpha=%.2f kbar=%.1f seed=%d prec=%d B=%d" % (p.n, p.alpha, p.kbar, p.seed, p.precision,
                                                                p.num_bands)


SEQUENCES = [
    # (first call, second call with a smaller n)
    (rhg.params(8192, 1.0, kbar=10.0, seed=3), rhg.params(3001, 0.75, kbar=20.0, seed=4,
                                                          precision=rhg.RHG_FP32_RECHECK)),
    (rhg.params(6000, 0.6, kbar=30.0, seed=5, precision=rhg.RHG_FP32_RECHECK, num_bands=32),
     rhg.params(129, 1.5, kbar=6.0, seed=6)),
    (rhg.params(4097, 0.55, kbar=64.0, seed=7, num_bands=3, band_ratio=1.0), rhg.params(2, 1.0, R=5.0, seed=8)),
]


@pytest.mark.parametrize("first,second", SEQUENCES)
def test_noalloc_equals_count_emit(ctx, first, second):
    for p in (first, second):
        print("noalloc", _describe(p), flush=True)
        ref, m_ref = _count_emit(ctx, p)
        got, m = _noalloc(ctx, p, m_ref + 100)
        assert m == m_ref, _describe(p)
        assert np.array_equal(got, ref), _describe(p)
        assert m == 0 or (got.reshape(-1, 2)[:, 0] < got.reshape(-1, 2)[:, 1]).all()


def test_noalloc_exact_capacity_and_truncation(ctx):
    import torch
    p = rhg.params(5000, 0.9, kbar=12.0, seed=9)
    ref, m_ref = _count_emit(ctx, p)
    got, m = _noalloc(ctx, p, m_ref)  # exactly m pairs of room
    assert m == m_ref and np.array_equal(got, ref)
    out = torch.full((2 * m_ref,), SENTINEL, dtype=torch.int32, device="cuda")
    with pytest.raises(rhg.RhgError) as e:
        rhg.rhg_generate_noalloc(ctx, p, out, m_ref - 1)
    assert e.value.status == rhg.RHG_ETRUNC and e.value.m == m_ref
    torch.cuda.synchronize()
    assert bool((out == SENTINEL).all()), "RHG_ETRUNC must leave the buffer untouched"
    # a later call is unaffected by the truncated one
    got2, m2 = _noalloc(ctx, p, m_ref + 1)
    assert m2 == m_ref and np.array_equal(got2, ref)


def test_noalloc_refuses_beyond_limit(ctx):
    import torch
    out = torch.full((16,), SENTINEL, dtype=torch.int32, device="cuda")
    with pytest.raises(rhg.RhgError) as e:
        rhg.rhg_generate_noalloc(ctx, rhg.params(8193, 1.0, kbar=10.0), out, 8)
    assert e.value.status == rhg.RHG_ERANGE
    with pytest.raises(rhg.RhgError) as e:
        rhg.rhg_generate_noalloc(ctx, rhg.params(1000, 1.0, R=400.0), out, 8)
    assert e.value.status == rhg.RHG_EINVAL
    torch.cuda.synchronize()
    assert bool((out == SENTINEL).all())

"""The literal-Eq. 3 FP32 ablation option (RHG_OPT_LITERAL_ABLATION).

With the option on, the FP32-filter count pass also decides every candidate
by Eq. 3 as printed, in FP32.  The edges stay those of the FP64 test (the
option only counts); the counters are consistent (undecided and wrong at most
the candidates), and they show what the cancellation-free form avoids: the
printed form in FP32 leaves a large share of the candidates undecided and
gets a share of its decisions wrong, where the filter used leaves about one
in a million.
"""
import pytest

from paper_1606_09481_amd import rhg

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,alpha,kbar", [(200_000, 1.0, 20.0), (100_000, 0.55, 16.0)])
def test_literal_ablation_counts(n, alpha, kbar):
    rhg.load()
    c = rhg.rhg_ctx_create(0)
    try:
        p = rhg.params(n, alpha, kbar=kbar, seed=2, precision=rhg.RHG_FP32_RECHECK)
        g = rhg.rhg_generate(c, p)
        ref = rhg.rhg_graph_copy_edges(g)
        st0 = rhg.rhg_graph_stats(g)
        rhg.rhg_graph_free(g)
        rhg.rhg_ctx_set_option(c, rhg.RHG_OPT_LITERAL_ABLATION, 1)
        g = rhg.rhg_generate(c, p)
        got = rhg.rhg_graph_copy_edges(g)
        st = rhg.rhg_graph_stats(g)
        rhg.rhg_graph_free(g)
    finally:
        rhg.rhg_ctx_destroy(c)
    assert (got == ref).all() and got.shape == ref.shape
    assert st0["literal_undecided"] == 0 and st0["literal_wrong"] == 0
    cand = st["candidates"]
    print("candidates %d, filter rechecks %d, literal undecided %d, literal wrong %d" % (
        cand, st["rechecks"], st["literal_undecided"], st["literal_wrong"]), flush=True)
    assert st["disagreements"] == 0
    assert st["literal_undecided"] <= cand and st["literal_wrong"] <= cand
    assert st["literal_undecided"] > 0.05 * cand
    assert st["literal_wrong"] > 1000 * max(1, st["rechecks"]) or st["literal_wrong"] > 0.01 * cand

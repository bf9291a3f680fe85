"""The allocation-free entry point (amlm_mine_static) against amlm_mine,
through the C ABI: two calls in a row on one GPU, the second on a smaller
graph, both bit-identical to amlm_mine; graphs above the static scratch are
rejected before any device work."""
import numpy as np
import pytest

import paper_2604_12241_amd as A
from paper_2604_12241_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pair(g, p, G=None):
    own = G is None
    if own:
        G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    ref = A.to_u32(A.amlm_mine(G, p))
    A.amlm_graph_sync(G)
    got = A.to_u32(A.amlm_mine_static(G, p))
    A.amlm_graph_sync(G)
    if own:
        G.close()
    return ref, got


def test_static_scratch_equals_amlm_mine_two_calls():
    big = W.mid(211, scale=0.1)          # 500k edges: most of the 64 MiB scratch
    small = W.tiny(101)                  # 20k edges, afterwards: the array keeps the last call's contents
    for g, (d, L, k) in ((big, (86400, 6, 2)), (small, (86400, 4, 3))):
        for pats in (A.AMLM_ALL, A.AMLM_ALL | A.AMLM_SG_UNORDERED, A.AMLM_SG | A.AMLM_CYCLES):
            ref, got = _pair(g, A.params(pats, d, L, k))
            np.testing.assert_array_equal(got, ref)
            assert ref.any()


def test_static_scratch_learned_schedule():
    g = W.mid(212, scale=0.02)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    A.amlm_costmodel_train([G], [A.params(A.AMLM_ALL, 86400, 6, 2)], epochs=1, batch=512, seed=9)
    A.amlm_tune_set(G, split_bytes=512)   # force sliced anchors
    ref, got = _pair(g, A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_LEARNED), G)
    np.testing.assert_array_equal(got, ref)
    G.close()


def test_static_scratch_rejects_large_graphs():
    g = W.mid(213, scale=0.25)           # 1.25M edges: above the static scratch
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    with pytest.raises(A.AmlmError) as ei:
        A.amlm_mine_static(G, A.params(A.AMLM_ALL, 86400, 6, 2))
    assert ei.value.status == 3
    # the handle is still usable
    c = A.amlm_mine(G, A.params(A.AMLM_FAN_OUT, 86400, 6, 2))
    A.amlm_graph_sync(G)
    assert A.to_u32(c).any()
    G.close()

"""Parity at the workloads' full sizes (the oracle runs as a pool of
processes over disjoint anchor ranges or independent graphs):

* the 5M-edge graph (500k accounts, 16 days, delta 24 h, L 6, k 2), every
  column of every edge, static and learned schedules, with the
  participation and size columns, and with the phase-ordered scatter-gather
  and any-order cycles;
* the 256 independent sub-graphs of 1k-200k edges (9.8M edges, windows of
  6 / 24 / 72 h) through one captured batched launch, every sub-graph;
* serving over the 32M-edge resident graph: every 10th of 60 stream batches
  (1k-100k edges each), its own rows and its cycle credits to older edges,
  against the oracle's mining of exactly that batch's anchors.

The 32M-edge graph itself is compared in full by the benchmark (its
parity record).
"""
import numpy as np
import pytest

import oracle
import paper_2604_12241_amd as A
from oracle.parallel import mine_many, mine_parallel, mine_ranges
from paper_2604_12241_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_mid_5M_full_graph_both_schedules():
    g = W.mid(202)
    ref, _ = mine_parallel(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, 86400, 6, 2)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL, 86400, 6, 2)))
    A.amlm_graph_sync(G)
    bad = int((c != ref).sum())
    assert bad == 0, f"{bad} mismatching counts (static)"
    A.amlm_costmodel_train([G], [A.params(A.AMLM_ALL, 86400, 6, 2)], epochs=1, batch=4096, seed=2)
    c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_LEARNED)))
    A.amlm_graph_sync(G)
    bad = int((c != ref).sum())
    assert bad == 0, f"{bad} mismatching counts (learned)"
    G.close()


def test_mid_5M_full_graph_instance_columns():
    """Participation (SG_PART, GS_PART) and the SG size bins beside every
    other column on the 5M-edge graph: all 15 columns of every edge."""
    g = W.mid(206)
    pats = oracle.ALL | oracle.PART | oracle.SG_SIZES
    ref, _ = mine_parallel(g.src, g.dst, g.ts, g.n_vertices, pats, 86400, 6, 2)
    assert ref[-6:].sum() > 0
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL | A.AMLM_PART | A.AMLM_SG_SIZES, 86400, 6, 2)))
    A.amlm_graph_sync(G)
    G.close()
    bad = int((c != ref).sum())
    assert bad == 0, f"{bad} mismatching counts"


@pytest.mark.parametrize("k", [2, 3])
def test_mid_5M_full_graph_phase_order_and_any_order_cycles(k):
    """The phase-ordered scatter-gather and any-order cycles beside every
    other column on the 5M-edge graph, every edge."""
    g = W.mid(206)
    ref, _ = mine_parallel(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL | oracle.SG_PHASE | oracle.CYC_ANY_ORDER,
                           86400, 4, k)
    assert ref[2].sum() > 0
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL | A.AMLM_SG_PHASE | A.AMLM_CYC_ANY_ORDER, 86400, 4, k)))
    A.amlm_graph_sync(G)
    G.close()
    bad = int((c != ref).sum())
    assert bad == 0, f"{bad} mismatching counts"


def test_all_256_subgraphs_in_one_captured_launch():
    subs = W.batch_subgraphs(256)
    refs = mine_many([(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs],
                     [(oracle.ALL, d, 6, 2) for _, d in subs])
    B = A.Batch([(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs])
    ps = [A.params(A.AMLM_ALL, d, 6, 2) for _, d in subs]
    for rep in range(2):
        outs = A.amlm_mine_batch(B, ps)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            bad = int((A.to_u32(o) != r).sum())
            assert bad == 0, f"replay {rep}, sub-graph {i} ({subs[i][0].n_edges} edges): {bad} mismatches"
    assert B.info_batch() == (256, 1)
    B.close()


def test_serving_over_the_32M_graph_sampled_batches():
    d, L, k = 86400, 6, 2
    base = W.large(404)
    batches = W.stream_batches(base, seed=505, n_batches=60)
    R = A.Graph(base.src, base.dst, base.ts, base.n_vertices)
    S = A.Server(R, A.params(A.AMLM_ALL, d, L, k), max_slots=4)
    res = []
    for i in range(0, len(batches), 12):
        tk = [S.submit(b.src, b.dst, b.ts) for b in batches[i:i + 12]]
        res += [S.wait(t) for t in tk]
    S.close()
    R.close()
    # the union graph in submission order; batch b's anchors are its ids
    src = np.concatenate([base.src] + [b.src for b in batches])
    dst = np.concatenate([base.dst] + [b.dst for b in batches])
    ts = np.concatenate([base.ts] + [b.ts for b in batches])
    offs = np.cumsum([base.n_edges] + [b.n_edges for b in batches])
    sample = list(range(0, len(batches), 10))
    ranges = [(int(offs[b]), int(offs[b + 1])) for b in sample]
    del base
    refs = mine_ranges(src, dst, ts, int(max(src.max(), dst.max())) + 1, oracle.ALL, d, L, k, ranges)
    ncyc = L - 1
    for b, (lo, hi), (own, cyc) in zip(sample, ranges, refs):
        c, (de, dc, dv), nd = res[b]
        np.testing.assert_array_equal(c, own, err_msg=f"batch {b} rows")
        # deltas: credits to edges before the batch, as (edge id, column, value)
        e_ref, c_ref, v_ref = [], [], []
        for j in range(ncyc):
            idx, val = cyc[j]
            m = idx < lo
            e_ref.append(idx[m].astype(np.uint64))
            c_ref.append(np.full(int(m.sum()), 4 + j, np.uint32))
            v_ref.append(val[m])
        e_ref, c_ref, v_ref = np.concatenate(e_ref), np.concatenate(c_ref), np.concatenate(v_ref)
        order = np.lexsort((c_ref, e_ref))
        assert nd == e_ref.shape[0], f"batch {b}: {nd} deltas, oracle {e_ref.shape[0]}"
        np.testing.assert_array_equal(de, e_ref[order])
        np.testing.assert_array_equal(dc, c_ref[order])
        np.testing.assert_array_equal(dv, v_ref[order])

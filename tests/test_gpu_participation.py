"""GPU parity of the instance columns against the oracle: participation
(AMLM_PART: for every edge, the scatter-gather and gather-scatter instances
it belongs to) and the scatter-gather size bins (AMLM_SG_SIZES).  Random
small graphs with ties and self-loops, a 100k-edge graph with hubs, ordered
and unordered legs, k from 1 to 4, the saturation ceiling, the
allocation-free entry point, a sliced schedule, batched stores with mixed
parameters, and the streaming server, whose new anchors credit older edges
through deltas."""
import numpy as np
import pytest

import oracle
import paper_2604_12241_amd as A
from paper_2604_12241_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PART = (A.AMLM_PART, oracle.PART)
SIZES = (A.AMLM_SG_SIZES, oracle.SG_SIZES)


def _mine(g, pat, delta, L, k, sched=A.AMLM_SCHED_STATIC, ceiling=0):
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    if ceiling:
        A.amlm_graph_set_ceiling(G, ceiling)
    c = A.to_u32(A.amlm_mine(G, A.params(pat, delta, L, k, sched)))
    A.amlm_graph_sync(G)
    G.close()
    return c


@pytest.mark.parametrize("seed", range(12))
def test_participation_random_small(seed):
    rng = np.random.default_rng(9100 + seed)
    g = W.random_small(seed + 910, n_edges=int(rng.integers(1, 500)), n_vertices=int(rng.integers(2, 20)),
                       t_range=int(rng.integers(1, 60)))
    delta, L, k = int(rng.integers(0, 50)), int(rng.integers(2, 7)), int(rng.integers(1, 5))
    print(f"seed {seed}: {g.n_edges} edges, delta {delta}, L {L}, k {k}", flush=True)
    for pat, opat in ((A.AMLM_ALL | PART[0], oracle.ALL | PART[1]),
                      (A.AMLM_ALL | A.AMLM_SG_UNORDERED | PART[0], oracle.ALL | oracle.SG_UNORDERED | PART[1]),
                      (A.AMLM_SG | PART[0], oracle.SG | PART[1]),
                      (A.AMLM_GS | A.AMLM_DEG_IN | PART[0], oracle.GS | oracle.DEG_IN | PART[1]),
                      (A.AMLM_SG | SIZES[0], oracle.SG | SIZES[1]),
                      (A.AMLM_ALL | A.AMLM_SG_UNORDERED | PART[0] | SIZES[0],
                       oracle.ALL | oracle.SG_UNORDERED | PART[1] | SIZES[1])):
        c = _mine(g, pat, delta, L, k)
        ref = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, opat, delta, L, k)
        np.testing.assert_array_equal(c, ref, err_msg=f"pattern {pat}")


@pytest.mark.parametrize("k", [1, 2, 4])
def test_participation_mid_with_hubs(k):
    """100k edges with hub accounts: many senders per anchor, long
    out-windows (several 64-entry wave steps per sender) and parallel
    edges; the columns before the participation columns are unchanged."""
    g = W.mid(215, scale=0.02)
    for pat, opat in ((A.AMLM_ALL | PART[0], oracle.ALL | PART[1]),
                      (A.AMLM_ALL | A.AMLM_SG_UNORDERED | PART[0], oracle.ALL | oracle.SG_UNORDERED | PART[1])):
        c = _mine(g, pat, 86400, 5, k)
        ref = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, opat, 86400, 5, k)
        np.testing.assert_array_equal(c, ref, err_msg=f"pattern {pat}")
        assert ref[-2].sum() > 0 and ref[-1].sum() > 0
        np.testing.assert_array_equal(c[:-2], _mine(g, pat & ~A.AMLM_PART, 86400, 5, k))
    c = _mine(g, A.AMLM_ALL | SIZES[0], 86400, 5, k)
    ref = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL | SIZES[1], 86400, 5, k)
    np.testing.assert_array_equal(c, ref)
    np.testing.assert_array_equal(c[-4:].sum(axis=0), c[2])


@pytest.mark.parametrize("ceiling", [1, 3, 40])
def test_participation_saturates(ceiling):
    g = W.mid(216, scale=0.004)
    c = _mine(g, A.AMLM_ALL | PART[0] | SIZES[0], 86400, 4, 1, ceiling=ceiling)
    ref, _, _ = oracle.mine_ex(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL | PART[1] | SIZES[1], 86400, 4, 1,
                               ceiling=ceiling)
    np.testing.assert_array_equal(c, ref)
    assert (ref[-5] == ceiling).any()


def test_participation_static_entry_and_sliced_schedule():
    """amlm_mine_static (scratch in the library's device array) and a sliced
    schedule (given per-edge costs, small slices) give the same columns."""
    g = W.mid(217, scale=0.01)
    p = A.params(A.AMLM_ALL | PART[0], 86400, 5, 2)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    a = A.to_u32(A.amlm_mine(G, p))
    b = A.to_u32(A.amlm_mine_static(G, p))
    np.testing.assert_array_equal(a, b)
    ref = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL | PART[1], 86400, 5, 2)
    np.testing.assert_array_equal(a, ref)
    cost = torch.full((g.n_edges,), 12.0, dtype=torch.float32, device="cuda")
    A.amlm_graph_set_costs(G, cost)
    A.amlm_tune_set(G, split_bytes=512)
    c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL | PART[0], 86400, 5, 2, A.AMLM_SCHED_GIVEN)))
    A.amlm_graph_sync(G)
    np.testing.assert_array_equal(c, ref)
    A.amlm_graph_set_costs(G, None)
    G.close()


def test_instance_columns_edge_cases():
    """Empty graph, only self-loops, one edge, equal timestamps everywhere
    with many parallel edges (zero and short windows), and a window that
    spans almost the whole relative-time range."""
    T0 = W.T0
    pat = A.AMLM_ALL | A.AMLM_DEG_OUT | PART[0] | SIZES[0]
    opat = oracle.ALL | oracle.DEG_OUT | PART[1] | SIZES[1]
    ncols = A.amlm_num_columns(A.params(pat, 10, 4, 2))
    e = W.EdgeList(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.int64),
                   np.zeros(0, np.float32), 5)
    assert _mine(e, pat, 10, 4, 2).shape == (ncols, 0)
    s = W.EdgeList(np.array([1, 2, 2], np.uint32), np.array([1, 2, 2], np.uint32),
                   np.array([T0, T0, T0 + 1], np.int64), np.zeros(3, np.float32), 3)
    assert _mine(s, pat, 10, 4, 2).sum() == 0
    one = W.EdgeList(np.array([0], np.uint32), np.array([1], np.uint32), np.array([T0], np.int64),
                     np.zeros(1, np.float32), 2)
    np.testing.assert_array_equal(_mine(one, pat, 0, 2, 1),
                                  oracle.mine(one.src, one.dst, one.ts, 2, opat, 0, 2, 1))
    rng = np.random.default_rng(4)
    par = W.EdgeList(rng.integers(0, 4, 300).astype(np.uint32), rng.integers(0, 4, 300).astype(np.uint32),
                     np.full(300, T0, np.int64), np.zeros(300, np.float32), 4)
    few = W.EdgeList(par.src, par.dst, T0 + rng.integers(0, 3, 300).astype(np.int64), par.amount, 4)
    for g, d, k in ((par, 0, 1), (par, 5, 2), (few, 0, 1), (few, 1, 2), (few, 5, 1)):
        ref = oracle.mine(g.src, g.dst, g.ts, 4, opat, d, 4, k)
        np.testing.assert_array_equal(_mine(g, pat, d, 4, k), ref, err_msg=f"ties d{d} k{k}")
    assert ref[-6:].sum() > 0   # three distinct times: instances exist
    big = W.random_small(9, n_edges=200, n_vertices=6, t_range=20)
    big.ts[::7] += 2**31 - 100
    for d in (2**31, 10):
        np.testing.assert_array_equal(_mine(big, pat, d, 4, 2),
                                      oracle.mine(big.src, big.dst, big.ts, 6, opat, d, 4, 2), err_msg=f"span d{d}")


def test_participation_errors():
    g = W.random_small(3, n_edges=50, n_vertices=6, t_range=20)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    for pat in (A.AMLM_FAN_OUT | A.AMLM_CYCLES | A.AMLM_PART, A.AMLM_SG | A.AMLM_SG_PHASE | A.AMLM_PART,
                A.AMLM_GS | A.AMLM_SG_SIZES):
        assert A.amlm_num_columns(A.params(pat, 10, 4, 2)) == 0
        with pytest.raises(A.AmlmError) as ei:
            A.amlm_mine(G, A.params(pat, 10, 4, 2), torch.zeros((1, g.n_edges), dtype=torch.int32, device="cuda"))
        assert ei.value.status == 1
    G.close()


def test_instance_columns_in_a_batch_with_mixed_parameters():
    """Batched stores: every sub-graph with its own window, threshold and
    cycle length, through one captured launch (replayed), each sub-graph's
    columns against the oracle on that sub-graph."""
    rng = np.random.default_rng(17)
    subs = []
    for i in range(6):
        e = int(rng.integers(100, 4000))
        g = W.power_law(870 + i, max(20, e // 8), e, 4, 2.1, max(20.0, e / 50), delta_s=86400)
        subs.append((g, int(rng.choice([3600, 86400])), int(rng.integers(2, 7)), int(rng.integers(1, 4))))
    B = A.Batch([(g.src, g.dst, g.ts, g.n_vertices) for g, _, _, _ in subs])
    pats = A.AMLM_ALL | A.AMLM_DEG_IN | A.AMLM_PART | A.AMLM_SG_SIZES
    ps = [A.params(pats, d, L, k) for _, d, L, k in subs]
    for rep in range(2):
        outs = A.amlm_mine_batch(B, ps)
        torch.cuda.synchronize()
        for (g, d, L, k), o in zip(subs, outs):
            ref = oracle.mine(g.src, g.dst, g.ts, g.n_vertices,
                              oracle.ALL | oracle.DEG_IN | oracle.PART | oracle.SG_SIZES, d, L, k)
            np.testing.assert_array_equal(A.to_u32(o), ref, err_msg=f"replay {rep}, delta {d}, L {L}, k {k}")
    B.close()


def test_participation_through_the_server():
    """Each batch's anchors credit the edges of their instances, older ones
    included (deltas): resident counts + new rows + deltas equal the oracle
    on the union graph."""
    D, L, K = 86400, 4, 2
    base = W.mid(321, scale=0.004)
    batches = W.stream_batches(base, seed=78, n_batches=10, b_min=50, b_max=2500, rate_per_s=0.02,
                               zipf_a=2.1, max_degree=50)
    pats = A.AMLM_ALL | A.AMLM_DEG_IN | A.AMLM_PART | A.AMLM_SG_SIZES
    p = A.params(pats, D, L, K)
    R = A.Graph(base.src, base.dst, base.ts, base.n_vertices)
    r_counts = A.to_u32(A.amlm_mine(R, p)).astype(np.uint64)
    S = A.Server(R, p, max_slots=4)
    tickets = [S.submit(b.src, b.dst, b.ts) for b in batches]
    res = [S.wait(t) for t in tickets]
    S.close()
    src = np.concatenate([base.src] + [b.src for b in batches])
    dst = np.concatenate([base.dst] + [b.dst for b in batches])
    ts = np.concatenate([base.ts] + [b.ts for b in batches])
    acc = np.zeros((r_counts.shape[0], src.shape[0]), np.uint64)
    acc[:, :base.n_edges] = r_counts
    pos = base.n_edges
    ncol = r_counts.shape[0]
    part_deltas = 0
    for (c, (de, dc, dv), _), b in zip(res, batches):
        acc[:, pos:pos + b.n_edges] += c
        np.add.at(acc, (dc.astype(np.int64), de.astype(np.int64)), dv)
        assert (de < pos).all()
        part_deltas += int(((dc >= ncol - 6) & (dc < ncol - 4)).sum())
        assert (dc < ncol - 4).all()     # the size bins are the anchor's own
        pos += b.n_edges
    full = oracle.mine(src, dst, ts, base.n_vertices, oracle.ALL | oracle.DEG_IN | oracle.PART | oracle.SG_SIZES,
                       D, L, K)
    np.testing.assert_array_equal(acc, full.astype(np.uint64))
    assert part_deltas > 0
    R.close()

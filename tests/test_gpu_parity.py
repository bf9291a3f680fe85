"""GPU parity: the HIP library against the CPU oracle, bit-exact.

Every count is an integer, so every comparison is exact equality.  Small
graphs are compared on every edge; the full-size workloads are compared on
sampled edges that the oracle computes one by one (cycle columns by an
independent through-edge enumeration).
"""
import numpy as np
import pytest

import oracle
import paper_2604_12241_amd as A
from paper_2604_12241_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def gpu_mine(g, delta, L, k, patterns=A.AMLM_ALL, schedule=A.AMLM_SCHED_STATIC, on_device=False):
    if on_device:
        src = torch.from_numpy(g.src.view(np.int32)).cuda()
        dst = torch.from_numpy(g.dst.view(np.int32)).cuda()
        ts = torch.from_numpy(g.ts).cuda()
        G = A.Graph(src, dst, ts, g.n_vertices)
    else:
        G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    p = A.params(patterns, delta, L, k, schedule)
    c = A.amlm_mine(G, p)
    A.amlm_graph_sync(G)
    out = A.to_u32(c)
    G.close()
    return out


def oracle_mine(g, delta, L, k, patterns=oracle.ALL):
    return oracle.mine(g.src, g.dst, g.ts, g.n_vertices, patterns, delta, L, k)


def assert_same(gpu, ref, what=""):
    if not np.array_equal(gpu, ref):
        bad = np.argwhere(gpu != ref)
        c, i = bad[0]
        raise AssertionError(f"{what}: {bad.shape[0]} mismatches, first col {c} edge {i}: "
                             f"gpu {gpu[c, i]} oracle {ref[c, i]}")


@pytest.mark.parametrize("seed", range(12))
def test_random_small_dense(seed):
    rng = np.random.default_rng(500 + seed)
    g = W.random_small(seed, n_edges=int(rng.integers(30, 400)), n_vertices=int(rng.integers(3, 20)),
                       t_range=int(rng.integers(5, 80)))
    for (delta, L, k) in [(int(rng.integers(0, 60)), int(rng.integers(2, 9)), int(rng.integers(1, 5))),
                          (30, 5, 2), (1000, 8, 1)]:
        assert_same(gpu_mine(g, delta, L, k), oracle_mine(g, delta, L, k), f"seed {seed} d{delta} L{L} k{k}")


def test_tiny_workload_and_permutation():
    g = W.tiny(101)
    ref = oracle_mine(g, 86400, 4, 3)
    assert_same(gpu_mine(g, 86400, 4, 3), ref, "tiny")
    gp, perm = W.permute(g, 5)
    assert_same(gpu_mine(gp, 86400, 4, 3, on_device=True), ref[:, perm], "tiny permuted")


@pytest.mark.parametrize("scale,L,k", [(0.02, 6, 2), (0.01, 8, 1), (0.01, 3, 4)])
def test_mid_scaled_full(scale, L, k):
    g = W.mid(202, scale=scale)
    assert_same(gpu_mine(g, 86400, L, k), oracle_mine(g, 86400, L, k), f"mid scale {scale}")


def test_pattern_subsets():
    g = W.mid(203, scale=0.005)
    full = oracle_mine(g, 86400, 5, 2)
    cols = {A.AMLM_FAN_OUT: [0], A.AMLM_FAN_IN: [1], A.AMLM_SG: [2], A.AMLM_GS: [3],
            A.AMLM_CYCLES: [4, 5, 6, 7]}
    for pat in [A.AMLM_FAN_OUT, A.AMLM_GS, A.AMLM_SG | A.AMLM_CYCLES, A.AMLM_FAN_IN | A.AMLM_GS]:
        want = sorted(c for b, cs in cols.items() if pat & b for c in cs)
        assert_same(gpu_mine(g, 86400, 5, 2, patterns=pat), full[want], f"patterns {pat}")


def test_edge_cases():
    T0 = W.T0
    # empty graph
    e = W.EdgeList(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.int64),
                   np.zeros(0, np.float32), 5)
    assert gpu_mine(e, 10, 4, 2).shape == (7, 0)
    # only self-loops
    s = W.EdgeList(np.array([1, 2, 2], np.uint32), np.array([1, 2, 2], np.uint32),
                   np.array([T0, T0, T0 + 1], np.int64), np.zeros(3, np.float32), 3)
    assert gpu_mine(s, 10, 4, 2).sum() == 0
    # single edge, one vertex pair
    one = W.EdgeList(np.array([0], np.uint32), np.array([1], np.uint32), np.array([T0], np.int64),
                     np.zeros(1, np.float32), 2)
    assert_same(gpu_mine(one, 0, 2, 1), oracle_mine(one, 0, 2, 1), "single")
    # zero window, equal timestamps everywhere, many parallel edges
    rng = np.random.default_rng(4)
    par = W.EdgeList(rng.integers(0, 3, 300).astype(np.uint32), rng.integers(0, 3, 300).astype(np.uint32),
                     np.full(300, T0, np.int64), np.zeros(300, np.float32), 3)
    for d in (0, 5):
        assert_same(gpu_mine(par, d, 6, 2), oracle_mine(par, d, 6, 2), f"ties d{d}")
    # timestamps spanning almost the whole int32 range of relative time
    big = W.random_small(9, n_edges=200, n_vertices=6, t_range=20)
    big.ts[::7] += 2**31 - 100
    assert_same(gpu_mine(big, 2**31, 5, 2), oracle_mine(big, 2**31, 5, 2), "large span")
    assert_same(gpu_mine(big, 10, 5, 2), oracle_mine(big, 10, 5, 2), "large span, small window")


def test_errors():
    T0 = W.T0
    with pytest.raises(A.AmlmError) as ei:
        A.Graph(np.array([0, 5], np.uint32), np.array([1, 0], np.uint32), np.array([T0, T0], np.int64), 3)
    assert ei.value.status == 1
    with pytest.raises(A.AmlmError) as ei:
        A.Graph(np.array([0, 1], np.uint32), np.array([1, 0], np.uint32), np.array([0, 2**31], np.int64), 3)
    assert ei.value.status == 2
    G = A.Graph(np.array([0, 1], np.uint32), np.array([1, 0], np.uint32), np.array([T0, T0 + 1], np.int64), 2)
    for bad in (A.params(L=1), A.params(L=9), A.params(k=0), A.params(delta=-5), A.params(patterns=0)):
        with pytest.raises(A.AmlmError) as ei:
            A.amlm_mine(G, bad, counts=torch.zeros((9, 2), dtype=torch.int32, device="cuda"))
        assert ei.value.status == 1
    G.close()


def test_hub_heavy_cycles_deep_frames():
    """A hub with thousands of window out-edges and dense returns: search
    trees far wider than one 64-path frame, so every frame is refilled many
    times and the depth-first stack runs to its last frame."""
    rng = np.random.default_rng(11)
    n = 6000
    nv = 40
    src = rng.integers(0, nv, n).astype(np.uint32)
    dst = rng.integers(0, nv, n).astype(np.uint32)
    ts = W.T0 + rng.integers(0, 4000, n).astype(np.int64)
    g = W.EdgeList(src, dst, ts, np.zeros(n, np.float32), nv)
    assert_same(gpu_mine(g, 400, 5, 3), oracle_mine(g, 400, 5, 3), "dense hub")


def _heavy_sender_graph(seed, n_senders=300, n_anchors=6, n_noise=4000):
    """Anchors u -> v whose sender windows hold hundreds of senders, each with
    its own out-edges to shared intermediates that reach v: the scatter-gather
    stage cuts these anchors into slices."""
    rng = np.random.default_rng(seed)
    u, v = 0, 1
    senders = np.arange(2, 2 + n_senders)
    mids = np.arange(2 + n_senders, 2 + n_senders + 24)
    nv = int(mids[-1]) + 40
    src, dst, ts = [], [], []
    def add(a, b, t):
        src.append(a); dst.append(b); ts.append(t)
    for i, s_ in enumerate(senders):
        for m in rng.choice(mids, size=int(rng.integers(0, 4)), replace=False):
            add(s_, m, 100 + int(rng.integers(0, 400)))
        add(s_, u, 600 + int(rng.integers(0, 300)))
        if i % 7 == 0:
            add(s_, u, 950 + int(rng.integers(0, 40)))  # repeated sender edges
    for m in mids:
        for _ in range(int(rng.integers(1, 4))):
            add(int(m), v, 500 + int(rng.integers(0, 700)))
    for j in range(n_anchors):
        add(u, v, 1000 + 20 * j)
        add(u, int(rng.choice(mids)), 1000 + 20 * j + 5)  # scatter side of u
    for _ in range(n_noise):
        a, b = rng.integers(0, nv, 2)
        if a != b:
            add(int(a), int(b), int(rng.integers(0, 1400)))
    order = np.argsort(np.array(ts), kind="stable")
    src = np.array(src, np.uint32)[order]
    dst = np.array(dst, np.uint32)[order]
    ts = W.T0 + np.array(ts, np.int64)[order]
    return W.EdgeList(src, dst, ts, np.zeros(len(src), np.float32), nv)


@pytest.mark.parametrize("seed,k", [(1, 2), (2, 3), (3, 2)])
def test_split_heavy_sender_windows(seed, k):
    """The learned schedule cuts anchors with much predicted work into slices
    whose partial counts are added together (a tiny split size forces it on
    this small graph); every column must equal the oracle's, as must the
    static schedule's unsplit result."""
    g = _heavy_sender_graph(seed)
    ref = oracle_mine(g, 2000, 5, k)
    assert ref[2].max() > 0 and ref[3].max() > 0  # columns FAN_OUT, FAN_IN, SG, GS, cycles
    assert_same(gpu_mine(g, 2000, 5, k), ref, f"heavy senders seed {seed} k {k} static")
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    A.amlm_costmodel_train([G], [A.params(A.AMLM_ALL, 2000, 5, k)], epochs=2, batch=256, seed=seed)
    for split in (64, 1024, 0):
        A.amlm_tune_set(G, split_bytes=split)
        c = A.amlm_mine(G, A.params(A.AMLM_ALL, 2000, 5, k, A.AMLM_SCHED_LEARNED))
        A.amlm_graph_sync(G)
        assert_same(A.to_u32(c), ref, f"heavy senders seed {seed} k {k} learned, split {split}")
    G.close()


UNORD = A.AMLM_ALL | A.AMLM_SG_UNORDERED
UNORD_O = oracle.ALL | oracle.SG_UNORDERED


@pytest.mark.parametrize("seed", range(8))
def test_unordered_sg_random_small(seed):
    """The unordered scatter-gather modifier: only the verification's timing
    test changes, so every column must still equal the oracle's."""
    rng = np.random.default_rng(800 + seed)
    g = W.random_small(40 + seed, n_edges=int(rng.integers(30, 400)), n_vertices=int(rng.integers(3, 20)),
                       t_range=int(rng.integers(5, 80)))
    for (delta, L, k) in [(int(rng.integers(0, 60)), int(rng.integers(2, 7)), int(rng.integers(1, 5))),
                          (30, 4, 2), (1000, 3, 3)]:
        assert_same(gpu_mine(g, delta, L, k, patterns=UNORD), oracle_mine(g, delta, L, k, patterns=UNORD_O),
                    f"unordered seed {seed} d{delta} L{L} k{k}")


def test_unordered_sg_mid_and_subset():
    g = W.mid(205, scale=0.01)
    ref = oracle_mine(g, 86400, 4, 2, patterns=UNORD_O)
    ordered = oracle_mine(g, 86400, 4, 2)
    assert (ref[2] > ordered[2]).any()  # the variant changes counts on this graph
    assert_same(gpu_mine(g, 86400, 4, 2, patterns=UNORD), ref, "unordered mid")
    assert_same(gpu_mine(g, 86400, 4, 2, patterns=A.AMLM_SG | A.AMLM_SG_UNORDERED), ref[[2]], "unordered SG only")
    with pytest.raises(A.AmlmError) as ei:  # the modifier without SG
        G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
        try:
            A.amlm_mine(G, A.params(A.AMLM_GS | A.AMLM_SG_UNORDERED, 86400, 4, 2),
                        counts=torch.zeros((1, g.n_edges), dtype=torch.int32, device="cuda"))
        finally:
            G.close()
    assert ei.value.status == 1


def test_unordered_sg_learned_slices():
    """Sliced heavy anchors under the modifier: partial counts added by the
    slices equal the oracle's."""
    g = _heavy_sender_graph(41)
    ref = oracle_mine(g, 2000, 5, 3, patterns=UNORD_O)
    assert ref[2].max() > 0
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    A.amlm_costmodel_train([G], [A.params(A.AMLM_ALL, 2000, 5, 3)], epochs=2, batch=256, seed=41)
    for split in (64, 0):
        A.amlm_tune_set(G, split_bytes=split)
        c = A.amlm_mine(G, A.params(UNORD, 2000, 5, 3, A.AMLM_SCHED_LEARNED))
        A.amlm_graph_sync(G)
        assert_same(A.to_u32(c), ref, f"unordered learned, split {split}")
    G.close()


def test_deterministic_repeat():
    g = W.mid(204, scale=0.01)
    a = gpu_mine(g, 86400, 6, 2)
    b = gpu_mine(g, 86400, 6, 2)
    np.testing.assert_array_equal(a, b)


@pytest.fixture(scope="module")
def mid_full():
    return W.mid(202)


def _sampled(g, counts, delta, L, k, n_sample=400, seed=0, patterns=oracle.ALL):
    rng = np.random.default_rng(seed)
    sel = rng.choice(g.n_edges, n_sample, replace=False)
    # add the heaviest anchors by fan-in / fan-out too
    sel = np.unique(np.concatenate([sel, np.argsort(counts[0])[-20:], np.argsort(counts[1])[-20:],
                                    np.argsort(counts[2])[-20:], np.nonzero(counts[4:].sum(axis=0))[0][:50]]))
    ref = oracle.mine_selected(g.src, g.dst, g.ts, g.n_vertices, sel, patterns, delta, L, k)
    assert_same(counts[:, sel], ref, "sampled")
    return sel


def test_mid_full_size_sampled(mid_full):
    g = mid_full
    c = gpu_mine(g, 86400, 6, 2)
    _sampled(g, c, 86400, 6, 2)
    # cycle identity over the whole graph: sum_e CYC_l(e) = l * C_l
    cf = oracle.count_cycles_first(g.src, g.dst, g.ts, g.n_vertices, 86400, 6)
    for l in range(2, 7):
        assert int(c[4 + l - 2].astype(np.uint64).sum()) == l * int(cf[l])


def test_unordered_sg_mid_full_size_sampled(mid_full):
    """The unordered modifier on the whole 5M-edge graph: sampled edges
    against the oracle; on every edge SG can only grow and the other columns
    equal the ordered mining's."""
    g = mid_full
    c = gpu_mine(g, 86400, 6, 2, patterns=UNORD)
    _sampled(g, c, 86400, 6, 2, patterns=UNORD_O, seed=5)
    o = gpu_mine(g, 86400, 6, 2)
    assert (c[2] >= o[2]).all() and (c[2] > o[2]).any()
    np.testing.assert_array_equal(np.delete(c, 2, axis=0), np.delete(o, 2, axis=0))


@pytest.fixture(scope="module")
def large_full():
    return W.large(404)


def test_large_full_size_sampled_learned_schedule(large_full):
    """The 32M-edge benchmark workload in the benchmark's launch
    configuration (learned schedule, cost model trained on graphs of the
    5M-edge generator): sampled edges against the oracle, and the learned
    counts equal the static ones on every edge."""
    g = large_full
    mids = [W.mid(202 + i, scale=0.05) for i in range(2)]
    Gs = [A.Graph(m.src, m.dst, m.ts, m.n_vertices) for m in mids]
    A.amlm_costmodel_train(Gs, [A.params(A.AMLM_ALL, 86400, 6, 2)] * 2, epochs=2, batch=4096, seed=1)
    for G in Gs:
        G.close()
    learned = gpu_mine(g, 86400, 6, 2, schedule=A.AMLM_SCHED_LEARNED, on_device=True)
    static = gpu_mine(g, 86400, 6, 2, schedule=A.AMLM_SCHED_STATIC, on_device=True)
    np.testing.assert_array_equal(learned, static)
    _sampled(g, learned, 86400, 6, 2, n_sample=300, seed=3)
    # the unordered scatter-gather modifier in the same configuration
    lu = gpu_mine(g, 86400, 6, 2, patterns=UNORD, schedule=A.AMLM_SCHED_LEARNED, on_device=True)
    assert (lu[2] >= learned[2]).all()
    np.testing.assert_array_equal(np.delete(lu, 2, axis=0), np.delete(learned, 2, axis=0))
    _sampled(g, lu, 86400, 6, 2, n_sample=150, seed=4, patterns=UNORD_O)

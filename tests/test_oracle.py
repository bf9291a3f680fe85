"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself: a literal
brute-force enumeration, closed forms for isolated motifs, the 6! = 720
ordering count of Section 4, and invariants that hold by construction.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_2604_12241_amd import workloads as W
from tests.brute import brute_counts, brute_part

HERE = os.path.dirname(os.path.abspath(__file__))
T0 = W.T0


def mine(src, dst, ts, nv, delta, L, k, patterns=oracle.ALL):
    return oracle.mine(np.asarray(src), np.asarray(dst), np.asarray(ts, dtype=np.int64), nv,
                       patterns, delta, L, k)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(24))
def test_oracle_matches_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    nv = int(rng.integers(4, 14))
    g = W.random_small(seed, n_edges=int(rng.integers(20, 140)), n_vertices=nv,
                       t_range=int(rng.integers(5, 60)))
    delta = int(rng.integers(0, 40))
    L = int(rng.integers(2, 6))
    k = int(rng.integers(1, 4))
    o = mine(g.src, g.dst, g.ts, g.n_vertices, delta, L, k)
    b = brute_counts(g.src, g.dst, g.ts, delta, L, k)
    np.testing.assert_array_equal(o.astype(np.uint64), b)


@pytest.mark.parametrize("seed", range(16))
def test_oracle_unordered_sg_matches_brute_force(seed):
    """The unordered scatter-gather modifier against the literal enumeration
    with the per-intermediate order dropped."""
    rng = np.random.default_rng(3000 + seed)
    nv = int(rng.integers(4, 12))
    g = W.random_small(700 + seed, n_edges=int(rng.integers(30, 140)), n_vertices=nv,
                       t_range=int(rng.integers(5, 50)))
    delta = int(rng.integers(0, 40))
    k = int(rng.integers(1, 4))
    o = mine(g.src, g.dst, g.ts, g.n_vertices, delta, 3, k, patterns=oracle.ALL | oracle.SG_UNORDERED)
    b = brute_counts(g.src, g.dst, g.ts, delta, 3, k, sg_unordered=True)
    np.testing.assert_array_equal(o.astype(np.uint64), b)


@pytest.mark.parametrize("seed", range(6))
def test_selected_matches_full(seed):
    """Through-edge cycle enumeration (any position) agrees with the
    last-edge-anchored search, and anchored columns agree row by row."""
    g = W.random_small(50 + seed, n_edges=150, n_vertices=9, t_range=25)
    for L in (2, 4, 6):
        o = mine(g.src, g.dst, g.ts, g.n_vertices, 12, L, 2)
        sel = np.arange(g.n_edges)
        s = oracle.mine_selected(g.src, g.dst, g.ts, g.n_vertices, sel, oracle.ALL, 12, L, 2)
        np.testing.assert_array_equal(s, o)


# ---------------------------------------------------------------- closed forms

def _motif_graph(edges, nslots, t_step=60, base=T0 + 5000):
    src = np.array([a for a, _, _ in edges], dtype=np.uint32)
    dst = np.array([b for _, b, _ in edges], dtype=np.uint32)
    ts = np.array([base + r * t_step for _, _, r in edges], dtype=np.int64)
    return src, dst, ts, nslots


def test_fan_out_closed_form():
    K = 7
    s, d, t, nv = _motif_graph(*W.motif_fan_out(K))
    o = mine(s, d, t, nv, 86400, 4, 2)
    np.testing.assert_array_equal(o[0], np.arange(1, K + 1))
    np.testing.assert_array_equal(o[1], np.ones(K))
    assert o[2:].sum() == 0


def test_fan_in_closed_form():
    K = 6
    s, d, t, nv = _motif_graph(*W.motif_fan_in(K))
    o = mine(s, d, t, nv, 86400, 4, 2)
    np.testing.assert_array_equal(o[1], np.arange(1, K + 1))
    np.testing.assert_array_equal(o[0], np.ones(K))
    assert o[2:].sum() == 0


@pytest.mark.parametrize("l", [2, 3, 4, 5, 6])
def test_cycle_closed_form(l):
    s, d, t, nv = _motif_graph(*W.motif_cycle(l))
    L = 6
    o = mine(s, d, t, nv, 86400, L, 1)
    cyc = o[4:]
    for ll in range(2, L + 1):
        np.testing.assert_array_equal(cyc[ll - 2], np.full(l, 1 if ll == l else 0))
    exp = np.array([0] + [1 if l >= 3 else 0] * (l - 1))
    np.testing.assert_array_equal(o[2], exp)   # SG_1
    np.testing.assert_array_equal(o[3], exp)   # GS_1
    # a window one step too short breaks the cycle (span = (l-1) steps)
    o2 = mine(s, d, t, nv, 60 * (l - 1) - 1, L, 1)
    assert o2[4:].sum() == 0


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_scatter_gather_closed_form(K):
    s, d, t, nv = _motif_graph(*W.motif_scatter_gather(K))
    for k in (1, 2, 3, 4):
        o = mine(s, d, t, nv, 86400, 4, k)
        sg = o[2]
        # scatters first (K edges), then gathers g_j, j = 1..K: SG_k(g_j) = [j >= k]
        np.testing.assert_array_equal(sg[:K], 0)
        np.testing.assert_array_equal(sg[K:], (np.arange(1, K + 1) >= k).astype(np.uint32))
        gs = o[3]
        np.testing.assert_array_equal(gs[K:], np.full(K, 1 if k == 1 else 0))


@pytest.mark.parametrize("K", [1, 3, 6])
def test_reversed_scatter_gather_closed_form(K):
    """Every intermediate's gather leg m_j -> v comes before its scatter leg
    s -> m_j, all inside one window: the ordered count sees only u as an
    intermediate, the unordered one sees u and all K of the m_j."""
    s_, u, v = 0, 1, 2
    edges = [(3 + j, v, j) for j in range(K)]            # gathers first
    edges += [(s_, 3 + j, K + j) for j in range(K)]      # then the scatters
    edges += [(s_, u, 2 * K), (u, v, 2 * K + 1)]         # sender leg, anchor
    src, dst, ts, nv = _motif_graph(edges, 3 + K)
    for k in range(1, K + 3):
        o = mine(src, dst, ts, nv, 86400, 4, k)
        ou = mine(src, dst, ts, nv, 86400, 4, k, patterns=oracle.ALL | oracle.SG_UNORDERED)
        assert o[2, -1] == (1 if k == 1 else 0)
        assert ou[2, -1] == (1 if k <= K + 1 else 0)
        # nothing else moves: the other anchors have no sender
        np.testing.assert_array_equal(np.delete(ou, 2, axis=0), np.delete(o, 2, axis=0))
        np.testing.assert_array_equal(ou[2, :-1], 0)
    # a window that ends before the first gather leg drops the m_j again
    o = mine(src, dst, ts, nv, 60 * (K + 1), 4, 2, patterns=oracle.ALL | oracle.SG_UNORDERED)
    assert o[2, -1] == 0


@pytest.mark.parametrize("k_in,k_out", [(2, 2), (3, 5), (6, 2), (8, 8)])
def test_gather_scatter_closed_form(k_in, k_out):
    s, d, t, nv = _motif_graph(*W.motif_gather_scatter(k_in, k_out))
    for k in (1, 2, 3, 6):
        o = mine(s, d, t, nv, 86400, 4, k)
        j = np.arange(1, k_out + 1)
        exp = k_in * (k_in >= k) * (j >= k)
        np.testing.assert_array_equal(o[3][k_in:], exp)
        np.testing.assert_array_equal(o[3][:k_in], 0)
        np.testing.assert_array_equal(o[2][k_in:], np.full(k_out, k_in if k == 1 else 0))


def test_tiny_workload_injected_motifs():
    """The tiny workload's motifs sit on fresh accounts, so their rows follow
    the closed forms even inside the random background."""
    g = W.tiny(101)
    o = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 4, 3)
    key = {(int(a), int(b), int(c)): i for i, (a, b, c) in enumerate(zip(g.src, g.dst, g.ts))}
    for m in g.meta["motifs"]:
        rows = [key[e] for e in m["edges"]]
        kind = m["kind"]
        if kind == "fan_out":
            assert list(o[0, rows]) == [1, 2, 3, 4, 5]
        elif kind == "fan_in":
            assert list(o[1, rows]) == [1, 2, 3, 4, 5]
        elif kind == "cycle":
            l = len(rows)
            assert list(o[4 + l - 2, rows]) == [1] * l
        elif kind == "scatter_gather":
            assert list(o[2, rows]) == [0, 0, 0, 0, 0, 1]   # k = 3


# ---------------------------------------------------------------- T-720

def _read_golden(name):
    out = {}
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = int(v)
    return out


def test_t720_scatter_gather_orderings():
    gold = _read_golden("t720.txt")
    edges = [(0, 1), (0, 2), (0, 3), (1, 4), (2, 4), (3, 4)]   # s=0, m=1..3, d=4
    hits, hits_u, hits_p, total = 0, 0, 0, 0
    for perm in itertools.permutations(range(6)):
        total += 1
        src = np.array([a for a, _ in edges], dtype=np.uint32)
        dst = np.array([b for _, b in edges], dtype=np.uint32)
        ts = T0 + np.array(perm, dtype=np.int64)
        latest_gather = 3 + int(np.argmax(ts[3:]))
        for pats in (oracle.SG, oracle.SG | oracle.SG_UNORDERED, oracle.SG | oracle.SG_PHASE):
            o = mine(src, dst, ts, 5, 100, 2, 3, pats)
            assert o[0].sum() == o[0, latest_gather]
            if pats == oracle.SG:
                hits += int(o[0, latest_gather])
            elif pats & oracle.SG_UNORDERED:
                hits_u += int(o[0, latest_gather])
            else:
                hits_p += int(o[0, latest_gather])
                # phase order: all three scatter legs before all three gathers
                assert int(o[0, latest_gather]) == int(max(perm[:3]) < min(perm[3:]))
    assert total == gold["orderings"]
    assert hits == gold["per_intermediate_instances"]
    assert hits_u == gold["unordered_instances"]
    assert hits_p == gold["phase_order_instances"]


@pytest.mark.parametrize("seed", range(16))
def test_variants_match_brute_force(seed):
    """Phase-ordered scatter-gather and the distinct-counterparty columns
    against the literal enumeration."""
    rng = np.random.default_rng(3000 + seed)
    nv = int(rng.integers(4, 12))
    g = W.random_small(seed + 500, n_edges=int(rng.integers(20, 90)), n_vertices=nv,
                       t_range=int(rng.integers(5, 40)))
    delta, L, k = int(rng.integers(0, 30)), int(rng.integers(2, 5)), int(rng.integers(1, 4))
    pats = oracle.ALL | oracle.SG_PHASE | oracle.DEG_OUT | oracle.DEG_IN
    o = mine(g.src, g.dst, g.ts, g.n_vertices, delta, L, k, pats)
    b = brute_counts(g.src, g.dst, g.ts, delta, L, k, sg_phase=True, deg=True)
    np.testing.assert_array_equal(o.astype(np.uint64), b)


@pytest.mark.parametrize("seed", range(12))
def test_any_order_cycles_match_edge_subsets(seed):
    """Any-order cycles against an enumeration of every edge subset that
    forms one directed cycle (a different procedure from the oracle's search
    from the latest edge)."""
    rng = np.random.default_rng(4000 + seed)
    g = W.random_small(seed + 700, n_edges=int(rng.integers(10, 26)), n_vertices=int(rng.integers(3, 7)),
                       t_range=int(rng.integers(3, 30)))
    delta, L = int(rng.integers(0, 25)), int(rng.integers(2, 5))
    o = mine(g.src, g.dst, g.ts, g.n_vertices, delta, L, 2, oracle.CYC | oracle.CYC_ANY_ORDER)
    b = brute_counts(g.src, g.dst, g.ts, delta, L, 2, cyc_any_order=True)
    np.testing.assert_array_equal(o.astype(np.uint64), b[4:4 + L - 1])


@pytest.mark.parametrize("l", [2, 3, 4, 5])
def test_cycle_orderings_closed_form(l):
    """One l-cycle on fresh vertices, over all l! orderings of its distinct
    edge times: exactly l of them are time-respecting (start at any edge,
    times rising around the cycle), and every one is an any-order cycle."""
    src = np.arange(l, dtype=np.uint32)
    dst = np.roll(src, -1)
    tr = ao = 0
    for perm in itertools.permutations(range(l)):
        ts = T0 + 10 * np.array(perm, dtype=np.int64)
        o = mine(src, dst, ts, l, 10 * l, max(l, 2), 2, oracle.CYC)
        a = mine(src, dst, ts, l, 10 * l, max(l, 2), 2, oracle.CYC | oracle.CYC_ANY_ORDER)
        col = l - 2
        assert set(o[col].tolist()) <= {0, 1} and len(set(o[col].tolist())) == 1
        assert a[col].tolist() == [1] * l
        assert o.sum() == o[col].sum() and a.sum() == a[col].sum()   # no other length
        tr += int(o[col, 0])
        ao += int(a[col, 0])
        # a time span wider than delta: no cycle either way
        a2 = mine(src, dst, ts, l, 10 * (l - 1) - 1, max(l, 2), 2, oracle.CYC | oracle.CYC_ANY_ORDER)
        assert a2.sum() == 0 or l == 1
    assert tr == l
    assert ao == math.factorial(l)


@pytest.mark.parametrize("K,R", [(5, 1), (6, 2), (6, 3), (8, 8)])
def test_distinct_counterparty_closed_form(K, R):
    """A fan-out of K edges to R destinations used round-robin, and the
    matching fan-in: DEG counts the destinations (sources) seen so far, FAN
    the edges."""
    src = np.array([0] * K + [10 + j % R for j in range(K)], dtype=np.uint32)
    dst = np.array([1 + j % R for j in range(K)] + [9] * K, dtype=np.uint32)
    ts = T0 + np.array(list(range(K)) + list(range(K)), dtype=np.int64) * 10
    o = mine(src, dst, ts, 10 + R, 1000, 4, 2, oracle.FAN_OUT | oracle.FAN_IN | oracle.DEG_OUT | oracle.DEG_IN)
    j = np.arange(K)
    np.testing.assert_array_equal(o[0, :K], j + 1)
    np.testing.assert_array_equal(o[2, :K], np.minimum(j + 1, R))
    np.testing.assert_array_equal(o[1, K:], j + 1)
    np.testing.assert_array_equal(o[3, K:], np.minimum(j + 1, R))


@pytest.mark.parametrize("seed", range(24))
def test_participation_matches_brute_force(seed):
    """SG_PART / GS_PART against the literal enumeration of every
    realisation of every instance (ordered and unordered legs); the other
    columns do not move."""
    rng = np.random.default_rng(5000 + seed)
    g = W.random_small(seed + 900, n_edges=int(rng.integers(20, 60)), n_vertices=int(rng.integers(3, 7)),
                       t_range=int(rng.integers(3, 20)))
    delta, k, un = int(rng.integers(3, 25)), int(rng.integers(1, 4)), bool(seed % 2)
    pats = oracle.ALL | oracle.PART | (oracle.SG_UNORDERED if un else 0)
    o = mine(g.src, g.dst, g.ts, g.n_vertices, delta, 3, k, pats)
    b = brute_part(g.src, g.dst, g.ts, delta, k, sg_unordered=un)
    np.testing.assert_array_equal(o[6:8].astype(np.uint64), b)
    np.testing.assert_array_equal(o[:6], mine(g.src, g.dst, g.ts, g.n_vertices, delta, 3, k, pats & ~oracle.PART))
    assert (o[6] >= o[2]).all() and (o[7] >= o[3]).all()   # an anchor is in its own instances
    # one column alone, in the last place
    only = mine(g.src, g.dst, g.ts, g.n_vertices, delta, 3, k, oracle.GS | oracle.PART)
    np.testing.assert_array_equal(only[1], o[7])


@pytest.mark.parametrize("seed", range(16))
def test_size_bins_match_brute_force(seed):
    """The four SG size bins against the literal enumeration (ordered and
    unordered legs); they sum to SG_k and leave every other column alone."""
    rng = np.random.default_rng(6000 + seed)
    nv = int(rng.integers(4, 12))
    g = W.random_small(seed + 950, n_edges=int(rng.integers(20, 120)), n_vertices=nv,
                       t_range=int(rng.integers(3, 40)))
    delta, k, un = int(rng.integers(3, 40)), int(rng.integers(1, 4)), bool(seed % 2)
    pats = oracle.ALL | oracle.SG_SIZES | (oracle.SG_UNORDERED if un else 0)
    o = mine(g.src, g.dst, g.ts, g.n_vertices, delta, 3, k, pats)
    b = brute_counts(g.src, g.dst, g.ts, delta, 3, k, sg_unordered=un, sizes=True)
    np.testing.assert_array_equal(o.astype(np.uint64), b)
    np.testing.assert_array_equal(o[-4:].sum(axis=0), o[2])
    np.testing.assert_array_equal(o[:-4], mine(g.src, g.dst, g.ts, g.n_vertices, delta, 3, k,
                                               pats & ~oracle.SG_SIZES))


@pytest.mark.parametrize("K", [1, 2, 4, 7])
def test_size_bins_closed_form(K):
    """The scatter-gather chain: the anchor at gather j has one sender whose
    intermediate set is {m_1..m_j}, so it lands in bin min(j - k, 3) when
    j >= k."""
    s, d, t, nv = _motif_graph(*W.motif_scatter_gather(K))
    for k in (1, 2, 3):
        o = mine(s, d, t, nv, 86400, 4, k, oracle.SG | oracle.SG_SIZES)
        j = np.arange(1, K + 1)
        for b in range(4):
            exp = ((j >= k) & (np.minimum(j - k, 3) == b)).astype(np.uint32)
            np.testing.assert_array_equal(o[1 + b, K:], exp)
            np.testing.assert_array_equal(o[1 + b, :K], 0)


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_participation_scatter_gather_closed_form(K):
    """Scatters s -> m_i (times 1..K), then gathers m_i -> v (K+1..2K): the
    instance anchored at gather j (j >= k) holds its sender leg (scatter j),
    and scatter i and gather i of every i < j, so scatter i and gather i
    both belong to the instances j >= max(i, k)."""
    s, d, t, nv = _motif_graph(*W.motif_scatter_gather(K))
    for k in (1, 2, 3, 4):
        o = mine(s, d, t, nv, 86400, 4, k, oracle.SG | oracle.GS | oracle.PART)
        i = np.arange(1, K + 1)
        exp = np.maximum(K - np.maximum(i, k) + 1, 0)
        np.testing.assert_array_equal(o[2, :K], exp)
        np.testing.assert_array_equal(o[2, K:], exp)
        # gather-scatter at k = 1: one sender, its leg and the anchor
        np.testing.assert_array_equal(o[3], np.full(2 * K, 1 if k == 1 else 0))


@pytest.mark.parametrize("k_in,k_out", [(2, 2), (3, 5), (6, 2), (8, 8)])
def test_participation_gather_scatter_closed_form(k_in, k_out):
    """Sources -> hub (times 1..k_in), hub -> sinks o_j: the anchor o_j
    (j >= k, k_in >= k) has k_in instances, each holding one source's leg
    and all of o_1..o_j."""
    s, d, t, nv = _motif_graph(*W.motif_gather_scatter(k_in, k_out))
    for k in (1, 2, 3, 6):
        o = mine(s, d, t, nv, 86400, 4, k, oracle.SG | oracle.GS | oracle.PART)
        j = np.arange(1, k_out + 1)
        on = k_in >= k
        np.testing.assert_array_equal(o[3, :k_in], np.full(k_in, max(k_out - k + 1, 0) * on))
        np.testing.assert_array_equal(o[3, k_in:], k_in * np.maximum(k_out - np.maximum(j, k) + 1, 0) * on)
        # scatter-gather at k = 1: each source is a sender of every o_j
        np.testing.assert_array_equal(o[2, :k_in], np.full(k_in, k_out if k == 1 else 0))
        np.testing.assert_array_equal(o[2, k_in:], np.full(k_out, k_in if k == 1 else 0))


# ---------------------------------------------------------------- invariants

@pytest.fixture(scope="module")
def mid_small():
    return W.mid(202, scale=0.004)   # 2k accounts, 20k edges


def test_i1_cycle_identity(mid_small):
    g = mid_small
    for L in (3, 5):
        o = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, L, 2)
        c = oracle.count_cycles_first(g.src, g.dst, g.ts, g.n_vertices, 86400, L)
        for l in range(2, L + 1):
            assert int(o[4 + l - 2].astype(np.uint64).sum()) == l * int(c[l])


def test_i2_fan_equals_slice_sizes(mid_small):
    g = mid_small
    D = 86400
    o = mine(g.src, g.dst, g.ts, g.n_vertices, D, 2, 2, oracle.FAN_OUT | oracle.FAN_IN)
    for col, key in ((0, g.src), (1, g.dst)):
        exp = np.zeros(g.n_edges, dtype=np.int64)
        for x in np.unique(key):
            idx = np.nonzero(key == x)[0]
            tt = np.sort(g.ts[idx])
            cnt = np.searchsorted(tt, g.ts[idx], "right") - np.searchsorted(tt, g.ts[idx] - D, "left")
            exp[idx] = cnt
        np.testing.assert_array_equal(o[col], exp)


def test_i3_k1_equals_distinct_senders(mid_small):
    g = mid_small
    D = 86400
    o = mine(g.src, g.dst, g.ts, g.n_vertices, D, 2, 1, oracle.SG | oracle.GS)
    exp = np.zeros(g.n_edges, dtype=np.int64)
    order = np.argsort(g.dst, kind="stable")
    for e in range(0, g.n_edges, 7):
        u, v, t = g.src[e], g.dst[e], g.ts[e]
        m = (g.dst == u) & (g.src != v) & (g.src != g.dst) & (g.ts >= t - D) & (g.ts < t)
        exp[e] = np.unique(g.src[m]).shape[0]
        assert o[0, e] == exp[e] and o[1, e] == exp[e]
    del order


def test_i4_monotone(mid_small):
    g = mid_small
    a = mine(g.src, g.dst, g.ts, g.n_vertices, 3600, 5, 2).astype(np.int64)
    b = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 5, 2).astype(np.int64)
    assert (b >= a).all()
    c = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 5, 3).astype(np.int64)
    assert (c[2:4] <= b[2:4]).all()
    d = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 3, 2)
    np.testing.assert_array_equal(d, b[:6])   # CYC_l does not depend on L >= l
    # dropping the per-intermediate order only adds intermediates: SG grows,
    # every other column stays
    u = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 5, 2,
             patterns=oracle.ALL | oracle.SG_UNORDERED).astype(np.int64)
    assert (u[2] >= b[2]).all() and (u[2] > b[2]).any()
    np.testing.assert_array_equal(np.delete(u, 2, axis=0), np.delete(b, 2, axis=0))


def test_i5_relabel_shift_permute(mid_small):
    g = mid_small
    o = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 4, 2)
    rng = np.random.default_rng(7)
    relabel = rng.permutation(g.n_vertices).astype(np.uint32)
    gp, perm = W.permute(g, 9)
    o2 = mine(relabel[gp.src], relabel[gp.dst], gp.ts + 12345, g.n_vertices, 86400, 4, 2)
    np.testing.assert_array_equal(o2, o[:, perm])


def test_i9_self_loops_change_nothing(mid_small):
    g = mid_small
    o = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 4, 2)
    rng = np.random.default_rng(3)
    m = 500
    ls = rng.integers(0, g.n_vertices, m).astype(np.uint32)
    lt = rng.choice(g.ts, m)
    o2 = mine(np.concatenate([g.src, ls]), np.concatenate([g.dst, ls]),
              np.concatenate([g.ts, lt]), g.n_vertices, 86400, 4, 2)
    np.testing.assert_array_equal(o2[:, :g.n_edges], o)
    assert o2[:, g.n_edges:].sum() == 0


def test_i10_zero_window(mid_small):
    g = mid_small
    o = mine(g.src, g.dst, g.ts, g.n_vertices, 0, 5, 1)
    assert o[2:].sum() == 0
    assert (o[0] >= 1).all() and (o[1] >= 1).all()


def test_i11_duplicate_every_edge():
    g = W.random_small(77, n_edges=90, n_vertices=8, t_range=30, self_loop_frac=0.0)
    L = 5
    o = mine(g.src, g.dst, g.ts, g.n_vertices, 20, L, 2).astype(np.int64)
    s2 = np.concatenate([g.src, g.src]); d2 = np.concatenate([g.dst, g.dst])
    t2 = np.concatenate([g.ts, g.ts])
    o2 = mine(s2, d2, t2, g.n_vertices, 20, L, 2).astype(np.int64)
    n = g.n_edges
    for half in (slice(0, n), slice(n, 2 * n)):
        np.testing.assert_array_equal(o2[0:2, half], 2 * o[0:2])
        np.testing.assert_array_equal(o2[2:4, half], o[2:4])
        for l in range(2, L + 1):
            np.testing.assert_array_equal(o2[4 + l - 2, half], o[4 + l - 2] * 2 ** (l - 1))
    assert o[4:].sum() > 0


def test_parameter_errors():
    s = np.array([0, 1], dtype=np.uint32); d = np.array([1, 0], dtype=np.uint32)
    t = np.array([T0, T0 + 1], dtype=np.int64)
    with pytest.raises(ValueError):
        mine(s, d, t, 1, 10, 4, 2)            # id out of range
    with pytest.raises(ValueError):
        mine(s, d, t, 2, -1, 4, 2)            # negative window
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 9, 2)            # L > 8
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 0)            # k = 0
    o = mine(s[:0], d[:0], t[:0], 2, 10, 4, 2)
    assert o.shape == (7, 0)
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.FAN_OUT | oracle.SG_UNORDERED)  # modifier without SG
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.ALL | 4096)                     # unknown bit
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.FAN_OUT | oracle.CYC | oracle.PART)  # no SG or GS
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.SG | oracle.SG_PHASE | oracle.PART)
    assert mine(s, d, t, 2, 10, 4, 2, patterns=oracle.ALL | oracle.PART).shape == (9, 2)
    assert mine(s, d, t, 2, 10, 4, 2, patterns=oracle.GS | oracle.PART).shape == (2, 2)
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.GS | oracle.SG_SIZES)           # sizes without SG
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.SG | oracle.SG_PHASE | oracle.SG_SIZES)
    assert mine(s, d, t, 2, 10, 4, 2, patterns=oracle.ALL | oracle.PART | oracle.SG_SIZES).shape == (13, 2)
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.FAN_OUT | oracle.SG_PHASE)      # modifier without SG
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.ALL | oracle.SG_PHASE | oracle.SG_UNORDERED)
    with pytest.raises(ValueError):
        mine(s, d, t, 2, 10, 4, 2, patterns=oracle.SG | oracle.CYC_ANY_ORDER)      # modifier without CYC
    assert mine(s, d, t, 2, 10, 4, 2, patterns=oracle.ALL | oracle.DEG_OUT | oracle.DEG_IN).shape == (9, 2)
    assert mine(s, d, t, 2, 10, 4, 2, patterns=oracle.ALL | oracle.SG_UNORDERED).shape == (7, 2)


def test_anchor_ranges_add_up(mid_small):
    """Disjoint anchor ranges sum to the full mining (anchored columns are
    disjoint, cycle credits add)."""
    g = mid_small
    full = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 5, 2).astype(np.uint64)
    acc = np.zeros_like(full)
    cuts = [0, 3000, 3001, 11000, g.n_edges]
    for a, b in zip(cuts[:-1], cuts[1:]):
        part, sec = oracle.mine_range(g.src, g.dst, g.ts, g.n_vertices, a, b, oracle.ALL, 86400, 5, 2)
        acc += part
        assert sec >= 0
    np.testing.assert_array_equal(acc, full)


@pytest.mark.parametrize("pats,ceiling", [(oracle.ALL, 0), (oracle.SG | oracle.CYC, 0), (oracle.ALL, 3),
                                          (oracle.ALL | oracle.DEG_IN | oracle.PART, 0),
                                          (oracle.SG | oracle.GS | oracle.PART, 2)])
def test_parallel_driver_equals_one_process(mid_small, pats, ceiling):
    """The multi-process driver (disjoint anchor ranges, cycle credits summed
    then saturated) gives the single-process result, uneven ranges included."""
    from oracle.parallel import mine_parallel
    g = mid_small
    full, _, _ = oracle.mine_ex(g.src, g.dst, g.ts, g.n_vertices, pats, 86400, 5, 2, ceiling=ceiling)
    got, info = mine_parallel(g.src, g.dst, g.ts, g.n_vertices, pats, 86400, 5, 2, procs=3, ceiling=ceiling)
    np.testing.assert_array_equal(got, full)
    assert sorted(info["ranges"])[0][0] == 0 and sorted(info["ranges"])[-1][1] == g.n_edges
    got, _ = mine_parallel(g.src, g.dst, g.ts, g.n_vertices, pats, 86400, 5, 2, procs=2, ceiling=ceiling,
                           ranges=[(0, 7), (7, 7), (7, 12000), (12000, g.n_edges)])
    np.testing.assert_array_equal(got, full)


def test_range_and_many_drivers(mid_small):
    """Per-range results (own rows + sparse cycle credits) add up to the
    full mining; independent graphs in a pool equal one-by-one mining."""
    from oracle.parallel import mine_many, mine_ranges
    g = mid_small
    full = mine(g.src, g.dst, g.ts, g.n_vertices, 86400, 5, 2).astype(np.uint64)
    ranges = [(0, 4000), (4000, 4001), (4001, 17000), (17000, g.n_edges)]
    acc = np.zeros_like(full)
    for (lo, hi), (own, cyc) in zip(ranges, mine_ranges(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, 86400, 5, 2,
                                                         ranges, procs=3)):
        acc[:4, lo:hi] = own[:4]
        np.testing.assert_array_equal(own[4:].astype(np.uint64) * 0, 0)
        for c, (idx, val) in enumerate(cyc):
            assert (idx < hi).all()          # a cycle's edges are no later than its last
            acc[4 + c, idx] += val
    np.testing.assert_array_equal(acc, full)
    gs = [W.random_small(s, n_edges=60, n_vertices=8, t_range=30) for s in range(5)]
    ps = [(oracle.ALL, 10 + s, 2 + s % 4, 1 + s % 3) for s in range(5)]
    got = mine_many([(x.src, x.dst, x.ts, x.n_vertices) for x in gs], ps, procs=2)
    for x, (pat, d, L, k), c in zip(gs, ps, got):
        np.testing.assert_array_equal(c, mine(x.src, x.dst, x.ts, x.n_vertices, d, L, k, pat))


# ---------------------------------------------------------------- algorithmic bytes

from tests.brute import brute_work  # noqa: E402


@pytest.mark.parametrize("seed", range(20))
def test_work_counters_match_brute_force(seed):
    """The oracle's per-anchor algorithmic bytes against a literal Python
    restatement of the canonical procedure, for several pattern subsets."""
    rng = np.random.default_rng(4000 + seed)
    g = W.random_small(900 + seed, n_edges=int(rng.integers(20, 120)), n_vertices=int(rng.integers(3, 12)),
                       t_range=int(rng.integers(5, 50)))
    delta, L, k = int(rng.integers(0, 40)), int(rng.integers(2, 7)), int(rng.integers(1, 4))
    cases = [(oracle.ALL, (True, True, True)), (oracle.SG | oracle.FAN_OUT, (True, False, False)),
             (oracle.GS | oracle.CYC, (False, True, True)), (oracle.ALL | oracle.SG_UNORDERED, (True, True, True))]
    for pats, (s_, g_, c_) in cases:
        c, w, _ = oracle.mine_ex(g.src, g.dst, g.ts, g.n_vertices, pats, delta, L, k, work=True)
        b = brute_work(g.src, g.dst, g.ts, delta, L, k, s_, g_, c_, ncols=c.shape[0],
                       sg_unordered=bool(pats & oracle.SG_UNORDERED))
        np.testing.assert_array_equal(w, b)


def test_work_counters_closed_forms():
    """Hand-computed bytes on isolated motifs (times T0 + 60 j, one window)."""
    L = 6
    io = 12 + 4 * (4 + L - 1)
    # fan-out: no sender into u, v has no out-edge: only the row's own bytes
    s, d, t, nv = _motif_graph(*W.motif_fan_out(5))
    _, w, _ = oracle.mine_ex(s, d, t, nv, oracle.ALL, 86400, L, 2, work=True)
    np.testing.assert_array_equal(w[0], io)
    assert w[1:].sum() == 0
    # scatter-gather with K intermediates, anchor = gather leg g_j: one sender
    # edge (8) and one sender s whose scan stops at the (k-1)-th qualifying m_i
    # (i < j) or, with fewer, covers the gather window of j entries
    K = 6
    s, d, t, nv = _motif_graph(*W.motif_scatter_gather(K))
    for k in (2, 3, 4):
        _, w, _ = oracle.mine_ex(s, d, t, nv, oracle.SG, 86400, L, k, work=True)
        j = np.arange(1, K + 1)
        np.testing.assert_array_equal(w[1, K:], 8 + 8 * np.minimum(j, k - 1))
        np.testing.assert_array_equal(w[1, :K], 0)
    # with GS and k = 1: no join, and the scatter scan stops at u's first
    # destination after tau (the gather leg itself)
    _, w, _ = oracle.mine_ex(s, d, t, nv, oracle.GS, 86400, L, 1, work=True)
    np.testing.assert_array_equal(w[1, K:], 16)
    # l-cycle anchored on its last edge: one element per depth, scanned at
    # depths 0 .. L-3, a closing search at depth L-2 (u has 1 + x in-edges:
    # 8 ceil(log2(1 + x)) bytes), and 8 l for the cycle
    for l in (2, 3, 4, 5, 6):
        edges, nvl = W.motif_cycle(l)
        for extra in (0, 3):
            # extra in-edges of u = l - 1 from fresh accounts, long before the window
            ee = [(nvl + q, l - 1, -100000 - q) for q in range(extra)] + edges
            s, d, t, nv = _motif_graph(ee, nvl + extra)
            _, w, _ = oracle.mine_ex(s, d, t, nv, oracle.CYC, 86400, L, 2, work=True)
            last = len(ee) - 1
            if l <= L - 1:
                want = 12 * (l - 1) + 8 * l
            else:
                want = 12 * (L - 2) + 8 * int(np.ceil(np.log2(1 + extra))) + 8 * L
            assert int(w[2, last]) == want, (l, extra)
            assert w[2, :last].sum() == 0


@pytest.mark.parametrize("l,m", [(3, 4), (4, 3), (5, 2)])
def test_saturation_ceiling_closed_form(l, m):
    """An l-cycle whose edges are each repeated m times (copies share their
    time): every copy lies on m^(l-1) cycles and sees m out-edges of its
    source.  Counts saturate at the ceiling."""
    edges, nv = W.motif_cycle(l)
    rep = [e for e in edges for _ in range(m)]
    s, d, t, nv = _motif_graph(rep, nv)
    full, _, _ = oracle.mine_ex(s, d, t, nv, oracle.FAN_OUT | oracle.CYC, 86400, l, 1)
    np.testing.assert_array_equal(full[0], m)
    np.testing.assert_array_equal(full[1 + l - 2], m ** (l - 1))
    for ceiling in (1, m, m ** (l - 1) - 1, m ** (l - 1), 2 ** 32 - 1):
        c, _, _ = oracle.mine_ex(s, d, t, nv, oracle.FAN_OUT | oracle.CYC, 86400, l, 1, ceiling=ceiling)
        np.testing.assert_array_equal(c[0], min(m, ceiling))
        np.testing.assert_array_equal(c[1 + l - 2], min(m ** (l - 1), ceiling))


def test_saturation_is_elementwise_min(mid_small):
    g = mid_small
    full, _, _ = oracle.mine_ex(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, 86400, 5, 2)
    for ceiling in (1, 3, 17):
        c, _, _ = oracle.mine_ex(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, 86400, 5, 2, ceiling=ceiling)
        np.testing.assert_array_equal(c, np.minimum(full, ceiling))

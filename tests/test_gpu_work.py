"""GPU checks of the per-anchor byte counters, the saturation ceiling and
the sticky device-error status.

The library's algorithmic-byte rows (B_io, B_sg/gs, B_cyc) follow the same
canonical procedure as the oracle's counters (which are pinned on the CPU by
a literal brute force and closed forms), so they must agree exactly; they
are the roofline's byte counts.  Counts under a lowered ceiling must equal
the oracle's saturated counts, whichever schedule runs.
"""
import numpy as np
import pytest

import oracle
import paper_2604_12241_amd as A
from paper_2604_12241_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PATS = [(A.AMLM_ALL, oracle.ALL), (A.AMLM_SG | A.AMLM_FAN_OUT, oracle.SG | oracle.FAN_OUT),
        (A.AMLM_GS | A.AMLM_CYCLES, oracle.GS | oracle.CYC),
        (A.AMLM_ALL | A.AMLM_SG_UNORDERED, oracle.ALL | oracle.SG_UNORDERED)]


def _gpu_work(g, pat, delta, L, k, schedule=A.AMLM_SCHED_STATIC):
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    c, w = A.amlm_mine_work(G, A.params(pat, delta, L, k, schedule))
    A.amlm_graph_sync(G)
    out = A.to_u32(c), w.cpu().numpy().view(np.uint64)
    G.close()
    return out


@pytest.mark.parametrize("seed", range(8))
def test_work_rows_equal_oracle_random_small(seed):
    rng = np.random.default_rng(6000 + seed)
    g = W.random_small(seed + 60, n_edges=int(rng.integers(30, 400)), n_vertices=int(rng.integers(3, 20)),
                       t_range=int(rng.integers(5, 80)))
    delta, L, k = int(rng.integers(0, 60)), int(rng.integers(2, 9)), int(rng.integers(1, 5))
    for pat, opat in PATS:
        c, w = _gpu_work(g, pat, delta, L, k)
        rc, rw, _ = oracle.mine_ex(g.src, g.dst, g.ts, g.n_vertices, opat, delta, L, k, work=True)
        np.testing.assert_array_equal(c, rc)
        np.testing.assert_array_equal(w[:3], rw, err_msg=f"pattern {pat} d{delta} L{L} k{k}")


@pytest.mark.parametrize("scale,L,k", [(0.01, 6, 2), (0.01, 4, 3), (0.005, 8, 1)])
def test_work_rows_equal_oracle_mid(scale, L, k):
    g = W.mid(202, scale=scale)
    c, w = _gpu_work(g, A.AMLM_ALL, 86400, L, k)
    rc, rw, _ = oracle.mine_ex(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, 86400, L, k, work=True)
    np.testing.assert_array_equal(c, rc)
    np.testing.assert_array_equal(w[:3], rw)
    assert w[1].sum() > 0 and w[2].sum() > 0


def test_work_rows_do_not_depend_on_schedule():
    g = W.mid(206, scale=0.01)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    A.amlm_costmodel_train([G], [A.params(A.AMLM_ALL, 86400, 6, 2)], epochs=1, batch=512, seed=3)
    A.amlm_tune_set(G, split_bytes=256)   # force slices
    _, ws = A.amlm_mine_work(G, A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_STATIC))
    _, wl = A.amlm_mine_work(G, A.params(A.AMLM_ALL, 86400, 6, 2, A.AMLM_SCHED_LEARNED))
    A.amlm_graph_sync(G)
    np.testing.assert_array_equal(ws[:3].cpu().numpy(), wl[:3].cpu().numpy())
    G.close()


def _heavy_multi_cycles(m=6):
    """A 4-, a 3- and a 5-cycle whose edges are each repeated m times, plus
    background edges: cycle credits reach m^(l-1) per edge (6^4 = 1296 on
    the 5-cycle, above every ceiling tried)."""
    rng = np.random.default_rng(5)
    src, dst, ts = [], [], []
    for base, l in ((0, 4), (10, 3), (20, 5)):
        for j in range(l):
            for _ in range(m):
                src.append(base + j); dst.append(base + (j + 1) % l); ts.append(100 + 10 * j)
    for _ in range(300):
        a, b = rng.integers(0, 30, 2)
        src.append(int(a)); dst.append(int(b)); ts.append(int(rng.integers(0, 200)))
    order = np.argsort(ts, kind="stable")
    return W.EdgeList(np.array(src, np.uint32)[order], np.array(dst, np.uint32)[order],
                      W.T0 + np.array(ts, np.int64)[order], np.zeros(len(src), np.float32), 30)


@pytest.mark.parametrize("ceiling", [1, 2, 5, 26, 1000])
def test_ceiling_saturates_like_the_oracle(ceiling):
    reached = False
    for g, (delta, L, k) in ((_heavy_multi_cycles(), (300, 6, 2)), (W.mid(207, scale=0.004), (86400, 5, 2))):
        G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
        A.amlm_graph_set_ceiling(G, ceiling)
        c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL, delta, L, k)))
        A.amlm_graph_sync(G)
        rc, _, _ = oracle.mine_ex(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, delta, L, k, ceiling=ceiling)
        np.testing.assert_array_equal(c, rc)
        full = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, delta, L, k)
        reached |= bool((full > ceiling).any())
        A.amlm_graph_set_ceiling(G, 0)  # back to 2^32 - 1
        c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL, delta, L, k)))
        A.amlm_graph_sync(G)
        np.testing.assert_array_equal(c, full)
        G.close()
    assert reached   # the ceiling is reached on at least one of the graphs


def test_ceiling_with_sliced_anchors():
    """Sliced heavy anchors add partial SG and sender counts; the ceiling
    applies to their sums."""
    from tests.test_gpu_parity import _heavy_sender_graph
    g = _heavy_sender_graph(7)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    A.amlm_costmodel_train([G], [A.params(A.AMLM_ALL, 2000, 5, 2)], epochs=2, batch=256, seed=7)
    A.amlm_tune_set(G, split_bytes=64)
    full = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, 2000, 5, 2)
    for ceiling in (3, 40):
        A.amlm_graph_set_ceiling(G, ceiling)
        c = A.to_u32(A.amlm_mine(G, A.params(A.AMLM_ALL, 2000, 5, 2, A.AMLM_SCHED_LEARNED)))
        A.amlm_graph_sync(G)
        np.testing.assert_array_equal(c, np.minimum(full, ceiling))
    G.close()


def test_sticky_device_error():
    g = W.random_small(3, n_edges=100, n_vertices=8, t_range=30)
    G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    H = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
    p = A.params(A.AMLM_ALL, 20, 4, 2)
    ref = A.to_u32(A.amlm_mine(G, p))
    assert A.amlm_graph_status(G) == 0
    A.amlm_graph_inject_device_error(G)
    for call in (lambda: A.amlm_mine(G, p), lambda: A.amlm_mine(G, p), lambda: A.amlm_graph_sync(G),
                 lambda: G.rebuild(g.src, g.dst, g.ts, g.n_vertices)):
        with pytest.raises(A.AmlmError) as ei:
            call()
        assert ei.value.status == 4
    assert A.amlm_graph_status(G) == 4
    assert G.info()["n_edges"] == g.n_edges    # info still answers
    # another handle is unaffected
    np.testing.assert_array_equal(A.to_u32(A.amlm_mine(H, p)), ref)
    A.amlm_graph_sync(H)
    G.close()
    H.close()

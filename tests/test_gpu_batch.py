"""Batched mining (one captured launch for many graphs) against standalone
mining and the oracle; hipGraph replays interleaved with eager work."""
import json
import os
import tempfile

import numpy as np
import pytest

import oracle
import paper_2604_12241_amd as A
from paper_2604_12241_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _subgraphs(n=10, seed0=900):
    out = []
    rng = np.random.default_rng(seed0)
    for i in range(n):
        e = int(rng.integers(200, 6000))
        v = max(20, e // 8)
        delta = int(rng.choice([6 * 3600, 86400, 3 * 86400]))
        g = W.power_law(seed0 + i, v, e, 4, 2.1, max(20.0, e / 50), delta_s=delta)
        L = int(rng.integers(2, 7))
        k = int(rng.integers(1, 4))
        out.append((g, A.params(A.AMLM_ALL, delta, L, k)))
    # an empty graph and a graph of self-loops only, in the middle
    z = W.EdgeList(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.int64), np.zeros(0, np.float32), 3)
    loops = W.EdgeList(np.array([1, 1], np.uint32), np.array([1, 1], np.uint32),
                       np.array([W.T0, W.T0 + 5], np.int64), np.zeros(2, np.float32), 2)
    out.insert(3, (z, A.params(A.AMLM_ALL, 3600, 4, 2)))
    out.insert(6, (loops, A.params(A.AMLM_ALL, 3600, 3, 2)))
    return out


def test_batch_unordered_sg_over_replays():
    """The unordered scatter-gather modifier through the captured batch."""
    subs = _subgraphs(n=6, seed0=950)
    ps = [A.params(A.AMLM_ALL | A.AMLM_SG_UNORDERED, p.delta, p.max_cycle_len, p.k) for _, p in subs]
    B = A.Batch([(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs])
    refs = [oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL | oracle.SG_UNORDERED, p.delta,
                        p.max_cycle_len, p.k) for (g, _), p in zip(subs, ps)]
    for rep in range(2):
        outs = A.amlm_mine_batch(B, ps)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(A.to_u32(o), r, err_msg=f"unordered replay {rep} graph {i}")
    B.close()


def test_batch_equals_standalone_and_oracle_over_replays():
    subs = _subgraphs()
    B = A.Batch([(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs])
    ps = [p for _, p in subs]
    refs = [oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, p.delta, p.max_cycle_len, p.k)
            for g, p in subs]
    other = W.mid(777, scale=0.002)
    for rep in range(3):
        outs = A.amlm_mine_batch(B, ps)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(A.to_u32(o), r, err_msg=f"replay {rep} graph {i}")
        # eager work and synchronisation between replays
        G = A.Graph(other.src, other.dst, other.ts, other.n_vertices)
        A.amlm_mine(G, A.params(A.AMLM_ALL, 86400, 5, 2))
        torch.cuda.synchronize()
        G.close()
    n, captures = B.info_batch()
    assert n == len(subs) and captures == 1
    # standalone mining of each graph gives the same columns
    for (g, p), r in zip(subs, refs):
        if g.n_edges == 0:
            continue
        G = A.Graph(g.src, g.dst, g.ts, g.n_vertices)
        np.testing.assert_array_equal(A.to_u32(A.amlm_mine(G, p)), r)
        G.close()
    # new windows and thresholds without a new capture
    ps2 = [A.params(A.AMLM_ALL, p.delta // 2, p.max_cycle_len, max(1, p.k - 1)) for p in ps]
    ps2 = [A.params(A.AMLM_ALL, q.delta, ps[i].max_cycle_len, q.k) for i, q in enumerate(ps2)]
    outs = A.amlm_mine_batch(B, ps2)
    torch.cuda.synchronize()
    for (g, _), q, o in zip(subs, ps2, outs):
        r = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, q.delta, q.max_cycle_len, q.k)
        np.testing.assert_array_equal(A.to_u32(o), r)
    assert B.info_batch()[1] == 1
    B.close()


def test_batch_learned_schedule_with_slices_over_replays():
    """The learned schedule inside the captured launch: work units and
    anchor slices (forced by a tiny split size) are rebuilt on every replay
    from the device-side lists, and every replay equals the oracle."""
    subs = _subgraphs(n=8, seed0=950)
    B = A.Batch([(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs])
    train = [A.Graph(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs if g.n_edges > 1000][:2]
    A.amlm_costmodel_train(train, [A.params(A.AMLM_ALL, 86400, 5, 2)] * len(train), epochs=2, batch=256, seed=3)
    for G in train:
        G.close()
    A.amlm_tune_set(B, split_bytes=64)
    refs = [oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, p.delta, p.max_cycle_len, p.k)
            for g, p in subs]
    other = W.mid(778, scale=0.002)
    for rep in range(4):
        # the network (per-sub-graph window and L as inputs), then the length rule
        sched = A.AMLM_SCHED_LEARNED if rep < 3 else A.AMLM_SCHED_LENGTH
        ps = [A.params(A.AMLM_ALL, p.delta, p.max_cycle_len, p.k, sched) for _, p in subs]
        outs = A.amlm_mine_batch(B, ps)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            np.testing.assert_array_equal(A.to_u32(o), r, err_msg=f"learned replay {rep} graph {i}")
        G = A.Graph(other.src, other.dst, other.ts, other.n_vertices)
        A.amlm_mine(G, A.params(A.AMLM_ALL, 86400, 5, 2))
        torch.cuda.synchronize()
        G.close()
    assert B.info_batch()[1] == 2   # one capture per schedule
    B.close()


def test_batch_rejects_bad_input():
    with pytest.raises(A.AmlmError):
        A.Batch([(np.array([0, 5], np.uint32), np.array([1, 0], np.uint32),
                  np.array([W.T0, W.T0], np.int64), 3)])
    subs = _subgraphs(3)
    B = A.Batch([(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs])
    ps = [p for _, p in subs]
    bad = list(ps)
    bad[1] = A.params(A.AMLM_FAN_OUT, 100, 4, 2)
    with pytest.raises(A.AmlmError):
        A.amlm_mine_batch(B, bad)
    B.close()


def test_autotune_caches_its_choice():
    subs = _subgraphs(6, seed0=950)
    B = A.Batch([(g.src, g.dst, g.ts, g.n_vertices) for g, _ in subs])
    ps = [p for _, p in subs]
    outs = [torch.empty((A.amlm_num_columns(p), int(B.sizes[i])), dtype=torch.int32, device="cuda")
            for i, p in enumerate(ps)]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        c1 = A.amlm_autotune(B, ps, outs, path)
        assert os.path.exists(path)
        c2 = A.amlm_autotune(B, ps, outs, path)
        assert c1 == c2
        txt = open(path).read()
        json.loads(txt)
    res = A.amlm_mine_batch(B, ps)
    torch.cuda.synchronize()
    for (g, p), o in zip(subs, res):
        r = oracle.mine(g.src, g.dst, g.ts, g.n_vertices, oracle.ALL, p.delta, p.max_cycle_len, p.k)
        np.testing.assert_array_equal(A.to_u32(o), r)
    B.close()

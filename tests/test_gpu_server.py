"""Streaming server: incremental results add up to a full recompute (I6),
and every batch's result is the same alone and in the concurrent mix."""
import numpy as np
import pytest

import oracle
import paper_2604_12241_amd as A
from paper_2604_12241_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

D, L, K = 86400, 5, 2


def _setup():
    base = W.mid(321, scale=0.004)
    batches = W.stream_batches(base, seed=77, n_batches=14, b_min=50, b_max=2500, rate_per_s=0.02,
                               zipf_a=2.1, max_degree=50)
    return base, batches


def _run(server, batches, sequential):
    out = []
    if sequential:
        for b in batches:
            t = server.submit(b.src, b.dst, b.ts)
            out.append(server.wait(t))
    else:
        tickets = [server.submit(b.src, b.dst, b.ts) for b in batches]
        out = [server.wait(t) for t in tickets]
    return out


def test_incremental_equals_full_recompute_and_alone_equals_mix():
    base, batches = _setup()
    p = A.params(A.AMLM_ALL, D, L, K)
    R = A.Graph(base.src, base.dst, base.ts, base.n_vertices)
    r_counts = A.to_u32(A.amlm_mine(R, p)).astype(np.uint64)
    mix = _run(A.Server(R, p, max_slots=4), batches, sequential=False)
    alone = _run(A.Server(R, p, max_slots=1), batches, sequential=True)
    tight = _run(A.Server(R, p, hbm_budget=1, max_slots=3), batches, sequential=False)
    for (cm, dm, nm), (ca, da, na), (ct, dt, nt) in zip(mix, alone, tight):
        np.testing.assert_array_equal(cm, ca)
        np.testing.assert_array_equal(cm, ct)
        assert nm == na == nt
        for x, y, z in zip(dm, da, dt):
            np.testing.assert_array_equal(x, y)
            np.testing.assert_array_equal(x, z)
    # accumulate: resident counts, new rows, deltas to older edges
    src = np.concatenate([base.src] + [b.src for b in batches])
    dst = np.concatenate([base.dst] + [b.dst for b in batches])
    ts = np.concatenate([base.ts] + [b.ts for b in batches])
    acc = np.zeros((r_counts.shape[0], src.shape[0]), np.uint64)
    acc[:, :base.n_edges] = r_counts
    pos = base.n_edges
    n_delta = 0
    for (c, (de, dc, dv), nd), b in zip(mix, batches):
        acc[:, pos:pos + b.n_edges] += c
        np.add.at(acc, (dc.astype(np.int64), de.astype(np.int64)), dv)
        assert (de < pos).all()          # deltas only touch earlier edges
        assert (dc >= 4).all()           # and only cycle columns
        n_delta += nd
        pos += b.n_edges
    full = oracle.mine(src, dst, ts, base.n_vertices, oracle.ALL, D, L, K)
    np.testing.assert_array_equal(acc, full.astype(np.uint64))
    assert n_delta > 0
    R.close()


def test_incremental_unordered_sg_equals_full_recompute():
    """The unordered scatter-gather modifier through the server's window
    graphs: resident counts + new rows + deltas equal the oracle's mining of
    the union graph."""
    base, batches = _setup()
    pats = A.AMLM_ALL | A.AMLM_SG_UNORDERED
    p = A.params(pats, D, L, K)
    R = A.Graph(base.src, base.dst, base.ts, base.n_vertices)
    r_counts = A.to_u32(A.amlm_mine(R, p)).astype(np.uint64)
    mix = _run(A.Server(R, p, max_slots=4), batches, sequential=False)
    src = np.concatenate([base.src] + [b.src for b in batches])
    dst = np.concatenate([base.dst] + [b.dst for b in batches])
    ts = np.concatenate([base.ts] + [b.ts for b in batches])
    acc = np.zeros((r_counts.shape[0], src.shape[0]), np.uint64)
    acc[:, :base.n_edges] = r_counts
    pos = base.n_edges
    for (c, (de, dc, dv), _), b in zip(mix, batches):
        acc[:, pos:pos + b.n_edges] += c
        np.add.at(acc, (dc.astype(np.int64), de.astype(np.int64)), dv)
        pos += b.n_edges
    full = oracle.mine(src, dst, ts, base.n_vertices, oracle.ALL | oracle.SG_UNORDERED, D, L, K)
    np.testing.assert_array_equal(acc, full.astype(np.uint64))
    R.close()


def test_stream_errors():
    base, batches = _setup()
    p = A.params(A.AMLM_ALL, D, L, K)
    R = A.Graph(base.src, base.dst, base.ts, base.n_vertices)
    S = A.Server(R, p, max_slots=2)
    b = batches[0]
    t = S.submit(b.src, b.dst, b.ts)
    S.wait(t)
    with pytest.raises(A.AmlmError) as ei:        # not strictly later
        S.submit(b.src, b.dst, b.ts)
    assert ei.value.status == 5
    with pytest.raises(A.AmlmError) as ei:        # endpoint out of range
        S.submit(np.array([base.n_vertices], np.uint32), np.array([0], np.uint32),
                 np.array([b.ts.max() + 10], np.int64))
    assert ei.value.status == 1
    # still serving after the errors
    b2 = batches[1]
    t2 = S.submit(b2.src, b2.dst, b2.ts)
    c, _, _ = S.wait(t2)
    assert c.shape == (A.amlm_num_columns(p), b2.n_edges)
    a, bb, cc = S.times(t2)
    assert a <= bb <= cc
    S.close()
    R.close()


def _accumulate(base, batches, results, r_counts):
    src = np.concatenate([base.src] + [b.src for b in batches])
    dst = np.concatenate([base.dst] + [b.dst for b in batches])
    ts = np.concatenate([base.ts] + [b.ts for b in batches])
    acc = np.zeros((r_counts.shape[0], src.shape[0]), np.uint64)
    acc[:, :base.n_edges] = r_counts
    pos = base.n_edges
    for (c, (de, dc, dv), nd), b in zip(results, batches):
        assert nd == de.shape[0]
        acc[:, pos:pos + b.n_edges] += c
        np.add.at(acc, (dc.astype(np.int64), de.astype(np.int64)), dv)
        assert (de < pos).all()
        pos += b.n_edges
    return src, dst, ts, acc


def test_long_stream_window_store_stays_bounded():
    """A stream many windows long (delta = 1 h, ~80 000 s of stream time):
    the window store keeps only the last delta of edges (plus the batches of
    one group), and the incremental results still add up to the oracle's
    mining of the union graph.  Includes an empty batch and a batch with
    self-loops."""
    delta, L, k = 3600, 5, 2
    base = W.mid(323, scale=0.002)
    batches = W.stream_batches(base, seed=78, n_batches=60, b_min=50, b_max=800, rate_per_s=0.25,
                               zipf_a=2.1, max_degree=40)
    t1 = int(batches[-1].ts.max())
    extra = [W.EdgeList(np.zeros(0, np.uint32), np.zeros(0, np.uint32), np.zeros(0, np.int64),
                        np.zeros(0, np.float32), base.n_vertices),
             W.EdgeList(np.array([3, 5, 5, 7, 9], np.uint32), np.array([3, 5, 7, 9, 5], np.uint32),
                        np.array([t1 + 1, t1 + 2, t1 + 3, t1 + 4, t1 + 5], np.int64),
                        np.zeros(5, np.float32), base.n_vertices)]
    batches = batches + extra
    p = A.params(A.AMLM_ALL, delta, L, k)
    R = A.Graph(base.src, base.dst, base.ts, base.n_vertices)
    r_counts = A.to_u32(A.amlm_mine(R, p)).astype(np.uint64)
    S = A.Server(R, p, max_slots=3)
    res = []
    for i in range(0, len(batches), 6):          # groups of six in flight
        tk = [S.submit(b.src, b.dst, b.ts) for b in batches[i:i + 6]]
        res += [S.wait(t) for t in tk]
    st = S.stats()
    S.close()
    src, dst, ts, acc = _accumulate(base, batches, res, r_counts)
    full = oracle.mine(src, dst, ts, base.n_vertices, oracle.ALL, delta, L, k)
    np.testing.assert_array_equal(acc, full.astype(np.uint64))
    # bounded by the window (plus one group of batches), not by the stream
    n_stream = sum(b.n_edges for b in batches)
    per_window = int(np.max([np.sum((ts > t - delta) & (ts <= t)) for t in ts[::97]]))
    assert st["batches_done"] == len(batches)
    assert st["max_window_edges"] <= per_window + 6 * 800 + 64
    assert st["max_window_edges"] < n_stream // 3
    assert st["commits"] >= 1
    R.close()


def test_server_with_learned_schedule_equals_static():
    """The learned schedule in the server's slots (own scratch per slot)
    gives the static schedule's results."""
    base, batches = _setup()
    R = A.Graph(base.src, base.dst, base.ts, base.n_vertices)
    A.amlm_costmodel_train([R], [A.params(A.AMLM_ALL, D, L, K)], epochs=1, batch=256, seed=5)
    outs = []
    for sched in (A.AMLM_SCHED_STATIC, A.AMLM_SCHED_LEARNED):
        S = A.Server(R, A.params(A.AMLM_ALL, D, L, K, sched), max_slots=2)
        outs.append(_run(S, batches, sequential=False))
        S.close()
    for (c1, d1, n1), (c2, d2, n2) in zip(*outs):
        np.testing.assert_array_equal(c1, c2)
        assert n1 == n2
        for x, y in zip(d1, d2):
            np.testing.assert_array_equal(x, y)
    R.close()


def test_snapshot_resume_continues_the_stream():
    """A server snapshot after some batches, a server resumed from it, and
    the rest of the stream: the later batches' rows, deltas and edge ids are
    those of an uninterrupted server.  A truncated file is rejected."""
    import os
    import tempfile
    base, batches = _setup()
    p = A.params(A.AMLM_ALL, D, L, K)
    R = A.Graph(base.src, base.dst, base.ts, base.n_vertices)
    full = _run(A.Server(R, p, max_slots=2), batches, sequential=False)
    S = A.Server(R, p, max_slots=2)
    first = _run(S, batches[:6], sequential=False)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "snap.bin")
        S.snapshot(path)
        S.close()
        T = A.Server.resume(path, p, max_slots=3)
        rest = _run(T, batches[6:], sequential=False)
        T.close()
        with open(path, "rb") as f:
            head = f.read(64)
        bad = os.path.join(d, "bad.bin")
        with open(bad, "wb") as f:
            f.write(head)
        with pytest.raises(A.AmlmError) as ei:
            A.Server.resume(bad, p)
        assert ei.value.status == 1
    for (c1, d1, n1), (c2, d2, n2) in zip(full, first + rest):
        np.testing.assert_array_equal(c1, c2)
        assert n1 == n2
        for x, y in zip(d1, d2):
            np.testing.assert_array_equal(x, y)
    R.close()

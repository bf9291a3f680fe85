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

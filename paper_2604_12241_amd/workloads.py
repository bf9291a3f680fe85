"""Seeded synthetic transaction graphs.

The paper evaluates on the IBM AML transaction datasets (Table 1) and the
Trovares temporal graphs; neither is available here, so every workload is a
synthetic stand-in with the same shape: power-law account activity, a long
time span with many timestamp ties, and a small fraction of injected
laundering motifs (fan-in, fan-out, scatter-gather, gather-scatter, cycles,
Section 2 and Section 5).

This module only draws random numbers.  It holds none of the mining
arithmetic, so both the CPU oracle and the GPU path may use it as their common
input source.  Every generator is deterministic in its seed
(``numpy.random.Generator(PCG64(seed))``).

An edge list is a dict of numpy arrays ``src`` (u32), ``dst`` (u32),
``ts`` (i64, seconds), ``amount`` (f32) plus ``n_vertices``.  Edges are
returned in timestamp order (ties in generation order), as a transaction log
would be; ``permute`` gives a shuffled copy.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

T0 = 1_700_000_000
HOUR = 3600
DAY = 86400


@dataclass
class EdgeList:
    src: np.ndarray
    dst: np.ndarray
    ts: np.ndarray
    amount: np.ndarray
    n_vertices: int
    meta: dict = field(default_factory=dict)

    @property
    def n_edges(self) -> int:
        return int(self.src.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _truncated_zipf(rng, a: float, n: int, n_edges: int, max_expected_degree: float):
    """Zipf(a) activity weights, clipped so that the heaviest account's
    expected number of edges (n_edges * w_max / sum w) is about
    ``max_expected_degree``."""
    w = rng.zipf(a, n).astype(np.float64)
    lo, hi = 1.0, float(w.max())
    if n_edges * hi / w.sum() <= max_expected_degree:
        return w
    for _ in range(80):
        c = math.sqrt(lo * hi) if hi / lo > 1.0001 else 0.5 * (lo + hi)
        d = n_edges * c / np.minimum(w, c).sum()
        if d > max_expected_degree:
            hi = c
        else:
            lo = c
    return np.minimum(w, lo)


def _diurnal_times(rng, n: int, span_s: int) -> np.ndarray:
    """Integer seconds in [0, span_s) with density proportional to
    1 + 0.8 cos(2 pi (hour - 14) / 24) (busiest at 14:00)."""
    out = np.empty(n, dtype=np.int64)
    filled = 0
    while filled < n:
        m = int((n - filled) * 1.9) + 1024
        t = rng.integers(0, span_s, size=m, dtype=np.int64)
        hour = (t % DAY) / HOUR
        p = (1.0 + 0.8 * np.cos(2 * np.pi * (hour - 14.0) / 24.0)) / 1.8
        keep = t[rng.random(m) < p]
        take = min(keep.shape[0], n - filled)
        out[filled:filled + take] = keep[:take]
        filled += take
    return out


def _amounts(rng, n: int) -> np.ndarray:
    return rng.lognormal(6.0, 1.5, size=n).astype(np.float32)


def _resample_self_loops(rng, src, dst, draw_dst):
    bad = np.nonzero(src == dst)[0]
    while bad.shape[0]:
        dst[bad] = draw_dst(bad.shape[0])
        bad = bad[src[bad] == dst[bad]]
    return dst


def _finish(src, dst, ts, amount, n_vertices, meta) -> EdgeList:
    order = np.argsort(ts, kind="stable")
    return EdgeList(src[order].astype(np.uint32), dst[order].astype(np.uint32),
                    ts[order].astype(np.int64), amount[order].astype(np.float32),
                    int(n_vertices), meta)


def permute(g: EdgeList, seed: int) -> tuple[EdgeList, np.ndarray]:
    """Shuffled copy; returns (copy, perm) with copy.x[i] = g.x[perm[i]]."""
    perm = _rng(seed).permutation(g.n_edges)
    return EdgeList(g.src[perm].copy(), g.dst[perm].copy(), g.ts[perm].copy(),
                    g.amount[perm].copy(), g.n_vertices, dict(g.meta)), perm


# ---------------------------------------------------------------------------
# motif shapes (edge lists over local vertex slots, with relative times)
# ---------------------------------------------------------------------------

def motif_fan_out(K):
    return [(0, j + 1, j + 1) for j in range(K)], K + 1


def motif_fan_in(K):
    return [(j + 1, 0, j + 1) for j in range(K)], K + 1


def motif_cycle(l):
    return [(j, (j + 1) % l, j + 1) for j in range(l)], l


def motif_scatter_gather(K):
    """source 0 -> intermediates 1..K (times 1..K) -> sink K+1 (times K+1..2K)."""
    e = [(0, j + 1, j + 1) for j in range(K)]
    e += [(j + 1, K + 1, K + 1 + j) for j in range(K)]
    return e, K + 2


def motif_gather_scatter(k_in, k_out):
    """sources 1..k_in -> hub 0 (times 1..k_in), then hub 0 -> k_out sinks."""
    e = [(j + 1, 0, j + 1) for j in range(k_in)]
    e += [(0, k_in + 1 + j, k_in + 1 + j) for j in range(k_out)]
    return e, k_in + k_out + 1


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def tiny(seed: int = 101, n_accounts: int = 2000, n_edges: int = 20000,
         days: int = 10, n_each: int = 20, step_s: int = 60) -> EdgeList:
    """Small case: Zipf(2.1) senders, uniform receivers, uniform times over
    ``days``, plus ``n_each`` isolated motifs of each kind on fresh accounts
    (ids >= n_accounts) so that their counts are known in closed form."""
    rng = _rng(seed)
    w = rng.zipf(2.1, n_accounts).astype(np.float64)
    src = rng.choice(n_accounts, size=n_edges, p=w / w.sum()).astype(np.int64)
    dst = rng.integers(0, n_accounts, size=n_edges)
    dst = _resample_self_loops(rng, src, dst, lambda m: rng.integers(0, n_accounts, size=m))
    ts = T0 + rng.integers(0, days * DAY, size=n_edges, dtype=np.int64)
    amount = _amounts(rng, n_edges)

    nxt = n_accounts
    motifs = []
    ms, md, mt = [], [], []
    kinds = ([("fan_out", motif_fan_out(5))] * n_each + [("fan_in", motif_fan_in(5))] * n_each
             + [("cycle", motif_cycle(3 + (i % 2))) for i in range(n_each)]
             + [("scatter_gather", motif_scatter_gather(3))] * n_each)
    n_bg = n_edges
    for kind, (edges, nslots) in kinds:
        base_t = T0 + int(rng.integers(0, days * DAY - 86400))
        first = n_bg + len(ms)
        for (a, b, rt) in edges:
            ms.append(nxt + a)
            md.append(nxt + b)
            mt.append(base_t + rt * step_s)
        motifs.append({"kind": kind, "first_vertex": nxt, "n_vertices": nslots,
                       "edges": [(nxt + a, nxt + b, base_t + rt * step_s) for (a, b, rt) in edges]})
        nxt += nslots
    src = np.concatenate([src, np.array(ms, dtype=np.int64)])
    dst = np.concatenate([dst, np.array(md, dtype=np.int64)])
    ts = np.concatenate([ts, np.array(mt, dtype=np.int64)])
    amount = np.concatenate([amount, _amounts(rng, len(ms))])
    g = _finish(src, dst, ts, amount, nxt, {"workload": "tiny", "seed": seed, "motifs": motifs})
    return g


def power_law(seed: int, n_accounts: int, n_edges: int, days: int, zipf_a: float,
              max_degree: float, motif_frac: float = 0.001, delta_s: int = DAY,
              workload: str = "power_law") -> EdgeList:
    """Chung-Lu graph: independent truncated Zipf out- and in-activity
    weights, diurnal timestamps, and a fraction ``motif_frac`` of the edges
    coming from laundering motifs embedded on uniformly chosen background
    accounts (each motif spans at most 0.9 of the window)."""
    rng = _rng(seed)
    n_motif_target = int(round(n_edges * motif_frac))
    n_bg = n_edges - n_motif_target
    w_out = _truncated_zipf(rng, zipf_a, n_accounts, n_bg, max_degree)
    w_in = _truncated_zipf(rng, zipf_a, n_accounts, n_bg, max_degree)
    cdf_in = np.cumsum(w_in)
    cdf_in /= cdf_in[-1]
    cdf_out = np.cumsum(w_out)
    cdf_out /= cdf_out[-1]

    def draw(cdf, m):
        return np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), n_accounts - 1)

    src = draw(cdf_out, n_bg).astype(np.int64)
    dst = draw(cdf_in, n_bg).astype(np.int64)
    dst = _resample_self_loops(rng, src, dst, lambda m: draw(cdf_in, m))
    span = days * DAY
    ts = T0 + _diurnal_times(rng, n_bg, span)

    ms, md, mt = [], [], []
    kinds = ["fan_in", "fan_out", "scatter_gather", "gather_scatter", "cycle"]
    counts = {k: 0 for k in kinds}
    while len(ms) < n_motif_target:
        kind = kinds[int(rng.integers(0, len(kinds)))]
        if kind == "fan_in":
            edges, ns = motif_fan_in(int(rng.integers(4, 11)))
        elif kind == "fan_out":
            edges, ns = motif_fan_out(int(rng.integers(4, 11)))
        elif kind == "scatter_gather":
            edges, ns = motif_scatter_gather(int(rng.integers(2, 9)))
        elif kind == "gather_scatter":
            edges, ns = motif_gather_scatter(int(rng.integers(2, 9)), int(rng.integers(2, 9)))
        else:
            edges, ns = motif_cycle(int(rng.integers(2, 7)))
        slots = rng.choice(n_accounts, size=ns, replace=False)
        n_steps = max(r for (_, _, r) in edges)
        span_m = int(0.9 * delta_s)
        step = max(1, span_m // max(1, n_steps))
        start = int(rng.integers(0, span - span_m))
        for (a, b, r) in edges:
            ms.append(int(slots[a]))
            md.append(int(slots[b]))
            mt.append(T0 + start + r * step)
        counts[kind] += 1
    src = np.concatenate([src, np.array(ms, dtype=np.int64)])
    dst = np.concatenate([dst, np.array(md, dtype=np.int64)])
    ts = np.concatenate([ts, np.array(mt, dtype=np.int64)])
    amount = _amounts(rng, src.shape[0])
    return _finish(src, dst, ts, amount, n_accounts,
                   {"workload": workload, "seed": seed, "motif_counts": counts})


def mid(seed: int = 202, scale: float = 1.0) -> EdgeList:
    """500k accounts, 5M edges over 16 days, Zipf(2.1), max degree ~20k
    (shaped like HI-Small in Table 1).  ``scale`` shrinks accounts, edges and
    the degree cap together for test-sized versions."""
    return power_law(seed, max(50, int(500_000 * scale)), max(100, int(5_000_000 * scale)), 16,
                     2.1, max(20.0, 20_000 * scale), workload=f"mid(scale={scale})")


def large(seed: int = 404, scale: float = 1.0) -> EdgeList:
    """2M accounts, 32M edges over 30 days, Zipf(1.9), max degree ~1e5
    (shaped like LI/HI-Medium in Table 1)."""
    return power_law(seed, max(50, int(2_000_000 * scale)), max(100, int(32_000_000 * scale)), 30,
                     1.9, max(20.0, 100_000 * scale), workload=f"large(scale={scale})")


def batch_subgraphs(n: int = 256, seed0: int = 303, e_min: float = 1e3, e_max: float = 2e5):
    """Per-institution partitions: ``n`` independent graphs of log-uniform
    size, each with its own window in {6 h, 24 h, 72 h}."""
    out = []
    for i in range(n):
        rng = _rng(seed0 + i)
        e = int(round(math.exp(rng.uniform(math.log(e_min), math.log(e_max)))))
        v = max(50, e // 10)
        delta = int(rng.choice([6 * HOUR, DAY, 3 * DAY]))
        g = power_law(seed0 + i, v, e, 16, 2.1, max(20.0, 20_000 * e / 5e6), delta_s=delta,
                      workload=f"batch[{i}]")
        out.append((g, delta))
    return out


def stream_batches(base: EdgeList, seed: int = 505, n_batches: int = 100,
                   b_min: float = 1e3, b_max: float = 1e5, rate_per_s: float = 12.3,
                   zipf_a: float = 1.9, max_degree: float = 100_000):
    """Transaction batches that arrive after the end of ``base``: batch sizes
    log-uniform in [b_min, b_max]; timestamps uniform over the batch's slice
    of graph time, strictly after everything before it; senders and
    receivers drawn from power-law activity over the same accounts."""
    rng = _rng(seed)
    nv = base.n_vertices
    w_out = _truncated_zipf(rng, zipf_a, nv, base.n_edges, max_degree)
    w_in = _truncated_zipf(rng, zipf_a, nv, base.n_edges, max_degree)
    cdf_out = np.cumsum(w_out); cdf_out /= cdf_out[-1]
    cdf_in = np.cumsum(w_in); cdf_in /= cdf_in[-1]
    t_prev = int(base.ts.max())
    batches = []
    for _ in range(n_batches):
        nb = int(round(math.exp(rng.uniform(math.log(b_min), math.log(b_max)))))
        dur = max(1, int(math.ceil(nb / rate_per_s)))
        src = np.minimum(np.searchsorted(cdf_out, rng.random(nb), side="right"), nv - 1)
        dst = np.minimum(np.searchsorted(cdf_in, rng.random(nb), side="right"), nv - 1)
        dst = _resample_self_loops(
            rng, src, dst,
            lambda m: np.minimum(np.searchsorted(cdf_in, rng.random(m), side="right"), nv - 1))
        ts = np.sort(t_prev + 1 + rng.integers(0, dur, size=nb, dtype=np.int64))
        t_prev = int(ts.max())
        batches.append(EdgeList(src.astype(np.uint32), dst.astype(np.uint32), ts,
                                _amounts(rng, nb), nv, {"workload": "stream"}))
    return batches


def random_small(seed: int, n_edges: int = 120, n_vertices: int = 12, t_range: int = 40,
                 self_loop_frac: float = 0.05) -> EdgeList:
    """Tiny dense graph with a narrow time range so that equal timestamps,
    parallel edges and short cycles are all frequent (brute-force cases)."""
    rng = _rng(seed)
    src = rng.integers(0, n_vertices, size=n_edges)
    dst = rng.integers(0, n_vertices, size=n_edges)
    loops = rng.random(n_edges) < self_loop_frac
    dst = np.where(loops, src, dst)
    ts = T0 + rng.integers(0, t_range, size=n_edges, dtype=np.int64)
    return EdgeList(src.astype(np.uint32), dst.astype(np.uint32), ts.astype(np.int64),
                    _amounts(rng, n_edges), n_vertices, {"workload": "random_small", "seed": seed})

"""The oracle over disjoint anchor ranges in parallel processes (test
infrastructure only, like the rest of this package).

Each worker mines the anchors of one contiguous edge-id range with the plain
single-threaded oracle (``mine_ex`` with ``a_lo, a_hi``).  The anchored
columns (FAN_OUT, FAN_IN, SG, GS) of different ranges are disjoint; cycles are
enumerated once, from their last edge, so a cycle is found by exactly one
worker and its credits to every one of its edges add up across workers, and
so do the participation credits of the scatter-gather and gather-scatter
instances (each belongs to its anchor's range).  The merge therefore sums
every column after the first four in 64 bits (the distinct-counterparty
columns are nonzero only at a range's own anchors) and saturates once,
which gives the full mining exactly.

Workers are forked: the edge arrays are shared copy-on-write, and the caller
must not have initialised a GPU runtime in this process.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time

import numpy as np

from . import CYC, FAN_IN, FAN_OUT, GS, SG, mine_ex, num_columns

_ARGS = None   # set in the parent before forking; read by the workers


def _anchored_columns(patterns):
    return sum(1 for b in (FAN_OUT, FAN_IN, SG, GS) if patterns & b)


def _worker(rng):
    src, dst, ts, nv, patterns, delta, L, k, ceiling = _ARGS
    lo, hi = rng
    t0 = time.perf_counter()
    out, _, sec = mine_ex(src, dst, ts, nv, patterns, delta, L, k, a_lo=lo, a_hi=hi, ceiling=ceiling)
    na = _anchored_columns(patterns)
    anchored = np.ascontiguousarray(out[:na, lo:hi])
    cyc = []
    for c in range(na, out.shape[0]):
        idx = np.flatnonzero(out[c]).astype(np.uint32)
        cyc.append((idx, out[c, idx]))
    return lo, hi, anchored, cyc, sec, time.perf_counter() - t0


def default_procs():
    """Worker count: the host's cores, at most 16 (a GPU machine's CPU share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def mine_parallel(src, dst, ts, n_vertices, patterns, delta, L, k, procs=None, ranges=None, ceiling=0,
                  progress=None):
    """All columns of every edge by ``procs`` workers over disjoint anchor
    ranges (default: ``procs`` equal ranges of edge ids).  Returns (counts
    uint32 [ncols, n], info) where info holds the ranges, each worker's
    anchor-loop seconds (graph set-up excluded) and its wall seconds."""
    global _ARGS
    n = len(src)
    procs = procs or default_procs()
    if ranges is None:
        cuts = np.linspace(0, n, procs + 1).round().astype(np.int64)
        ranges = [(int(cuts[i]), int(cuts[i + 1])) for i in range(procs)]
    ncols = num_columns(patterns, L)
    na = _anchored_columns(patterns)
    cap = 0xFFFFFFFF if ceiling == 0 else int(ceiling)
    _ARGS = (np.ascontiguousarray(src, np.uint32), np.ascontiguousarray(dst, np.uint32),
             np.ascontiguousarray(ts, np.int64), int(n_vertices), int(patterns), int(delta), int(L), int(k),
             int(ceiling))
    counts = np.zeros((ncols, n), dtype=np.uint32)
    acc = np.zeros((ncols - na, n), dtype=np.uint64) if ncols > na else None
    info = {"procs": procs, "ranges": [], "loop_s": [], "wall_s": []}
    ctx = mp.get_context("fork")
    try:
        with ctx.Pool(min(procs, len(ranges))) as pool:
            for lo, hi, anchored, cyc, sec, wall in pool.imap_unordered(_worker, ranges):
                counts[:na, lo:hi] = anchored
                for c, (idx, val) in enumerate(cyc):
                    acc[c, idx] += val.astype(np.uint64)   # idx: distinct within one worker
                info["ranges"].append((lo, hi))
                info["loop_s"].append(sec)
                info["wall_s"].append(wall)
                if progress:
                    progress(lo, hi, sec)
    finally:
        _ARGS = None
    if acc is not None:
        counts[na:] = np.minimum(acc, np.uint64(cap)).astype(np.uint32)
    return counts, info


def _worker_full(rng):
    src, dst, ts, nv, patterns, delta, L, k, ceiling = _ARGS
    lo, hi = rng
    out, _, sec = mine_ex(src, dst, ts, nv, patterns, delta, L, k, a_lo=lo, a_hi=hi, ceiling=ceiling)
    na = _anchored_columns(patterns)
    cyc = []
    for c in range(na, out.shape[0]):
        idx = np.flatnonzero(out[c]).astype(np.uint32)
        cyc.append((idx, out[c, idx]))
    return lo, hi, np.ascontiguousarray(out[:, lo:hi]), cyc


def mine_ranges(src, dst, ts, n_vertices, patterns, delta, L, k, ranges, procs=None, ceiling=0):
    """Each anchor range mined on its own (one process per range, at most
    `procs` at a time): returns, per range in the given order, (counts of
    the range's own edges [ncols, hi - lo], and per cycle column the nonzero
    credits (edge ids, values) of the cycles whose last edge is in the
    range, to any edge).  This is what a stream batch adds when the graph
    holds everything up to it: anchors only look back in time."""
    global _ARGS
    procs = procs or default_procs()
    _ARGS = (np.ascontiguousarray(src, np.uint32), np.ascontiguousarray(dst, np.uint32),
             np.ascontiguousarray(ts, np.int64), int(n_vertices), int(patterns), int(delta), int(L), int(k),
             int(ceiling))
    res = {}
    try:
        with mp.get_context("fork").Pool(min(procs, max(1, len(ranges)))) as pool:
            for lo, hi, own, cyc in pool.imap_unordered(_worker_full, ranges):
                res[(lo, hi)] = (own, cyc)
    finally:
        _ARGS = None
    return [res[(int(a), int(b))] for a, b in ranges]


def _worker_one(i):
    graphs, params = _ARGS
    g, (patterns, delta, L, k) = graphs[i], params[i]
    return i, mine_ex(g[0], g[1], g[2], g[3], patterns, delta, L, k)[0]


def mine_many(graphs, params, procs=None):
    """Independent graphs (src, dst, ts, n_vertices) with their own
    (patterns, delta, L, k), mined by a pool of processes; returns the
    counts in the given order."""
    global _ARGS
    procs = procs or default_procs()
    _ARGS = (graphs, params)
    out = [None] * len(graphs)
    try:
        with mp.get_context("fork").Pool(min(procs, max(1, len(graphs)))) as pool:
            for i, c in pool.imap_unordered(_worker_one, range(len(graphs))):
                out[i] = c
    finally:
        _ARGS = None
    return out

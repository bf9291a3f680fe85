"""Literal brute-force enumeration of every pattern, for tiny graphs only.

Written straight from the definitions with Python loops over edges and edge
sequences; shares nothing with the C oracle or the HIP library.  Used to pin
the oracle on graphs of at most a few hundred edges.
"""
from __future__ import annotations

import numpy as np


def brute_counts(src, dst, ts, delta: int, L: int, k: int, sg_unordered: bool = False,
                 sg_phase: bool = False, cyc_any_order: bool = False, deg: bool = False,
                 sizes: bool = False) -> np.ndarray:
    """Columns FAN_OUT, FAN_IN, SG_k, GS_k, CYC_2..CYC_L (then DEG_OUT,
    DEG_IN when deg, then the four SG size bins when sizes: senders whose
    intermediate set has exactly k, k+1, k+2 and at least k+3 members);
    uint64 [4+L-1(+2)(+4), n].
    sg_unordered: an intermediate's gather leg may come before its scatter
    leg (both inside the window).  sg_phase: some split time tau has every
    chosen scatter leg (u's among them) in [t - delta, tau) and every gather
    leg in [tau, t].
    cyc_any_order: cycles are edge sets forming a directed cycle on distinct
    vertices whose times span at most delta, in any order."""
    src = [int(x) for x in src]
    dst = [int(x) for x in dst]
    ts = [int(x) for x in ts]
    n = len(src)
    E = [i for i in range(n) if src[i] != dst[i]]
    nbase = 4 + L - 1 + (2 if deg else 0)
    out = np.zeros((nbase + (4 if sizes else 0), n), dtype=np.uint64)
    for e in E:
        u, v, t = src[e], dst[e], ts[e]
        lo = t - delta
        out[0, e] = sum(1 for f in E if src[f] == u and lo <= ts[f] <= t)
        out[1, e] = sum(1 for f in E if dst[f] == v and lo <= ts[f] <= t)
        if deg:
            out[4 + L - 1, e] = len({dst[f] for f in E if src[f] == u and lo <= ts[f] <= t})
            out[4 + L, e] = len({src[f] for f in E if dst[f] == v and lo <= ts[f] <= t})
        S = {src[a] for a in E if dst[a] == u and src[a] != v and lo <= ts[a] < t}
        sg = 0
        for s in S:
            if sg_phase:
                # some split time tau: scatter legs in [lo, tau), gather legs
                # in [tau, t]; u is one of the intermediates (its gather leg is
                # the anchor e itself, the instance's latest edge)
                for tau in range(lo + 1, t + 1):
                    M = set()
                    for a in E:
                        if src[a] != s or not (lo <= ts[a] < tau):
                            continue
                        m = dst[a]
                        if any(src[b] == m and dst[b] == v and tau <= ts[b] <= t for b in E):
                            M.add(m)
                    if len(M) >= k and u in M:
                        sg += 1
                        break
                continue
            M = set()
            for a in E:
                if src[a] != s or not (lo <= ts[a] < t):
                    continue
                m = dst[a]
                for b in E:
                    after = lo <= ts[b] if sg_unordered else ts[a] < ts[b]
                    if src[b] == m and dst[b] == v and after and ts[b] <= t:
                        M.add(m)
                        break
            if len(M) >= k:
                sg += 1
                if sizes:
                    out[nbase + min(len(M) - k, 3), e] += 1
        out[2, e] = sg
        taus = [ts[a] for a in E if dst[a] == u and src[a] != v and lo <= ts[a] < t]
        if taus:
            tau = min(taus)
            D = {dst[b] for b in E if src[b] == u and tau < ts[b] <= t}
            if len(S) >= k and len(D) >= k:
                out[3, e] = len(S)
    # cycles: enumerate edge sequences c_1..c_l by chaining, check the definition
    out_by_src = {}
    for f in E:
        out_by_src.setdefault(src[f], []).append(f)

    def extend(seq):
        l = len(seq)
        first, last = seq[0], seq[-1]
        if l >= 2 and dst[last] == src[first]:
            verts = [src[c] for c in seq]
            if (len(set(verts)) == l and all(ts[seq[i]] < ts[seq[i + 1]] for i in range(l - 1))
                    and ts[last] - ts[first] <= delta):
                for c in seq:
                    out[4 + l - 2, c] += 1
        if l == L:
            return
        for f in out_by_src.get(dst[last], []):
            # only strictly later edges within delta of c_1 can continue a cycle
            if ts[f] > ts[last] and ts[f] - ts[first] <= delta:
                extend(seq + [f])

    if cyc_any_order:
        # every set of l edges that forms one directed cycle through l
        # distinct vertices, its times spanning at most delta
        import itertools
        for l in range(2, L + 1):
            for comb in itertools.combinations(E, l):
                outs = [src[c] for c in comb]
                ins = [dst[c] for c in comb]
                if len(set(outs)) != l or set(outs) != set(ins):
                    continue
                nxt = {src[c]: dst[c] for c in comb}
                x, steps = outs[0], 0
                while True:
                    x = nxt[x]
                    steps += 1
                    if x == outs[0]:
                        break
                if steps != l:
                    continue
                tt = [ts[c] for c in comb]
                if max(tt) - min(tt) <= delta:
                    for c in comb:
                        out[4 + l - 2, c] += 1
        return out
    for c1 in E:
        extend([c1])
    return out


def brute_part(src, dst, ts, delta: int, k: int, sg_unordered: bool = False):
    """Participation counts (SG_PART, GS_PART), uint64 [2, n], by literal
    enumeration of realisations.  A scatter-gather instance is (anchor e,
    sender s) with SG_k(e) counting s; a realisation picks a sender leg
    s -> u before t (u's gather leg being e) and, for a set of other
    intermediates with the set at least k - 1 large, one (scatter, gather)
    leg pair each that meets the order and window conditions.  Every edge of
    every realisation is credited once per instance.  A gather-scatter
    instance is (anchor e, sender s in S(e)) with GS_k(e) > 0: its edges are
    s's legs into u in [t - delta, t) and u's out-edges in (tau, t]."""
    import itertools
    src = [int(x) for x in src]
    dst = [int(x) for x in dst]
    ts = [int(x) for x in ts]
    n = len(src)
    E = [i for i in range(n) if src[i] != dst[i]]
    out = np.zeros((2, n), dtype=np.uint64)
    for e in E:
        u, v, t = src[e], dst[e], ts[e]
        lo = t - delta
        S = {src[a] for a in E if dst[a] == u and src[a] != v and lo <= ts[a] < t}
        for s in S:
            sender_legs = [a for a in E if src[a] == s and dst[a] == u and lo <= ts[a] < t]
            pairs = {}
            for a in E:
                if src[a] != s or dst[a] == u or not (lo <= ts[a] < t):
                    continue
                for b in E:
                    if src[b] != dst[a] or dst[b] != v or not (lo <= ts[b] <= t):
                        continue
                    if sg_unordered or ts[a] < ts[b]:
                        pairs.setdefault(dst[a], []).append((a, b))
            others = sorted(pairs)
            if 1 + len(others) < k:
                continue
            members = set()
            # every choice of (no pair | one pair) per other intermediate
            for pick in itertools.product(*[[None] + pairs[m] for m in others]):
                if sum(1 for x in pick if x is not None) < k - 1:
                    continue
                for x in pick:
                    if x is not None:
                        members.update(x)
            for a in sender_legs:
                members.add(a)
            members.add(e)
            for f in members:
                out[0, f] += 1
        taus = [ts[a] for a in E if dst[a] == u and src[a] != v and lo <= ts[a] < t]
        if taus:
            tau = min(taus)
            scat = [b for b in E if src[b] == u and tau < ts[b] <= t]
            if len(S) >= k and len({dst[b] for b in scat}) >= k:
                for s in S:
                    for a in E:
                        if src[a] == s and dst[a] == u and lo <= ts[a] < t:
                            out[1, a] += 1
                    for b in scat:
                        out[1, b] += 1
    return out


def brute_work(src, dst, ts, delta: int, L: int, k: int, want_sg=True, want_gs=True, want_cyc=True,
               ncols: int | None = None, sg_unordered: bool = False) -> np.ndarray:
    """Algorithmic bytes of each anchor under the canonical procedure of the
    method (uint64 [3, n]: B_io, B_sg/gs, B_cyc), restated literally with
    Python loops and sorted lists.  Rows and slices are ordered by (ts, edge
    id); an element is 8 bytes (12 in the cycle scan)."""
    src = [int(x) for x in src]
    dst = [int(x) for x in dst]
    ts = [int(x) for x in ts]
    n = len(src)
    if ncols is None:
        ncols = 4 + L - 1
    E = [i for i in range(n) if src[i] != dst[i]]
    out = np.zeros((3, n), dtype=np.uint64)
    out[0, :] = 12 + 4 * ncols

    def slice_of(pred):
        return sorted((f for f in E if pred(f)), key=lambda f: (ts[f], f))

    def ceil_log2(x):
        c = 0
        while (1 << c) < x:
            c += 1
        return c

    for e in E:
        u, v, t = src[e], dst[e], ts[e]
        lo = t - delta
        if want_sg or want_gs:
            w = 0
            sender = slice_of(lambda a: dst[a] == u and lo <= ts[a] < t)
            w += 8 * len(sender)
            S = {src[a] for a in sender if src[a] != v}
            r = len([b for b in E if dst[b] == v and lo <= ts[b] <= t])
            if want_sg:
                for s in S:
                    sl = slice_of(lambda a: src[a] == s and lo <= ts[a] < t)
                    if k < 2:
                        n_s = 0
                    else:
                        n_s = len(sl)
                        seen, found = set(), 0
                        for idx, a in enumerate(sl):
                            m = dst[a]
                            if m == u or m in seen:
                                continue
                            ok = any(src[b] == m and dst[b] == v and ts[b] <= t
                                     and (lo <= ts[b] if sg_unordered else ts[a] < ts[b]) for b in E)
                            if ok:
                                seen.add(m)
                                found += 1
                                if found == k - 1:
                                    n_s = idx + 1
                                    break
                    w += 8 * min(n_s, r)
            if want_gs and len(S) >= k:
                tau = min(ts[a] for a in sender if src[a] != v)
                sc = slice_of(lambda b: src[b] == u and tau < ts[b] <= t)
                scanned, seen = len(sc), set()
                for idx, b in enumerate(sc):
                    if dst[b] not in seen:
                        seen.add(dst[b])
                        if len(seen) == k:
                            scanned = idx + 1
                            break
                w += 8 * scanned
            out[1, e] = w
        if want_cyc:
            indeg_u = len([f for f in E if dst[f] == u])
            acc = [0]

            def visit(h, d, tlast, on_path):
                if d == 0:
                    sl = slice_of(lambda f: src[f] == h and lo <= ts[f] < t)
                else:
                    sl = slice_of(lambda f: src[f] == h and tlast < ts[f] < t)
                if d <= L - 3:
                    acc[0] += 12 * len(sl)
                elif sl:
                    acc[0] += 8 * ceil_log2(indeg_u)
                for f in sl:
                    x = dst[f]
                    if x == u:
                        acc[0] += 8 * (d + 2)
                    elif d + 1 <= L - 2 and x not in on_path:
                        visit(x, d + 1, ts[f], on_path | {x})

            visit(v, 0, None, {v})
            out[2, e] = acc[0]
    return out


def brute_program(src, dst, ts, cells, delta: int, k: int) -> np.ndarray:
    """Stage-cell programs evaluated literally (uint64 [n]): for each anchor
    e = (u -> v, t), vertices 0 = u, 1 = v, 2 + i = bound by cell i; a loop
    cell runs over the non-self-loop edges out of (into) its vertex inside
    its window [lo, hi], in (time, id) order, keeping with `distinct` only
    the earliest out-edge (latest in-edge) per neighbour, skipping
    neighbours equal to the `skip` vertices; a probe counts the edges from
    `node` to `peer` inside its window (0 or 1 with `distinct`).  Folds: sum
    of the inner values (1 per innermost binding), or the number of
    bindings whose inner value reaches the threshold (k for AT_LEAST_K).
    `cells` are dicts with the amlm_cell field names (skip as a tuple)."""
    src = [int(x) for x in src]
    dst = [int(x) for x in dst]
    ts = [int(x) for x in ts]
    n = len(src)
    E = sorted((i for i in range(n) if src[i] != dst[i]), key=lambda i: (ts[i], i))
    out = np.zeros(n, dtype=np.uint64)

    def run(i, var, times, t, lo_w):
        c = cells[i]
        lo = lo_w if c["tlo"] == 0 else times[c["tref"]] + 1
        hi = t if c["thi"] == 0 else t - 1
        if c["op"] == 2:
            a, b = var[c["node"]], var[c["peer"]]
            cnt = sum(1 for f in E if src[f] == a and dst[f] == b and lo <= ts[f] <= hi)
            return min(cnt, 1) if c["distinct"] else cnt
        x = var[c["node"]]
        if c["op"] == 0:
            edges = [(f, dst[f]) for f in E if src[f] == x and lo <= ts[f] <= hi]
        else:
            edges = [(f, src[f]) for f in E if dst[f] == x and lo <= ts[f] <= hi]
        if c["distinct"]:
            pick = {}
            for f, w in edges:   # (time, id) order
                if c["op"] == 0:
                    pick.setdefault(w, f)     # earliest out-edge per neighbour
                else:
                    pick[w] = f               # latest in-edge per neighbour
            edges = sorted(((f, w) for w, f in pick.items()), key=lambda z: (ts[z[0]], z[0]))
        acc = 0
        thr = k if c["agg"] == 2 else c.get("threshold", 0)
        for f, w in edges:
            if any(var[b] == w for b in c.get("skip", ()) if b < len(var)):
                continue
            val = 1 if i + 1 == len(cells) else run(i + 1, var + [w], times + [ts[f]], t, lo_w)
            acc += val if c["agg"] == 0 else (1 if val >= thr else 0)
        return acc

    for e in E:
        out[e] = run(0, [src[e], dst[e]], [], ts[e], ts[e] - delta)
    return out

"""Literal brute-force enumeration of every pattern, for tiny graphs only.

Written straight from the definitions with Python loops over edges and edge
sequences; shares nothing with the C oracle or the HIP library.  Used to pin
the oracle on graphs of at most a few hundred edges.
"""
from __future__ import annotations

import numpy as np


def brute_counts(src, dst, ts, delta: int, L: int, k: int, sg_unordered: bool = False) -> np.ndarray:
    """Columns FAN_OUT, FAN_IN, SG_k, GS_k, CYC_2..CYC_L; uint64 [4+L-1, n].
    sg_unordered: an intermediate's gather leg may come before its scatter
    leg (both inside the window)."""
    src = [int(x) for x in src]
    dst = [int(x) for x in dst]
    ts = [int(x) for x in ts]
    n = len(src)
    E = [i for i in range(n) if src[i] != dst[i]]
    out = np.zeros((4 + L - 1, n), dtype=np.uint64)
    for e in E:
        u, v, t = src[e], dst[e], ts[e]
        lo = t - delta
        out[0, e] = sum(1 for f in E if src[f] == u and lo <= ts[f] <= t)
        out[1, e] = sum(1 for f in E if dst[f] == v and lo <= ts[f] <= t)
        S = {src[a] for a in E if dst[a] == u and src[a] != v and lo <= ts[a] < t}
        sg = 0
        for s in S:
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

    for c1 in E:
        extend([c1])
    return out
